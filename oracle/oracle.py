"""ctypes binding of the FP64 C oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the library.  The oracle works
in SI units and FP64; float32 GPU states are widened before they are passed in.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "_liboracle.so")

ORC_OK, ORC_EINVAL, ORC_ERANGE, ORC_ECFL, ORC_EOVERFLOW = 0, 1, 2, 3, 4
W_UNIT = 2.0 ** -20


LIB_OMP = os.path.join(HERE, "_liboracle_omp.so")


def build(force: bool = False, threaded: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA target).
    threaded: the same source with -fopenmp (its particle and grid loops split
    over threads), used only to time the oracle on all host cores; the tests
    use the serial build."""
    out = LIB_OMP if threaded else LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "pic_oracle.h"))):
        tmp = f"{out}.tmp{os.getpid()}"  # parallel test workers may build at once
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", *(["-fopenmp"] if threaded else []), "-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("bc", C.c_int * 3),
                ("depth2d", C.c_double), ("quantized", C.c_int)]


class _Pot(C.Structure):
    _fields_ = [("D", C.c_double), ("r0", C.c_double), ("s_rep", C.c_double), ("c_att", C.c_double),
                ("g_clamp", C.c_double), ("n_floor", C.c_double), ("mass", C.c_double), ("kind", C.c_int),
                ("lattice", C.c_int), ("alpha", C.c_double)]


class _Diag(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("px", C.c_double), ("py", C.c_double),
                ("pz", C.c_double), ("wsum", C.c_double), ("bond", C.c_double), ("step", C.c_int64)]


_lib = None
_lib_omp = None


def lib_threaded(threads: int):
    """The OpenMP build of the oracle with `threads` threads."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = C.CDLL(build(threaded=True))
        _declare(_lib_omp)
    C.CDLL("libgomp.so.1").omp_set_num_threads(int(threads))
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


def _declare(_lib):
    P = C.POINTER
    d, i64, i32 = C.c_double, C.c_int64, C.c_int32
    _lib.orc_num_nodes.restype = i64
    _lib.orc_num_nodes.argtypes = [P(_Grid)]
    _lib.orc_num_cells.restype = i64
    _lib.orc_num_cells.argtypes = [P(_Grid)]
    _lib.orc_deposit.argtypes = [P(_Grid), i64, P(i32), P(d), P(i32), P(i64), P(d)]
    _lib.orc_density.argtypes = [P(_Grid), P(d), P(d)]
    _lib.orc_gradient.argtypes = [P(_Grid), P(d), P(d)]
    _lib.orc_gather.argtypes = [P(_Grid), P(d), P(d), i32, P(d), P(d), P(d)]
    _lib.orc_neighbour_distances.argtypes = [P(_Pot), d, d, P(d), P(d)]
    _lib.orc_local_force.argtypes = [P(_Pot), C.c_int, d, P(d), P(d)]
    _lib.orc_phi_prime.restype = d
    _lib.orc_phi_prime.argtypes = [P(_Pot), d]
    _lib.orc_phi.restype = d
    _lib.orc_phi.argtypes = [P(_Pot), d]
    _lib.orc_energy_density.restype = d
    _lib.orc_energy_density.argtypes = [P(_Pot), d]
    _lib.orc_hcp_direction.restype = None
    _lib.orc_hcp_direction.argtypes = [C.c_int, P(d)]
    _lib.orc_energy_density_quad.restype = d
    _lib.orc_energy_density_quad.argtypes = [P(_Pot), d]
    _lib.orc_forces.argtypes = [P(_Grid), P(_Pot), P(d), i64, P(i32), P(d), P(d)]
    _lib.orc_push_one.argtypes = [P(_Grid), P(_Pot), d, P(d), P(i32), P(d), P(d)]
    _lib.orc_kick.argtypes = [P(_Grid), P(_Pot), d, d, i64, P(d), P(d)]
    _lib.orc_run.argtypes = [P(_Grid), P(_Pot), d, i64, P(i32), P(d), P(d), P(i32), C.c_int,
                             C.c_int, P(_Diag)]
    _lib.orc_calibrate_catt.argtypes = [P(_Grid), P(_Pot), d, C.c_int, C.c_int, P(d), P(d), P(d)]
    _lib.orc_functional.restype = d
    _lib.orc_functional.argtypes = [P(_Grid), i64, P(i32), P(d), P(i32), d, d]


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def grid_struct(grid, quantized: bool = True) -> _Grid:
    g = _Grid()
    g.ndim = grid.ndim
    for d in range(3):
        g.n[d] = int(grid.n[d])
        g.h[d] = float(grid.h[d])
        g.bc[d] = int(grid.bc[d])
    g.depth2d = float(grid.depth2d) if grid.ndim == 2 else 0.0
    g.quantized = 1 if quantized else 0
    return g


def pot_struct(pot) -> _Pot:
    return _Pot(pot.D, pot.r0, pot.s_rep, pot.c_att, pot.g_clamp, pot.n_floor, pot.mass,
                int(getattr(pot, "kind", 0)), int(getattr(pot, "lattice", 0)), float(getattr(pot, "alpha", 0.0)))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(rc, what)


def num_nodes(grid) -> int:
    return int(lib().orc_num_nodes(C.byref(grid_struct(grid))))


def _state(cell, off, wq, vel=None):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.float64)
    wq = np.ascontiguousarray(wq, dtype=np.int32)
    out = [cell, off, wq]
    if vel is not None:
        out.append(np.ascontiguousarray(vel, dtype=np.float64))
    return out


def deposit(grid, cell, off, wq, quantized: bool = True):
    """Node sums: int64 array (quantized) or float64 (unquantized), weight units."""
    cell, off, wq = _state(cell, off, wq)
    g = grid_struct(grid, quantized)
    nn = num_nodes(grid)
    node_f = np.zeros(nn, dtype=np.float64)
    node_q = np.zeros(nn, dtype=np.int64) if quantized else None
    rc = lib().orc_deposit(C.byref(g), cell.shape[0], _ptr(cell, C.c_int32), _ptr(off, C.c_double),
                           _ptr(wq, C.c_int32), _ptr(node_q, C.c_int64) if quantized else None,
                           _ptr(node_f, C.c_double))
    _check(rc, "deposit")
    return node_q if quantized else node_f


def density(grid, node_sums):
    g = grid_struct(grid)
    nf = np.ascontiguousarray(node_sums, dtype=np.float64)
    out = np.zeros_like(nf)
    lib().orc_density(C.byref(g), _ptr(nf, C.c_double), _ptr(out, C.c_double))
    return out


def gradient(grid, dens):
    g = grid_struct(grid)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    out = np.zeros(grid.ndim * grid.ncells, dtype=np.float64)
    lib().orc_gradient(C.byref(g), _ptr(dens, C.c_double), _ptr(out, C.c_double))
    return out.reshape(grid.ndim, grid.ncells)


def gather(grid, dens, G, cell: int, f):
    g = grid_struct(grid)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    fa = np.ascontiguousarray(list(f) + [0.0] * (3 - len(f)), dtype=np.float64)
    n_p = C.c_double()
    G_p = np.zeros(3)
    lib().orc_gather(C.byref(g), _ptr(dens, C.c_double), _ptr(G, C.c_double), int(cell),
                     _ptr(fa, C.c_double), C.byref(n_p), _ptr(G_p, C.c_double))
    return n_p.value, G_p[: grid.ndim].copy()


def local_force(pot, ndim, n_p, G_p):
    Gp = np.ascontiguousarray(list(G_p) + [0.0] * (3 - len(G_p)), dtype=np.float64)
    F = np.zeros(3)
    lib().orc_local_force(C.byref(pot_struct(pot)), ndim, float(n_p), _ptr(Gp, C.c_double),
                          _ptr(F, C.c_double))
    return F[:ndim].copy()


def neighbour_distances(pot, n_p, G_pd):
    rp, rm = C.c_double(), C.c_double()
    lib().orc_neighbour_distances(C.byref(pot_struct(pot)), float(n_p), float(G_pd), C.byref(rp),
                                  C.byref(rm))
    return rp.value, rm.value


def phi_prime(pot, r):
    return lib().orc_phi_prime(C.byref(pot_struct(pot)), float(r))


def phi(pot, r):
    return lib().orc_phi(C.byref(pot_struct(pot)), float(r))


def energy_density(pot, n):
    return lib().orc_energy_density(C.byref(pot_struct(pot)), float(n))


def hcp_directions():
    """The 12 nearest-neighbour unit vectors of the oracle's hexagonal
    close-packed lattice, (basal 1, basal 2, c) axes, shape [12, 3]."""
    out = np.zeros((12, 3))
    for k in range(12):
        u = (C.c_double * 3)()
        lib().orc_hcp_direction(k, u)
        out[k] = list(u)
    return out


def energy_density_quad(pot, n):
    """The energy density by quadrature of mu (any kind of pair potential)."""
    return lib().orc_energy_density_quad(C.byref(pot_struct(pot)), float(n))


def forces(grid, pot, cell, off, wq, quantized: bool = True):
    """Per-atom force [ndim, N] (newtons) from the deposit of the same particles."""
    node = deposit(grid, cell, off, wq, quantized).astype(np.float64)
    cell, off, wq = _state(cell, off, wq)
    F = np.zeros((grid.ndim, cell.shape[0]), dtype=np.float64)
    lib().orc_forces(C.byref(grid_struct(grid, quantized)), C.byref(pot_struct(pot)),
                     _ptr(node, C.c_double), cell.shape[0], _ptr(cell, C.c_int32),
                     _ptr(off, C.c_double), _ptr(F, C.c_double))
    return F


def push_one(grid, pot, dt, F, cell, f, v):
    Fa = np.ascontiguousarray(list(F) + [0.0] * (3 - len(F)), dtype=np.float64)
    c = C.c_int32(int(cell))
    fa = np.ascontiguousarray(list(f) + [0.0] * (3 - len(f)), dtype=np.float64)
    va = np.ascontiguousarray(v, dtype=np.float64).copy()
    rc = lib().orc_push_one(C.byref(grid_struct(grid)), C.byref(pot_struct(pot)), float(dt),
                            _ptr(Fa, C.c_double), C.byref(c), _ptr(fa, C.c_double),
                            _ptr(va, C.c_double))
    _check(rc, "push")
    return c.value, fa[: grid.ndim].copy(), va


def kick(grid, pot, dt, frac, F, vel):
    vel = np.ascontiguousarray(vel, dtype=np.float64).copy()
    F = np.ascontiguousarray(F, dtype=np.float64)
    lib().orc_kick(C.byref(grid_struct(grid)), C.byref(pot_struct(pot)), float(dt), float(frac),
                   vel.shape[1], _ptr(F, C.c_double), _ptr(vel, C.c_double))
    return vel


DIAG_FIELDS = ("ke", "pe", "px", "py", "pz", "wsum", "bond", "step")


def run(grid, pot, dt, cell, off, vel, wq, nsteps, diag_every=0, quantized=True, threads=0, copy=True):
    """Advance a copy of the state nsteps leapfrog cycles (vel = v(n-1/2)).
    Returns (cell, off, vel, diags) with diags a list of dicts.  threads > 0
    runs the OpenMP build with that many threads (same state bits when
    quantized; diagnostic sums in another order).  copy=False advances
    cell (int32), off and vel (float64, C-contiguous) in place."""
    L = lib_threaded(threads) if threads > 0 else lib()
    if copy:
        cell, off, vel = np.array(cell, copy=True), np.array(off, dtype=np.float64, copy=True), \
            np.array(vel, dtype=np.float64, copy=True)
    elif not (cell.dtype == np.int32 and off.dtype == np.float64 and vel.dtype == np.float64
              and cell.flags.c_contiguous and off.flags.c_contiguous and vel.flags.c_contiguous):
        raise ValueError("copy=False needs int32 cell and C-contiguous float64 off and vel")
    cell, off, wq, vel = _state(cell, off, wq, vel)
    nd = 0 if diag_every <= 0 else (nsteps + diag_every - 1) // diag_every
    diags = (_Diag * max(nd, 1))()
    rc = L.orc_run(C.byref(grid_struct(grid, quantized)), C.byref(pot_struct(pot)), float(dt),
                       cell.shape[0], _ptr(cell, C.c_int32), _ptr(off, C.c_double),
                       _ptr(vel, C.c_double), _ptr(wq, C.c_int32), int(nsteps), int(diag_every),
                       diags if nd > 0 else None)
    _check(rc, "run")
    out = [{k: getattr(diags[i], k) for k in DIAG_FIELDS} for i in range(nd)]
    return cell, off, vel, out


def start_leapfrog(grid, pot, dt, cell, off, vel, wq, quantized=True):
    """v(-1/2) = v(0) - F(0)/m dt/2."""
    F = forces(grid, pot, cell, off, wq, quantized)
    return kick(grid, pot, dt, -0.5, F, vel)


def calibrate_catt(grid, pot, n_solid, slab_layers=8, lattice_k=2):
    c = C.c_double()
    W = C.c_double()
    ys = C.c_double()
    rc = lib().orc_calibrate_catt(C.byref(grid_struct(grid, False)), C.byref(pot_struct(pot)),
                                  float(n_solid), int(slab_layers), int(lattice_k), C.byref(c),
                                  C.byref(W), C.byref(ys))
    _check(rc, "calibrate")
    return c.value, W.value, ys.value


def functional(grid, cell, off, wq, y_s, tau):
    cell, off, wq = _state(cell, off, wq)
    return lib().orc_functional(C.byref(grid_struct(grid)), cell.shape[0], _ptr(cell, C.c_int32),
                                _ptr(off, C.c_double), _ptr(wq, C.c_int32), float(y_s), float(tau))


def heated_start(v_thermal, xi, sigma_ref, fluence_ref, fluence):
    """v(0) = v_th + sigma(F) xi with the kick std proportional to sqrt(F)
    (absorbed energy per atom proportional to the fluence)."""
    s = np.asarray(sigma_ref, dtype=np.float64) * np.sqrt(fluence / fluence_ref)
    return np.asarray(v_thermal, dtype=np.float64) + s[None, :] * np.asarray(xi, dtype=np.float64)


def crater_objective(grid, pot, dt, nsteps, cell, off, v_thermal, xi, sigma_ref, fluence_ref, fluence, wq,
                     y_s, tau, quantized=False):
    """J = sum_p w_p sigmoid((y_p(T) - y_s)/tau) after nsteps from the heated
    start, v(-1/2) = v(0) - F(0)/m dt/2.  Unquantized by default: the
    fixed-point deposit is piecewise constant in the positions."""
    v0 = heated_start(v_thermal, xi, sigma_ref, fluence_ref, fluence)
    off = np.asarray(off, dtype=np.float64)
    vh = start_leapfrog(grid, pot, dt, cell, off, v0, wq, quantized)
    c, o, _, _ = run(grid, pot, dt, cell, off, vh, wq, nsteps, quantized=quantized)
    return functional(grid, c, o, wq, y_s, tau)


def forces_from_nodes(grid, pot, node_sums, cell, off, quantized: bool = True):
    """Per-atom force [ndim, N] (newtons) of the given particles from node sums
    of the whole grid (int64 weight units, e.g. the deposit of every
    particle), not only of the particles passed."""
    node = np.ascontiguousarray(node_sums, dtype=np.float64)
    cell, off, _ = _state(cell, off, np.zeros(len(cell), np.int32))
    F = np.zeros((grid.ndim, cell.shape[0]), dtype=np.float64)
    lib().orc_forces(C.byref(grid_struct(grid, quantized)), C.byref(pot_struct(pot)),
                     _ptr(node, C.c_double), cell.shape[0], _ptr(cell, C.c_int32),
                     _ptr(off, C.c_double), _ptr(F, C.c_double))
    return F
