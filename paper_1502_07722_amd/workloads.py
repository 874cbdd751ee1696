"""Seeded synthetic inputs for the PIC pair-potential transport stage.

This module only draws particles: positions, thermal velocities and the
Gaussian-times-exponential heating kick that initialises a laser-heated copper
slab (the paper allows an "empirical heating profile" as the temperature
source of the transport run).  It holds none of the deposit / force / push
arithmetic, so both the GPU path and the FP64 CPU oracle can take their inputs
from here.

Units are SI.  Positions are stored the way the method stores them: an integer
linear cell id ``cell = i + nx*(j + ny*k)`` plus an in-cell offset
``off[d] in [0, 1)`` per evolved axis.  Velocities always have three components
(2D PIC keeps three-component momenta; the paper's 2D paragraph).  Weights are
numbers of real atoms per macroparticle, quantised to ``wq = round(w * 2**20)``.

Every array is generated on the host from ``numpy.random.SeedSequence(seed)``
spawned into three PCG64 streams (positions, Maxwellian, kick), so the same
seed always gives the same particles, whatever consumes them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------------------
# Physical constants (CODATA) and copper parameters.
# ---------------------------------------------------------------------------
AMU = 1.66053906660e-27          # kg
EV = 1.602176634e-19             # J
KB = 1.380649e-23                # J/K
M_CU = 63.546 * AMU              # kg, copper atomic mass
N_SOLID = 8.49e28                # m^-3, solid copper number density (paper: 8.5e22 cm^-3)
R0_CU = N_SOLID ** (-1.0 / 3.0)  # m, L-J equilibrium distance chosen so a cubic lattice at
                                 # solid density sits exactly at r0 (paper leaves D, r0 to a ref.)
D_CU = 0.4093 * EV               # J, L-J well depth (placeholder Cu value; an input everywhere)
W_SHIFT = 20                     # weights are carried as wq = round(w * 2**W_SHIFT)


KIND_LJ, KIND_MORSE = 0, 1
# Morse copper (Girifalco and Weizer, Phys. Rev. 114, 687 (1959)): well depth
# and width; the equilibrium distance is set like the L-J one (R0_CU).
D_MORSE_CU = 0.3429 * EV         # J
ALPHA_MORSE_CU = 1.3588e10       # 1/m


@dataclasses.dataclass
class Potential:
    """Altered pair potential parameters (paper eq. (3) and the paragraph on
    the altered potential and the attractive correction).  kind 0 is the
    paper's Lennard-Jones eq. (3); kind 1 the Morse potential
    D(e^2 - 2e), e = exp(-alpha (r - r0)), which the paper names as an
    alternative."""
    D: float = D_CU
    r0: float = R0_CU
    s_rep: float = 1.0        # multiplier on the repulsive branch (r < r0)
    c_att: float = 1.0        # multiplier on the attractive branch (r >= r0)
    g_clamp: float = 1.0      # clamp on |d rbar/dx| in eq. (2)
    n_floor: float = 1e-6 * N_SOLID   # below this density the force is zero
    mass: float = M_CU
    kind: int = KIND_LJ
    alpha: float = 0.0        # Morse width, 1/m (kind 1)
    lattice: int = 0          # 0 cubic (eqs. (1)-(2) per axis), 1 hexagonal close-packed


LATTICE_CUBIC, LATTICE_HCP = 0, 1
HCP_C = 2.0 ** (1.0 / 6.0)       # nearest-neighbour distance / rbar on a close-packed lattice


def hcp(pot: Optional["Potential"] = None, **kw) -> "Potential":
    """The pair potential on the hexagonal close-packed lattice with r0 at the
    close-packed nearest-neighbour distance of solid copper, 2^(1/6)
    n_s^(-1/3), so that the solid sits at the potential minimum as it does on
    the cubic lattice."""
    pot = pot or Potential()
    args = dict(lattice=LATTICE_HCP, r0=HCP_C * R0_CU)
    args.update(kw)
    return dataclasses.replace(pot, **args)


def morse_cu(**kw) -> Potential:
    """The Morse copper potential at the L-J equilibrium distance."""
    args = dict(D=D_MORSE_CU, kind=KIND_MORSE, alpha=ALPHA_MORSE_CU)
    args.update(kw)
    return Potential(**args)


@dataclasses.dataclass
class Grid:
    ndim: int
    n: tuple                  # cells per axis (3 entries; 2D uses n[2] = 1)
    h: tuple                  # cell size per axis, m
    bc: tuple                 # 0 periodic, 1 reflecting, per axis
    depth2d: float = 0.0      # 2D slab thickness a macroparticle represents (default h[0])

    def __post_init__(self):
        self.n = tuple(int(v) for v in (list(self.n) + [1, 1, 1])[:3])
        self.h = tuple(float(v) for v in (list(self.h) + [self.h[0]] * 3)[:3])
        self.bc = tuple(int(v) for v in (list(self.bc) + [0, 0, 0])[:3])
        if self.ndim == 2 and self.depth2d <= 0.0:
            self.depth2d = self.h[0]

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n[: self.ndim]))

    @property
    def nnodes(self) -> int:
        return int(np.prod([self.n[d] + self.bc[d] for d in range(self.ndim)]))

    @property
    def normal_axis(self) -> int:
        return self.ndim - 1


@dataclasses.dataclass
class Particles:
    """Host particle arrays (float32 state as the GPU keeps it)."""
    cell: np.ndarray          # int32 [N]
    off: np.ndarray           # float32 [ndim, N], each in [0, 1)
    vel: np.ndarray           # float32 [3, N], m/s
    wq: np.ndarray            # int32 [N], weight * 2**20
    xi: Optional[np.ndarray] = None      # float32 [3, N] kick noise (None without laser)
    sigma: Optional[np.ndarray] = None   # float64 [N] kick std per component, m/s
    v_thermal: Optional[np.ndarray] = None  # float32 [3, N] before the kick

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    pot: Potential
    dt: float
    steps: int
    parts: Particles
    slab_rows: int
    fluence: float            # J/m^2 peak absorbed
    extra: dict = dataclasses.field(default_factory=dict)


def weight_q(w_atoms: float) -> int:
    return int(round(w_atoms * (1 << W_SHIFT)))


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]


def _uniform_f32(rng, shape):
    # float32 draws are in [0, 1) by construction; keep an explicit guard.
    u = rng.random(shape, dtype=np.float32)
    return np.minimum(u, np.float32(np.nextafter(np.float32(1), np.float32(0))))


def heating_sigma(x, y_depth, fluence, R, x_c, delta=15e-9, n_s=N_SOLID, mass=M_CU):
    """Per-component std of the heating kick (SI).

    Absorbed energy per atom dE = F/(delta*n_s) * exp(-2 (x-x_c)^2 / R^2) *
    exp(-depth/delta); a Gaussian kick with sigma^2 = 2 dE / (3 m) per
    component raises the mean kinetic energy by dE.  ``y_depth`` is the depth
    below the initial surface (>= 0 inside the slab)."""
    if fluence <= 0.0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    dE = (fluence / (delta * n_s)) * np.exp(-2.0 * (x - x_c) ** 2 / R ** 2) * np.exp(-np.maximum(y_depth, 0.0) / delta)
    return np.sqrt(2.0 * dE / (3.0 * mass))


def make_slab(ndim: int, n: tuple, slab_layers: int, ppc: int, h: float, seed: int,
              fluence_Jcm2: float = 0.0, R_cells: float = 200.0, x_c_cells: Optional[float] = None,
              delta: float = 15e-9, T: float = 300.0, pot: Optional[Potential] = None,
              bc: Optional[tuple] = None, quiet: float = -1.0, depth2d: float = 0.0) -> tuple:
    """A copper slab filling the lowest ``slab_layers`` layers along the normal
    (last) axis, exactly ``ppc`` macroparticles per cell, uniform-random
    offsets, Maxwellian velocities at ``T`` plus the optional heating kick.

    quiet >= 0: quiet-start loading instead of uniform-random offsets: the
    cell's ppc = k^ndim macroparticles sit on a k^ndim sub-lattice, each moved
    by quiet * (u - 1/2) of the sub-spacing per axis (u uniform in [0, 1);
    quiet = 0 is the exact sub-lattice, whose deposit is uniform).

    depth2d > 0 (2D): the thickness the plane stands for (default one cell
    edge); it sets the atoms per macroparticle, not the density.

    Particles are emitted cell by cell in linear cell order."""
    pot = pot or Potential()
    n = tuple(list(n) + [1] * (3 - len(n)))
    if bc is None:
        bc = (0, 1, 0) if ndim == 2 else (0, 0, 1)
    grid = Grid(ndim=ndim, n=n, h=(h, h, h), bc=bc, depth2d=depth2d if ndim == 2 else 0.0)
    rng_pos, rng_mb, rng_kick = _streams(seed)
    lateral = int(np.prod(n[: ndim - 1]))
    ncell_slab = lateral * slab_layers
    N = ncell_slab * ppc
    cell = np.repeat(np.arange(ncell_slab, dtype=np.int64), ppc).astype(np.int32)
    if quiet >= 0.0:
        k = int(round(ppc ** (1.0 / ndim)))
        if k ** ndim != ppc or not quiet <= 1.0:
            raise ValueError("quiet start needs ppc = k^ndim and 0 <= quiet <= 1")
        sub = np.stack(np.meshgrid(*[np.arange(k)] * ndim, indexing="ij"), axis=0).reshape(ndim, ppc)
        base = np.tile(sub, (1, ncell_slab)).astype(np.float64)
        u = rng_pos.random((ndim, N))
        off = ((base + 0.5 + quiet * (u - 0.5)) / k).astype(np.float32)
        off = np.minimum(off, np.float32(np.nextafter(np.float32(1), np.float32(0))))
    else:
        off = _uniform_f32(rng_pos, (ndim, N))
    atoms_per_cell = N_SOLID * h ** 3 if ndim == 3 else N_SOLID * h * h * grid.depth2d
    w = atoms_per_cell / ppc
    wq = np.full(N, weight_q(w), dtype=np.int32)
    sig_th = math.sqrt(KB * T / pot.mass) if T > 0 else 0.0
    v_th = rng_mb.standard_normal((3, N), dtype=np.float32)
    v_th *= np.float32(sig_th)
    xi = sigma = None
    vel = v_th
    if fluence_Jcm2 > 0.0:
        xi = rng_kick.standard_normal((3, N), dtype=np.float32)
        nx = n[0]
        i = cell.astype(np.int64) % nx
        layer = cell.astype(np.int64) // lateral
        x = (i + off[0].astype(np.float64)) * h
        y = (layer + off[ndim - 1].astype(np.float64)) * h
        y_s = slab_layers * h
        x_c = (x_c_cells if x_c_cells is not None else nx / 2.0) * h
        sigma = heating_sigma(x, y_s - y, fluence_Jcm2 * 1e4, R_cells * h, x_c, delta=delta, mass=pot.mass)
        vel = (v_th + sigma[None, :] * xi).astype(np.float32)
    parts = Particles(cell=cell, off=off, vel=np.ascontiguousarray(vel, dtype=np.float32), wq=wq,
                      xi=xi, sigma=sigma, v_thermal=v_th if xi is not None else None)
    return grid, parts


def make_lattice(ndim: int, n: tuple, k: int, h: float, fill_layers: Optional[int] = None,
                 bc: Optional[tuple] = None, T: float = 0.0, seed: int = 7) -> tuple:
    """A commensurate lattice: k^ndim macroparticles per cell at offsets
    (a + 1/2)/k, in the lowest ``fill_layers`` layers (all layers by default),
    each macroparticle carrying solid density.  T = 0 gives a static state."""
    n = tuple(list(n) + [1] * (3 - len(n)))
    if bc is None:
        bc = (0,) * 3
    grid = Grid(ndim=ndim, n=n, h=(h, h, h), bc=bc)
    lateral = int(np.prod(n[: ndim - 1]))
    layers = n[ndim - 1] if fill_layers is None else fill_layers
    ncell = lateral * layers
    per = k ** ndim
    cell = np.repeat(np.arange(ncell, dtype=np.int64), per).astype(np.int32)
    sub = np.stack(np.meshgrid(*[np.arange(k)] * ndim, indexing="ij"), axis=0).reshape(ndim, per)
    off = ((np.tile(sub, (1, ncell)) + 0.5) / k).astype(np.float32)
    w = N_SOLID * h ** 3 / per
    wq = np.full(ncell * per, weight_q(w), dtype=np.int32)
    vel = np.zeros((3, ncell * per), dtype=np.float32)
    if T > 0:
        rng = _streams(seed)[1]
        vel = (rng.standard_normal((3, ncell * per)) * math.sqrt(KB * T / M_CU)).astype(np.float32)
    return grid, Particles(cell=cell, off=off, vel=vel, wq=wq)


# ---------------------------------------------------------------------------
# The named workloads (2 nm cells, dt 1 fs, Cu at 8.49e28 m^-3, 300 K).
# ---------------------------------------------------------------------------
H_CELL = 2e-9
DT = 1e-15


def cfg_small_slab(seed: int = 1) -> Workload:
    """64x64 cells, x periodic / y reflecting, lower 32 rows at 16 ppc
    (32,768 particles), 300 K, no laser, 200 steps."""
    grid, parts = make_slab(2, (64, 64), 32, 16, H_CELL, seed)
    return Workload("slab2d_64x64_16ppc", grid, Potential(), DT, 200, parts, 32, 0.0)


def cfg_heated_slab(seed: int = 2) -> Workload:
    """1024x512 cells, slab in lower 256 rows, 32 ppc (8,388,608 particles),
    300 K plus a 1 J/cm^2 Gaussian (1/e^2 radius 200 cells) x exp(-depth/15 nm)
    heating kick, 5000 steps."""
    grid, parts = make_slab(2, (1024, 512), 256, 32, H_CELL, seed, fluence_Jcm2=1.0, R_cells=200.0)
    return Workload("slab2d_1024x512_32ppc_1Jcm2", grid, Potential(), DT, 5000, parts, 256, 1e4)


def cfg_large_slab(seed: int = 3) -> Workload:
    """4096x2048 cells, slab in lower 1024 rows, 32 ppc (134,217,728
    particles), 2 J/cm^2 heating centred at x = 2048 cells, 2000 steps."""
    grid, parts = make_slab(2, (4096, 2048), 1024, 32, H_CELL, seed, fluence_Jcm2=2.0, R_cells=200.0)
    return Workload("slab2d_4096x2048_32ppc_2Jcm2", grid, Potential(), DT, 2000, parts, 1024, 2e4)


def sweep_table(seed: int = 4, nslab: int = 24) -> List[dict]:
    """The intensity sweep: widths U{256..2048} cells, depths U{128..512}
    rows, box height 2*depth, ppc U{16..32}, fluences 0.2 * 25**(k/23) J/cm^2."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    out = []
    for k in range(nslab):
        width = int(rng.integers(256, 2049))
        depth = int(rng.integers(128, 513))
        ppc = int(rng.integers(16, 33))
        F = 0.2 * 25.0 ** (k / max(nslab - 1, 1))
        out.append(dict(width=width, depth=depth, height=2 * depth, ppc=ppc, fluence_Jcm2=F,
                        seed=int(seed * 1000 + k)))
    return out


def cfg_sweep(seed: int = 4, nslab: int = 24, scale: float = 1.0) -> List[Workload]:
    """24 independent slabs of uneven size (the paper's intensity sweep).
    ``scale`` < 1 shrinks widths/depths for tests (same structure)."""
    wls = []
    for row in sweep_table(seed, nslab):
        W = max(8, int(row["width"] * scale))
        Dp = max(4, int(row["depth"] * scale))
        grid, parts = make_slab(2, (W, 2 * Dp), Dp, row["ppc"], H_CELL, row["seed"],
                                fluence_Jcm2=row["fluence_Jcm2"], R_cells=200.0 * scale)
        wls.append(Workload(f"sweep_{W}x{2*Dp}_{row['ppc']}ppc_{row['fluence_Jcm2']:.3f}Jcm2",
                            grid, Potential(), DT, 1000, parts, Dp, row["fluence_Jcm2"] * 1e4))
    return wls


def cfg_adjoint_3d(seed: int = 5, n: int = 128, layers: Optional[int] = None) -> Workload:
    """3D n^3 cells of 2 nm (x, y periodic, z reflecting), slab in the lower
    half, 8 ppc, 1.5 J/cm^2 heating (R = 400 nm), 400 steps, checkpoints
    every 20 steps."""
    layers = n // 2 if layers is None else layers
    grid, parts = make_slab(3, (n, n, n), layers, 8, H_CELL, seed, fluence_Jcm2=1.5,
                            R_cells=200.0, x_c_cells=n / 2.0)
    return Workload(f"slab3d_{n}cube_8ppc_1.5Jcm2", grid, Potential(), DT, 400, parts, layers, 1.5e4,
                    extra=dict(checkpoint_every=20))


WORKLOADS = {
    "small": cfg_small_slab,
    "heated": cfg_heated_slab,
    "large": cfg_large_slab,
    "adjoint3d": cfg_adjoint_3d,
}
