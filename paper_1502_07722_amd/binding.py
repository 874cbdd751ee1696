"""Thin Python binding of libpic.so (the C ABI in include/pic.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the HIP stream.  There
is no fallback: if the library has not been built, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ERANGE, PIC_ECFL, PIC_EOVERFLOW, PIC_EHIP, PIC_ENOSPACE = range(7)
_NAMES = {0: "PIC_OK", 1: "PIC_EINVAL", 2: "PIC_ERANGE", 3: "PIC_ECFL", 4: "PIC_EOVERFLOW",
          5: "PIC_EHIP", 6: "PIC_ENOSPACE"}


class pic_grid_t(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 3),
                ("depth2d", C.c_double)]


class pic_potential_t(C.Structure):
    _fields_ = [("D", C.c_double), ("r0", C.c_double), ("s_rep", C.c_double), ("c_att", C.c_double),
                ("g_clamp", C.c_double), ("n_floor", C.c_double), ("mass", C.c_double), ("kind", C.c_int32),
                ("lattice", C.c_int32), ("alpha", C.c_double)]


class pic_particles_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("cell", C.c_void_p), ("off", C.c_void_p), ("vel", C.c_void_p),
                ("wq", C.c_void_p)]


class pic_diag_t(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("px", C.c_double), ("py", C.c_double),
                ("pz", C.c_double), ("wsum", C.c_double), ("bond", C.c_double), ("step", C.c_int64)]


DIAG_FIELDS = ("ke", "pe", "px", "py", "pz", "wsum", "bond", "step")
PHASES = ("deposit", "grid", "force_push", "sort", "diag", "import_export", "unused", "graph")


class pic_tuning_t(C.Structure):
    _fields_ = [("tile", C.c_int32), ("halo", C.c_int32), ("chunk", C.c_int32), ("candidates", C.c_int32),
                ("ms_per_step", C.c_double), ("tile_last", C.c_int32)]


class pic_timing_t(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8), ("drifters_last", C.c_int64),
                ("items_last", C.c_int64)]

class pic_crater_spec_t(C.Structure):
    _fields_ = [("n_solid", C.c_double), ("cut", C.c_double), ("depth_min", C.c_double)]


class pic_crater_t(C.Structure):
    _fields_ = [("depth", C.c_double), ("width", C.c_double), ("t_min", C.c_double), ("t_max", C.c_double),
                ("f_th", C.c_double), ("ncols", C.c_int64)]


CRATER_FIELDS = ("depth", "width", "t_min", "t_max", "f_th", "ncols")
NTHETA = 5  # reverse-mode parameters: D, r0, s_rep, c_att, alpha

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")

lib = C.CDLL(LIB_PATH)
_P = C.POINTER
_vp = C.c_void_p
lib.pic_num_nodes.restype = C.c_int64
lib.pic_num_nodes.argtypes = [_P(pic_grid_t)]
lib.pic_workspace_bytes.restype = C.c_size_t
lib.pic_workspace_bytes.argtypes = [_P(pic_grid_t), C.c_int64]
lib.pic_init.argtypes = [_P(_vp), _P(pic_grid_t), _P(pic_potential_t), C.c_double, C.c_int64, _vp, C.c_size_t, _vp]
lib.pic_destroy.argtypes = [_vp]
lib.pic_last_error.restype = C.c_char_p
lib.pic_last_error.argtypes = [_vp]
lib.pic_sync.argtypes = [_vp]
lib.pic_deposit.argtypes = [_vp, _P(pic_particles_t), _vp]
lib.pic_force.argtypes = [_vp, _P(pic_particles_t), _vp, _vp, _P(pic_diag_t)]
lib.pic_kick.argtypes = [_vp, _P(pic_particles_t), _vp, C.c_double]
lib.pic_force_noalloc.argtypes = [_P(pic_grid_t), _P(pic_potential_t), _P(pic_particles_t), _vp, _vp, _vp]
NOALLOC_SCRATCH_BYTES = 64 << 20
lib.pic_push.argtypes = [_vp, _P(pic_particles_t), _vp]
lib.pic_step.argtypes = [_vp, _P(pic_particles_t), C.c_int32, _P(pic_diag_t), C.c_int32]
lib.pic_set_timing.argtypes = [_vp, C.c_int32]
lib.pic_set_tiling.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
lib.pic_get_tiling.argtypes = [_vp, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)]
lib.pic_set_tile_shape.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
lib.pic_get_tile_shape.argtypes = [_vp, _P(C.c_int32), _P(C.c_int32)]
lib.pic_set_graph.argtypes = [_vp, C.c_int32]
lib.pic_set_record_states.argtypes = [_vp, C.c_int32]
lib.pic_autotune.argtypes = [_vp, _P(pic_particles_t), C.c_int32, _P(pic_tuning_t)]
lib.pic_workspace_bytes_batch.restype = C.c_size_t
lib.pic_workspace_bytes_batch.argtypes = [_P(pic_grid_t), C.c_int32, _P(C.c_int64)]
lib.pic_init_batch.argtypes = [_P(_vp), _P(pic_grid_t), C.c_int32, _P(pic_potential_t), C.c_double, _P(C.c_int64),
                               _vp, C.c_size_t, _vp]
lib.pic_step_batch.argtypes = [_vp, _P(pic_particles_t), C.c_int32, _P(pic_diag_t), C.c_int32]
lib.pic_set_path.argtypes = [_vp, C.c_int32]
lib.pic_step_nodes.argtypes = [_vp, _vp]
lib.pic_get_timing.argtypes = [_vp, _P(pic_timing_t)]
lib.pic_adjoint_step.argtypes = [_vp, _P(pic_particles_t), _vp, _vp, _vp, _vp, _vp, _vp]
lib.pic_force_vjp.argtypes = [_vp, _P(pic_particles_t), _vp, _vp, _vp, _vp, _vp]
lib.pic_deposit_vjp.argtypes = [_vp, _P(pic_particles_t), _vp, _vp]
lib.pic_record_bytes.argtypes = [_vp, C.c_int32, C.c_int32]
lib.pic_record_bytes.restype = C.c_size_t
lib.pic_backward_bytes.argtypes = [_vp, C.c_int32]
lib.pic_backward_bytes.restype = C.c_size_t
lib.pic_forward_record.argtypes = [_vp, _P(pic_particles_t), C.c_int32, C.c_int32, _vp, C.c_size_t]
lib.pic_backward_record.argtypes = [_vp, _P(pic_particles_t), C.c_int32, C.c_int32, _vp, C.c_size_t, _vp,
                                    C.c_size_t, _vp, _vp, _vp, C.c_double]
lib.pic_calibrate_catt.argtypes = [_P(pic_grid_t), _P(pic_potential_t), C.c_double, C.c_int32, _P(C.c_double),
                                   _P(C.c_double)]
lib.pic_num_columns.restype = C.c_int64
lib.pic_num_columns.argtypes = [_P(pic_grid_t)]
lib.pic_crater.argtypes = [_vp, _vp, _P(pic_crater_spec_t), _P(C.c_double), _P(C.c_double), _P(C.c_double), _vp,
                           _vp, _vp]
lib.pic_threshold_fit.argtypes = [C.c_int32, _P(C.c_double), _P(C.c_double), C.c_double, _P(C.c_double),
                                  _P(C.c_double), _P(C.c_double)]


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def grid_t(grid: W.Grid) -> pic_grid_t:
    g = pic_grid_t()
    g.ndim = grid.ndim
    for d in range(3):
        g.n[d] = int(grid.n[d])
        g.h[d] = float(grid.h[d])
        g.bc[d] = int(grid.bc[d])
    g.depth2d = float(grid.depth2d) if grid.ndim == 2 else 0.0
    return g


def potential_t(pot: W.Potential) -> pic_potential_t:
    return pic_potential_t(pot.D, pot.r0, pot.s_rep, pot.c_att, pot.g_clamp, pot.n_floor, pot.mass,
                           int(pot.kind), int(pot.lattice), float(pot.alpha))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class DeviceParticles:
    """Caller-owned device arrays in the layout of pic_particles_t."""

    def __init__(self, cell, off, vel, wq):
        self.cell, self.off, self.vel, self.wq = cell, off, vel, wq
        for t in (cell, off, vel, wq):
            assert t.is_cuda and t.is_contiguous()
        assert cell.dtype == torch.int32 and wq.dtype == torch.int32
        assert off.dtype == torch.float32 and vel.dtype == torch.float32

    @classmethod
    def from_host(cls, parts: W.Particles, device="cuda"):
        return cls(torch.from_numpy(parts.cell).to(device).contiguous(),
                   torch.from_numpy(parts.off).to(device).contiguous(),
                   torch.from_numpy(parts.vel).to(device).contiguous(),
                   torch.from_numpy(parts.wq).to(device).contiguous())

    @property
    def n(self):
        return int(self.cell.shape[0])

    def struct(self) -> pic_particles_t:
        return pic_particles_t(self.n, self.cell.data_ptr(), self.off.data_ptr(), self.vel.data_ptr(),
                               self.wq.data_ptr())

    def clone(self):
        return DeviceParticles(self.cell.clone(), self.off.clone(), self.vel.clone(), self.wq.clone())

    def to_host(self):
        return (self.cell.cpu().numpy(), self.off.cpu().numpy(), self.vel.cpu().numpy(), self.wq.cpu().numpy())


def pic_num_nodes(grid: W.Grid) -> int:
    return int(lib.pic_num_nodes(C.byref(grid_t(grid))))


def pic_workspace_bytes(grid: W.Grid, max_n: int) -> int:
    return int(lib.pic_workspace_bytes(C.byref(grid_t(grid)), int(max_n)))


def pic_calibrate_catt(grid: W.Grid, pot: W.Potential, n_solid: float, slab_layers: int = 8):
    c, w = C.c_double(), C.c_double()
    rc = lib.pic_calibrate_catt(C.byref(grid_t(grid)), C.byref(potential_t(pot)), float(n_solid),
                                int(slab_layers), C.byref(c), C.byref(w))
    if rc:
        raise PicError(rc, "calibration failed")
    return c.value, w.value


def pic_num_columns(grid: W.Grid) -> int:
    return int(lib.pic_num_columns(C.byref(grid_t(grid))))


def pic_threshold_fit(fluences, widths, beam_d: float):
    """(fixed-diameter estimate, fitted estimate, fitted diameter) of the
    threshold fluence over a sweep (NaN where undetermined)."""
    n = len(fluences)
    F = (C.c_double * max(n, 1))(*[float(x) for x in fluences])
    G = (C.c_double * max(n, 1))(*[float(x) for x in widths])
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    rc = lib.pic_threshold_fit(n, F, G, float(beam_d), C.byref(a), C.byref(b), C.byref(c))
    if rc:
        raise PicError(rc, "pic_threshold_fit failed")
    return a.value, b.value, c.value


def pic_force_noalloc(grid: W.Grid, pot: W.Potential, parts: DeviceParticles, force=None, device_error=None,
                      stream=None):
    """pic_deposit + pic_force without a context, the library's grids in its
    static scratch array (no allocation by the library).  force: float32
    [ndim, n] (a new tensor when None); device_error: optional int32 [1]
    device word (error bits OR-ed in).  Returns force."""
    dev = parts.cell.device
    n = parts.n
    if force is None:
        force = torch.empty((grid.ndim, n), dtype=torch.float32, device=dev)
    if not (force.is_cuda and force.is_contiguous() and force.dtype == torch.float32
            and force.numel() >= grid.ndim * n):
        raise PicError(PIC_EINVAL, "force must be a contiguous float32 CUDA tensor of ndim * n elements")
    if device_error is not None and not (device_error.is_cuda and device_error.dtype == torch.int32):
        raise PicError(PIC_EINVAL, "device_error must be an int32 CUDA tensor")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    s = parts.struct()
    rc = lib.pic_force_noalloc(C.byref(grid_t(grid)), C.byref(potential_t(pot)), C.byref(s), _ptr(force),
                               _ptr(device_error), C.c_void_p(st.cuda_stream))
    if rc:
        raise PicError(rc, "pic_force_noalloc failed")
    return force


class Context:
    """One pic_ctx_t with its workspace tensor, bound to a torch stream."""

    nslab = 1

    def __init__(self, grid: W.Grid, pot: W.Potential, dt: float, max_n: int, device="cuda", stream=None):
        self.grid, self.pot, self.dt, self.max_n = grid, pot, dt, int(max_n)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = pic_workspace_bytes(grid, max_n)
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "invalid grid")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = C.c_void_p()
        rc = lib.pic_init(C.byref(self.ctx), C.byref(grid_t(grid)), C.byref(potential_t(pot)), float(dt),
                          self.max_n, C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream))
        if rc:
            raise PicError(rc, "pic_init failed")
        self.nnodes = pic_num_nodes(grid)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and lib is not None:  # the module may already be torn down at exit
            lib.pic_destroy(ctx)
            self.ctx = None

    def _need(self, t, numel, dtype, what):
        """Host-side size check of a caller buffer before any launch."""
        if t is None or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() < numel:
            raise ValueError(f"{what}: need a contiguous {dtype} device tensor of >= {numel} elements")

    def _parts_ok(self, parts):
        n = parts.n
        if parts.off.numel() < self.grid.ndim * n or parts.vel.numel() < 3 * n or parts.wq.numel() < n:
            raise ValueError("particle arrays are smaller than n")

    def _check(self, rc, what):
        if rc:
            raise PicError(rc, f"{what}: {lib.pic_last_error(self.ctx).decode()}")

    def pic_sync(self):
        self._check(lib.pic_sync(self.ctx), "pic_sync")

    def pic_deposit(self, parts: DeviceParticles, node_w=None):
        if node_w is None:
            node_w = torch.empty(self.nnodes, dtype=torch.int64, device=self.device)
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        self._parts_ok(parts)
        s = parts.struct()
        self._check(lib.pic_deposit(self.ctx, C.byref(s), _ptr(node_w)), "pic_deposit")
        return node_w

    def pic_force(self, parts: DeviceParticles, node_w, force=None, want_pe=False):
        if force is None:
            force = torch.empty((self.grid.ndim, parts.n), dtype=torch.float32, device=self.device)
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        self._need(force, self.grid.ndim * parts.n, torch.float32, "force")
        self._parts_ok(parts)
        s = parts.struct()
        d = pic_diag_t()
        self._check(lib.pic_force(self.ctx, C.byref(s), _ptr(node_w), _ptr(force),
                                  C.byref(d) if want_pe else None), "pic_force")
        return (force, d.pe) if want_pe else force

    def pic_kick(self, parts: DeviceParticles, force, frac: float):
        self._need(force, self.grid.ndim * parts.n, torch.float32, "force")
        self._parts_ok(parts)
        s = parts.struct()
        self._check(lib.pic_kick(self.ctx, C.byref(s), _ptr(force), float(frac)), "pic_kick")

    def pic_push(self, parts: DeviceParticles, force):
        self._need(force, self.grid.ndim * parts.n, torch.float32, "force")
        self._parts_ok(parts)
        s = parts.struct()
        self._check(lib.pic_push(self.ctx, C.byref(s), _ptr(force)), "pic_push")

    def pic_step(self, parts: DeviceParticles, nsteps: int, diag_every: int = 0):
        self._parts_ok(parts)
        s = parts.struct()
        nd = 0 if diag_every <= 0 else (nsteps + diag_every - 1) // diag_every
        buf = (pic_diag_t * max(nd, 1))()
        self._check(lib.pic_step(self.ctx, C.byref(s), int(nsteps), buf if nd else None,
                                 int(diag_every) if nd else 0), "pic_step")
        return [{k: getattr(buf[i], k) for k in DIAG_FIELDS} for i in range(nd)]

    def pic_set_tiling(self, tile: int, halo: int, chunk: int, sort_every: int):
        self._check(lib.pic_set_tiling(self.ctx, tile, halo, chunk, sort_every), "pic_set_tiling")

    def pic_get_tiling(self):
        v = [C.c_int32() for _ in range(4)]
        self._check(lib.pic_get_tiling(self.ctx, *[C.byref(x) for x in v]), "pic_get_tiling")
        return tuple(x.value for x in v)

    def pic_set_tile_shape(self, tile: int, tile_last: int, halo: int, chunk: int, sort_every: int):
        self._check(lib.pic_set_tile_shape(self.ctx, tile, tile_last, halo, chunk, sort_every),
                    "pic_set_tile_shape")

    def pic_get_tile_shape(self):
        v = [C.c_int32() for _ in range(2)]
        self._check(lib.pic_get_tile_shape(self.ctx, *[C.byref(x) for x in v]), "pic_get_tile_shape")
        return tuple(x.value for x in v)

    def pic_autotune(self, parts, probe_steps: int = 10):
        """parts: one DeviceParticles (single slab) or a list (batch)."""
        plist = parts if isinstance(parts, (list, tuple)) else [parts]
        arr = (pic_particles_t * len(plist))(*[p.struct() for p in plist])
        t = pic_tuning_t()
        self._check(lib.pic_autotune(self.ctx, arr, int(probe_steps), C.byref(t)), "pic_autotune")
        return {"tile": t.tile, "tile_last": t.tile_last, "halo": t.halo, "chunk": t.chunk,
                "candidates": t.candidates, "ms_per_step": t.ms_per_step}

    def pic_set_graph(self, on: bool):
        self._check(lib.pic_set_graph(self.ctx, 1 if on else 0), "pic_set_graph")

    def pic_set_record_states(self, all_states: bool):
        """True: records keep every state and node sum (no recompute in the
        reverse sweep, records about nsteps x a state); False: checkpoints only."""
        self._check(lib.pic_set_record_states(self.ctx, 1 if all_states else 0), "pic_set_record_states")

    def pic_set_path(self, untiled: bool):
        self._check(lib.pic_set_path(self.ctx, 1 if untiled else 0), "pic_set_path")

    def pic_step_nodes(self, node_w=None):
        if node_w is None:
            node_w = torch.empty(self.nnodes, dtype=torch.int64, device=self.device)
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        self._check(lib.pic_step_nodes(self.ctx, _ptr(node_w)), "pic_step_nodes")
        return node_w

    def _grids(self):
        return getattr(self, "grids", None) or [self.grid]

    def crater_buffers(self, want_rho: bool = False):
        """Device outputs of pic_crater: (col_w, rho or None, out)."""
        ncols = sum(pic_num_columns(g) for g in self._grids())
        col_w = torch.empty(ncols, dtype=torch.int64, device=self.device)
        rho = torch.empty(self.nnodes, dtype=torch.float32, device=self.device) if want_rho else None
        out = torch.empty(self.nslab * C.sizeof(pic_crater_t), dtype=torch.uint8, device=self.device)
        return col_w, rho, out

    def pic_crater_launch(self, node_w, n_solid: float, y_s, cut: float = 0.01, depth_min=None, fluence=None,
                          beam_d=None, bufs=None):
        """Enqueue pic_crater (asynchronous); returns the device buffers
        (col_w, rho, out).  Per-slab arguments are sequences of nslab values
        (a scalar is taken for every slab); depth_min defaults to one cell
        along the normal axis."""
        grids = self._grids()
        k = self.nslab

        def per_slab(v):
            v = list(v) if hasattr(v, "__len__") else [v] * k
            if len(v) != k:
                raise ValueError("one value per slab")
            return (C.c_double * k)(*[float(x) for x in v])

        if depth_min is None:
            depth_min = grids[0].h[grids[0].ndim - 1]
        col_w, rho, out = bufs if bufs is not None else self.crater_buffers()
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        self._need(col_w, sum(pic_num_columns(g) for g in grids), torch.int64, "col_w")
        if rho is not None:
            self._need(rho, self.nnodes, torch.float32, "rho")
        self._need(out, k * C.sizeof(pic_crater_t), torch.uint8, "out")
        spec = pic_crater_spec_t(float(n_solid), float(cut), float(depth_min))
        F = per_slab(fluence) if fluence is not None else None
        A = per_slab(beam_d) if beam_d is not None else None
        self._check(lib.pic_crater(self.ctx, _ptr(node_w), C.byref(spec), per_slab(y_s), F, A, _ptr(rho),
                                   _ptr(col_w), _ptr(out)), "pic_crater")
        return col_w, rho, out

    def crater_results(self, out):
        """Unpack pic_crater's device results (waits for the bound stream)."""
        self.stream.synchronize()
        raw = bytes(out.cpu().numpy().tobytes())
        recs = (pic_crater_t * self.nslab).from_buffer_copy(raw[: self.nslab * C.sizeof(pic_crater_t)])
        return [{f: getattr(r, f) for f in CRATER_FIELDS} for r in recs]

    def pic_crater(self, node_w, n_solid: float, y_s, cut: float = 0.01, depth_min=None, fluence=None,
                   beam_d=None, want_rho: bool = False):
        """Crater measurement of every slab: (per-slab result dicts, col_w, rho)."""
        bufs = self.crater_buffers(want_rho)
        col_w, rho, out = self.pic_crater_launch(node_w, n_solid, y_s, cut, depth_min, fluence, beam_d, bufs)
        return self.crater_results(out), col_w, rho

    def pic_set_timing(self, on: bool):
        self._check(lib.pic_set_timing(self.ctx, 1 if on else 0), "pic_set_timing")

    def pic_get_timing(self):
        t = pic_timing_t()
        self._check(lib.pic_get_timing(self.ctx, C.byref(t)), "pic_get_timing")
        out = {PHASES[i]: (t.ms[i], t.launches[i]) for i in range(8) if t.launches[i]}
        out["drifters_last"] = t.drifters_last
        out["items_last"] = t.items_last
        return out

    # reverse mode -----------------------------------------------------------
    def _adj_bufs(self, parts, lam_x, lam_v, nbar, dtheta):
        nd, n = self.grid.ndim, parts.n
        if lam_x is not None:
            self._need(lam_x, nd * n, torch.float32, "lam_x")
        if lam_v is not None:
            self._need(lam_v, 3 * n, torch.float32, "lam_v")
        if nbar is None:
            nbar = torch.empty(self.nnodes, dtype=torch.float32, device=self.device)
        self._need(nbar, self.nnodes, torch.float32, "nbar")
        if dtheta is None:
            dtheta = torch.zeros(NTHETA, dtype=torch.float64, device=self.device)
        self._need(dtheta, NTHETA, torch.float64, "dtheta")
        return nbar, dtheta

    def pic_adjoint_step(self, state: DeviceParticles, node_w, nbar_next, lam_x, lam_v, nbar=None, dtheta=None):
        """One reverse step; lam_x and lam_v are updated in place.  Returns
        (nbar, dtheta) with dtheta accumulated."""
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        if nbar_next is not None:
            self._need(nbar_next, self.nnodes, torch.float32, "nbar_next")
        self._parts_ok(state)
        nbar, dtheta = self._adj_bufs(state, lam_x, lam_v, nbar, dtheta)
        s = state.struct()
        self._check(lib.pic_adjoint_step(self.ctx, C.byref(s), _ptr(node_w),
                                         _ptr(nbar_next) if nbar_next is not None else None,
                                         _ptr(lam_x), _ptr(lam_v), _ptr(nbar), _ptr(dtheta)), "pic_adjoint_step")
        return nbar, dtheta

    def pic_force_vjp(self, state: DeviceParticles, node_w, force_bar, lam_x, nbar=None, dtheta=None):
        self._need(node_w, self.nnodes, torch.int64, "node_w")
        self._need(force_bar, self.grid.ndim * state.n, torch.float32, "force_bar")
        self._parts_ok(state)
        nbar, dtheta = self._adj_bufs(state, lam_x, None, nbar, dtheta)
        s = state.struct()
        self._check(lib.pic_force_vjp(self.ctx, C.byref(s), _ptr(node_w), _ptr(force_bar), _ptr(lam_x),
                                      _ptr(nbar), _ptr(dtheta)), "pic_force_vjp")
        return nbar, dtheta

    def pic_deposit_vjp(self, state: DeviceParticles, nbar, lam_x):
        self._need(nbar, self.nnodes, torch.float32, "nbar")
        self._need(lam_x, self.grid.ndim * state.n, torch.float32, "lam_x")
        self._parts_ok(state)
        s = state.struct()
        self._check(lib.pic_deposit_vjp(self.ctx, C.byref(s), _ptr(nbar), _ptr(lam_x)), "pic_deposit_vjp")

    def _aligned(self, nbytes):
        """A caller-owned device buffer of nbytes, 256-byte aligned: (tensor, ptr)."""
        t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        return t, (t.data_ptr() + 255) // 256 * 256

    def pic_forward_record(self, parts: DeviceParticles, nsteps: int, every: int):
        """nsteps cycles in place with checkpoints every `every` steps; returns
        the record (an opaque device buffer) for pic_backward_record."""
        self._parts_ok(parts)
        nbytes = lib.pic_record_bytes(self.ctx, int(nsteps), int(every))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "recorded runs need a single-slab context on the tiled path")
        buf, ptr = self._aligned(nbytes)
        s = parts.struct()
        self._check(lib.pic_forward_record(self.ctx, C.byref(s), int(nsteps), int(every), C.c_void_p(ptr), nbytes),
                    "pic_forward_record")
        return {"buf": buf, "ptr": ptr, "bytes": nbytes, "nsteps": int(nsteps), "every": int(every)}

    def pic_backward_record(self, parts: DeviceParticles, record, lam_x, lam_v, dtheta=None, start_kick=0.0):
        """Reverse sweep of a recorded run; lam_x and lam_v (caller order) are
        replaced by the initial-state cotangents.  start_kick = f folds in a
        start kick v(-1/2) = v(0) + f F(x0) dt / m (lam_v then is dJ/dv(0)).
        Returns dtheta (+=)."""
        self._parts_ok(parts)
        self._need(lam_x, self.grid.ndim * parts.n, torch.float32, "lam_x")
        self._need(lam_v, 3 * parts.n, torch.float32, "lam_v")
        if dtheta is None:
            dtheta = torch.zeros(NTHETA, dtype=torch.float64, device=self.device)
        self._need(dtheta, NTHETA, torch.float64, "dtheta")
        nbytes = lib.pic_backward_bytes(self.ctx, record["every"])
        scratch, sptr = self._aligned(nbytes)
        s = parts.struct()
        self._check(lib.pic_backward_record(self.ctx, C.byref(s), record["nsteps"], record["every"],
                                            C.c_void_p(record["ptr"]), record["bytes"], C.c_void_p(sptr), nbytes,
                                            _ptr(lam_x), _ptr(lam_v), _ptr(dtheta), float(start_kick)),
                    "pic_backward_record")
        del scratch
        return dtheta

    def start_leapfrog(self, parts: DeviceParticles):
        """v(0) -> v(-1/2) = v(0) - F(0)/m dt/2."""
        node = self.pic_deposit(parts)
        F = self.pic_force(parts, node)
        self.pic_kick(parts, F, -0.5)
        return F


class BatchContext(Context):
    """A pic_ctx_t over several slabs (pic_init_batch / pic_step_batch)."""

    def __init__(self, grids, pot: W.Potential, dt: float, max_n, device="cuda", stream=None):
        self.grids, self.pot, self.dt = list(grids), pot, dt
        self.grid = self.grids[0]
        self.nslab = len(self.grids)
        self.max_ns = [int(m) for m in max_n]
        self.max_n = max(self.max_ns)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        gs = (pic_grid_t * self.nslab)(*[grid_t(g) for g in self.grids])
        mn = (C.c_int64 * self.nslab)(*self.max_ns)
        nbytes = int(lib.pic_workspace_bytes_batch(gs, self.nslab, mn))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "invalid batch")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.ctx = C.c_void_p()
        rc = lib.pic_init_batch(C.byref(self.ctx), gs, self.nslab, C.byref(potential_t(pot)), float(dt), mn,
                                C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream))
        if rc:
            raise PicError(rc, "pic_init_batch failed")
        self.nnodes = sum(pic_num_nodes(g) for g in self.grids)

    def pic_step_batch(self, parts_list, nsteps: int, diag_every: int = 0):
        if len(parts_list) != self.nslab:
            raise ValueError("one particle set per slab")
        for p, m in zip(parts_list, self.max_ns):
            self._parts_ok(p)
            if p.n > m:
                raise ValueError("particle count above the slab's max_n")
        arr = (pic_particles_t * self.nslab)(*[p.struct() for p in parts_list])
        nd = 0 if diag_every <= 0 else (nsteps + diag_every - 1) // diag_every
        buf = (pic_diag_t * max(nd * self.nslab, 1))()
        self._check(lib.pic_step_batch(self.ctx, arr, int(nsteps), buf if nd else None,
                                       int(diag_every) if nd else 0), "pic_step_batch")
        return [[{k: getattr(buf[s * nd + i], k) for k in DIAG_FIELDS} for i in range(nd)]
                for s in range(self.nslab)]
