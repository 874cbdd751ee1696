"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Bars (derivations in the design notes):
  - node sums: bit-exact (int64 fixed point, identical inputs);
  - forces, one evaluation on identical inputs: |dF| <= 1e-4 |F| + 1e-5 F_scale,
    F_scale = 12 D / r0.  The floor comes from FP32 cancellation in
    phi'(s+) - phi'(s-): each term s^7 - s^13 carries about 6 x 4 ulp of
    absolute error near s = 1, i.e. ~1.5e-6 each, ~3e-6 for the pair (measured
    3.9e-6 at most); the floor keeps a 2.5x margin;
  - after 100 FP32 steps: max position error <= 1e-4 cell, relative L2
    velocity error <= 1e-4, relative total-energy error <= 1e-4 at every
    diagnostic step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1502_07722_amd import binding as B  # noqa: E402
from paper_1502_07722_amd import workloads as W  # noqa: E402
from parity_util import check_diagnostics  # noqa: E402

DT = 1e-15
H = W.H_CELL


def banner(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def positions(grid, cell, off):
    """Continuous coordinates in cell units, [ndim, N]."""
    c = cell.astype(np.int64)
    out = []
    for d in range(grid.ndim):
        out.append(c % grid.n[d] + off[d].astype(np.float64))
        c //= grid.n[d]
    return np.stack(out)


def pos_error(grid, cell_a, off_a, cell_b, off_b):
    xa, xb = positions(grid, cell_a, off_a), positions(grid, cell_b, off_b)
    err = np.abs(xa - xb)
    for d in range(grid.ndim):
        if grid.bc[d] == 0:  # periodic: distance on the circle
            err[d] = np.minimum(err[d], grid.n[d] - err[d])
    return err.max() if err.size else 0.0


def random_particles(grid, N, seed, edge=True):
    rng = np.random.default_rng(seed)
    cell = rng.integers(0, grid.ncells, N).astype(np.int32)
    off = rng.random((grid.ndim, N), dtype=np.float32)
    if edge and N >= 16:
        off[:, :4] = 0.0
        off[:, 4:8] = np.float32(np.nextafter(np.float32(1), np.float32(0)))
        off[:, 8:12] = 0.5
        off[:, 12:16] = np.float32(1.0 - 2.0 ** -16)
    vel = (rng.standard_normal((3, N)) * 300.0).astype(np.float32)
    wq = rng.integers(0, (1 << 31) - 1, N).astype(np.int32)
    wq[: min(N, 3)] = [(1 << 31) - 1, 0, 1][: min(N, 3)]
    return W.Particles(cell=cell, off=off, vel=vel, wq=wq)


# ------------------------------------------------------------------ deposit
DEPOSIT_CASES = [
    ("slab2d_64x64_16ppc", None),
    ("2d_ragged_reflect_all", (W.Grid(ndim=2, n=(37, 29), h=(H, 1.3 * H), bc=(1, 1)), 100_003)),
    ("2d_periodic", (W.Grid(ndim=2, n=(64, 17), h=(H, H), bc=(0, 0)), 65_537)),
    ("3d_ragged", (W.Grid(ndim=3, n=(13, 11, 9), h=(H, H, 0.8 * H), bc=(0, 0, 1)), 77_777)),
    ("3d_reflect_all", (W.Grid(ndim=3, n=(6, 7, 8), h=(H, H, H), bc=(1, 1, 1)), 4_097)),
    ("single", (W.Grid(ndim=2, n=(5, 5), h=(H, H), bc=(0, 1)), 1)),
]


@pytest.mark.parametrize("name,case", DEPOSIT_CASES, ids=[c[0] for c in DEPOSIT_CASES])
def test_deposit_bit_exact(name, case):
    if case is None:
        wl = W.cfg_small_slab()
        grid, parts = wl.grid, wl.parts
    else:
        grid, N = case
        parts = random_particles(grid, N, seed=N)
    banner(f"deposit {name} N={parts.n}")
    ctx = B.Context(grid, W.Potential(), DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    got = ctx.pic_deposit(dp).cpu().numpy()
    ref = O.deposit(grid, parts.cell, parts.off, parts.wq)
    assert got.dtype == np.int64 and np.array_equal(got, ref)
    ctx.pic_sync()


def test_deposit_empty_input_zeroes_the_grid():
    grid = W.Grid(ndim=2, n=(16, 8), h=(H, H), bc=(0, 1))
    ctx = B.Context(grid, W.Potential(), DT, 10)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    dp = B.DeviceParticles(e, torch.empty((2, 0), device="cuda"), torch.empty((3, 0), device="cuda"), e.clone())
    node = torch.full((B.pic_num_nodes(grid),), 7, dtype=torch.int64, device="cuda")
    ctx.pic_deposit(dp, node)
    assert int(node.abs().sum()) == 0
    ctx.pic_step(dp, 3)


@pytest.mark.parametrize("ndim", [2, 3])
def test_empty_input_on_the_tiled_path(ndim):
    """No particles on a grid large enough for the tiled path: the fused
    step, the graph replay, the recorded forward and the reverse sweep run
    and leave the node sums zero and dtheta zero."""
    grid = (W.Grid(ndim=2, n=(64, 64), h=(H, H), bc=(0, 1)) if ndim == 2
            else W.Grid(ndim=3, n=(16, 16, 16), h=(H, H, H), bc=(0, 0, 1)))
    banner(f"empty tiled {ndim}D")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = B.Context(grid, W.Potential(c_att=0.27), DT, 100, stream=stream)
        assert ctx.pic_get_tiling()[0] > 0  # the tiled path
        e = torch.empty(0, dtype=torch.int32, device="cuda")
        dp = B.DeviceParticles(e, torch.empty((ndim, 0), device="cuda"), torch.empty((3, 0), device="cuda"),
                               e.clone())
        diags = ctx.pic_step(dp, 13, 5)
        assert [d["wsum"] for d in diags] == [0.0, 0.0, 0.0]
        assert int(ctx.pic_step_nodes().abs().sum()) == 0
        rec = ctx.pic_forward_record(dp, 12, 4)
        lam_x = torch.zeros((ndim, 0), device="cuda")
        lam_v = torch.zeros((3, 0), device="cuda")
        dth = ctx.pic_backward_record(dp, rec, lam_x, lam_v)
    stream.synchronize()
    assert torch.count_nonzero(dth).item() == 0


# ------------------------------------------------------------------ force / push, one evaluation
def force_tolerance(F_ref, pot):
    return 1e-4 * np.abs(F_ref) + 1e-5 * 12 * pot.D / pot.r0


@pytest.mark.parametrize("which", ["slab2d", "slab3d", "heated2d"])
def test_force_matches_oracle(which):
    pot = W.Potential(c_att=0.27, s_rep=1.0)
    if which == "slab2d":
        grid, parts = W.cfg_small_slab().grid, W.cfg_small_slab().parts
    elif which == "slab3d":
        grid, parts = W.make_slab(3, (16, 16, 16), 8, 8, H, 21)
    else:
        grid, parts = W.make_slab(2, (96, 64), 32, 32, H, 22, fluence_Jcm2=1.0, R_cells=20)
    banner(f"force {which} N={parts.n}")
    ctx = B.Context(grid, pot, DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    node = ctx.pic_deposit(dp)
    F, pe = ctx.pic_force(dp, node, want_pe=True)
    F = F.cpu().numpy().astype(np.float64)
    ref = O.forces(grid, pot, parts.cell, parts.off, parts.wq)
    tol = force_tolerance(ref, pot)
    bad = np.abs(F - ref) > tol
    print(f"max |dF|/F_scale = {np.abs(F - ref).max() / (12 * pot.D / pot.r0):.3e}, violations {bad.sum()}")
    assert not bad.any()
    # grid energy of the same deposit (the oracle's step-0 diagnostic)
    _, _, _, diags = O.run(grid, pot, DT, parts.cell, parts.off, parts.vel, parts.wq, 1, diag_every=1)
    assert pe == pytest.approx(diags[0]["pe"], rel=1e-12, abs=0)


def test_push_and_kick_match_oracle():
    pot = W.Potential(c_att=0.27)
    wl = W.cfg_small_slab()
    grid, parts = wl.grid, wl.parts
    banner(f"push small slab N={parts.n}")
    ctx = B.Context(grid, pot, DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    node = ctx.pic_deposit(dp)
    F = ctx.pic_force(dp, node)
    F = F * 40.0  # larger kicks so cell crossings happen
    Fh = F.cpu().numpy().astype(np.float64)
    ctx.pic_push(dp, F)
    ctx.pic_sync()
    cell, off, vel, _ = dp.to_host()
    ref_cell, ref_off, ref_vel = [], [], []
    for i in range(0, parts.n, 97):
        c, f, v = O.push_one(grid, pot, DT, Fh[:, i], parts.cell[i], parts.off[:, i].astype(np.float64),
                             parts.vel[:, i].astype(np.float64))
        ref_cell.append(c)
        ref_off.append(f)
        ref_vel.append(v)
    sel = np.arange(0, parts.n, 97)
    assert pos_error(grid, cell[sel], off[:, sel], np.array(ref_cell), np.array(ref_off).T) < 1e-6
    assert np.allclose(vel[:, sel], np.array(ref_vel).T, rtol=1e-6, atol=1e-4)
    v_before = torch.from_numpy(vel).cuda()
    ctx.pic_kick(dp, F, -0.5)
    dv = (dp.vel - v_before).cpu().numpy()[:2]
    # float velocities near 300 m/s carry 3e-5 m/s ulps, hence the absolute floor
    assert np.allclose(dv, -0.5 * Fh / pot.mass * DT, rtol=1e-5, atol=1e-4)


# ------------------------------------------------------------------ trajectories
def run_both(grid, parts, pot, nsteps, diag_every):
    ctx = B.Context(grid, pot, DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    gd = ctx.pic_step(dp, nsteps, diag_every)
    v0 = O.start_leapfrog(grid, pot, DT, parts.cell, parts.off, parts.vel, parts.wq)
    c2, o2, v2, od = O.run(grid, pot, DT, parts.cell, parts.off, v0, parts.wq, nsteps, diag_every=diag_every)
    return dp.to_host(), (c2, o2, v2), gd, od


@pytest.mark.parametrize("which", ["slab2d_64x64_16ppc", "heated2d", "slab3d"])
def test_100_steps_match_oracle(which):
    pot = W.Potential(c_att=0.27)
    if which == "slab2d_64x64_16ppc":
        wl = W.cfg_small_slab()
        grid, parts = wl.grid, wl.parts
    elif which == "heated2d":
        grid, parts = W.make_slab(2, (96, 64), 32, 32, H, 22, fluence_Jcm2=1.0, R_cells=20)
    else:
        grid, parts = W.make_slab(3, (16, 16, 16), 8, 8, H, 21, fluence_Jcm2=1.5, R_cells=200)
    banner(f"100 steps {which} N={parts.n}")
    (cell, off, vel, _), (c2, o2, v2), gd, od = run_both(grid, parts, pot, 100, 10)
    perr = pos_error(grid, cell, off, c2, o2)
    verr = np.linalg.norm(vel - v2) / np.linalg.norm(v2)
    E = np.array([d["ke"] + d["pe"] for d in gd])
    Eo = np.array([d["ke"] + d["pe"] for d in od])
    eerr = np.abs(E - Eo).max() / np.abs(Eo).max()
    kerr = max(abs(a["ke"] - b["ke"]) / abs(b["ke"]) for a, b in zip(gd, od))
    print(f"position {perr:.3e} cells, velocity {verr:.3e}, energy {eerr:.3e}, KE {kerr:.3e}")
    worst = check_diagnostics(gd, od, parts, pot.mass)
    print(f"momentum {worst['p']:.3e} of sum |w m v|, bond {worst['bond']:.3e}")
    assert perr <= 1e-4 and verr <= 1e-4 and eerr <= 1e-4
    for a, b in zip(gd, od):
        assert a["wsum"] == pytest.approx(b["wsum"], rel=1e-12, abs=0)
        assert a["pe"] == pytest.approx(b["pe"], rel=1e-4, abs=0)


def test_step_is_bit_identical_to_separate_calls():
    pot = W.Potential(c_att=0.27)
    grid, parts = W.make_slab(2, (48, 40), 20, 16, H, 31, fluence_Jcm2=2.0, R_cells=16)
    banner(f"step vs separate calls N={parts.n}")
    ctx = B.Context(grid, pot, DT, parts.n)
    a = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(a)
    b = a.clone()
    ctx.pic_step(a, 25)
    for _ in range(25):
        node = ctx.pic_deposit(b)
        F = ctx.pic_force(b, node)
        ctx.pic_push(b, F)
    ctx.pic_sync()
    for x, y in zip(a.to_host(), b.to_host()):
        assert np.array_equal(x, y)


def _run_config(grid, parts, pot, nsteps, tiling=None, untiled=False, diag_every=0):
    """tiling: (tile, halo, chunk, sort_every) or (tile, tile_last, halo,
    chunk, sort_every)."""
    ctx = B.Context(grid, pot, DT, parts.n)
    if tiling and len(tiling) == 5:
        ctx.pic_set_tile_shape(*tiling)
    elif tiling:
        ctx.pic_set_tiling(*tiling)
    ctx.pic_set_path(untiled)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    diags = ctx.pic_step(dp, nsteps, diag_every)
    nodes = None if untiled else ctx.pic_step_nodes().cpu().numpy()
    return dp, diags, nodes, ctx


@pytest.mark.parametrize("ndim", [2, 3])
def test_tiled_step_is_bit_identical_to_untiled_and_to_any_tiling(ndim):
    """Node sums are exact integers and every particle is updated from its own
    state, so the fused tiled step, the untiled kernels, and every tiling /
    binning period must give the same bits -- including particles that drift
    out of their tile window (halo 1, never re-binned: the global path)."""
    pot = W.Potential(c_att=0.27)
    if ndim == 2:
        grid, parts = W.make_slab(2, (80, 72), 36, 24, H, 51, fluence_Jcm2=4.0, R_cells=20)
        tilings = [(16, 2, 8192, 32), (8, 1, 1024, 0), (32, 3, 4096, 7), (32, 8, 2, 2048, 9)]
    else:
        grid, parts = W.make_slab(3, (20, 18, 24), 12, 8, H, 52, fluence_Jcm2=4.0, R_cells=10)
        tilings = [(8, 1, 4096, 16), (4, 1, 1024, 0), (4, 2, 2048, 3), (8, 4, 1, 1024, 0), (8, 4, 2, 4096, 5)]
    nsteps = 60
    banner(f"tiled vs untiled {ndim}D N={parts.n}")
    ref, _, _, _ = _run_config(grid, parts, pot, nsteps, untiled=True)
    ref_h = ref.to_host()
    for t in tilings:
        banner(f"tiling {t}")
        dp, _, nodes, ctx = _run_config(grid, parts, pot, nsteps, tiling=t)
        for x, y in zip(dp.to_host(), ref_h):
            assert np.array_equal(x, y), f"tiling {t} differs"
        # the fused kernel's own deposit of the final positions
        assert np.array_equal(nodes, ctx.pic_deposit(dp).cpu().numpy())


@pytest.mark.parametrize("ndim", [2, 3])
def test_many_drifters_per_item_match_untiled(ndim):
    """A uniform drift of 0.4 cells per step along the periodic x axis with
    re-binning off: after a few steps most particles of every work item lie
    outside their tile window, several 256-particle rounds of drifters per
    item, which the fused step advances through the global node sums at the
    end of the item.  Positions, velocities, cells and node sums must still
    be the untiled path's bits, and the diagnostics its values."""
    import dataclasses
    pot = W.Potential(c_att=0.27)
    if ndim == 2:
        grid, parts = W.make_slab(2, (64, 48), 20, 24, H, 61, fluence_Jcm2=2.0, R_cells=16)
        tiling = (8, 1, 1024, 0)
    else:
        grid, parts = W.make_slab(3, (16, 16, 20), 10, 8, H, 62, fluence_Jcm2=2.0, R_cells=8)
        tiling = (4, 1, 512, 0)
    vel = parts.vel.copy()
    vel[0] += np.float32(0.4 * H / DT)
    parts = dataclasses.replace(parts, vel=vel)
    nsteps = 15
    banner(f"many drifters {ndim}D N={parts.n}")
    ref, d_ref, _, _ = _run_config(grid, parts, pot, nsteps, untiled=True, diag_every=5)
    ctx = B.Context(grid, pot, DT, parts.n)
    ctx.pic_set_tiling(*tiling)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    ctx.pic_set_timing(True)
    d_t = ctx.pic_step(dp, nsteps, 5)
    timing = ctx.pic_get_timing()
    ctx.pic_set_timing(False)
    nodes = ctx.pic_step_nodes().cpu().numpy()
    assert timing["drifters_last"] > 0.5 * parts.n, timing
    assert timing["drifters_last"] > 256 * timing["items_last"] // 2, timing
    for x, y in zip(dp.to_host(), ref.to_host()):
        assert np.array_equal(x, y)
    assert np.array_equal(nodes, ctx.pic_deposit(dp).cpu().numpy())
    assert len(d_ref) == len(d_t)
    for a, b in zip(d_ref, d_t):
        for k in ("ke", "pe", "px", "py", "pz", "wsum", "bond"):
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-30), k


def test_tiled_diagnostics_match_untiled():
    pot = W.Potential(c_att=0.27)
    grid, parts = W.make_slab(2, (64, 48), 24, 16, H, 53, fluence_Jcm2=2.0, R_cells=12)
    banner(f"tiled diagnostics N={parts.n}")
    _, d_ref, _, _ = _run_config(grid, parts, pot, 40, untiled=True, diag_every=10)
    _, d_t, _, _ = _run_config(grid, parts, pot, 40, diag_every=10)
    assert len(d_ref) == len(d_t) == 4
    for a, b in zip(d_ref, d_t):
        for k in ("ke", "pe", "px", "py", "pz", "wsum", "bond"):
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-30), k


def test_step_is_deterministic_and_lattice_is_static():
    grid, parts = W.make_lattice(2, (32, 32), 3, H)
    banner("lattice static")
    ctx = B.Context(grid, W.Potential(), DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    node = ctx.pic_deposit(dp)
    F = ctx.pic_force(dp, node)
    assert float(F.abs().max()) == 0.0
    ctx.pic_step(dp, 50)
    cell, off, vel, _ = dp.to_host()
    assert np.array_equal(cell, parts.cell) and np.array_equal(off, parts.off) and not vel.any()
    grid, parts = W.make_slab(2, (40, 40), 20, 16, H, 41, fluence_Jcm2=1.0, R_cells=10)
    runs = []
    for _ in range(2):
        dp = B.DeviceParticles.from_host(parts)
        ctx2 = B.Context(grid, W.Potential(), DT, parts.n)
        diags = ctx2.pic_step(dp, 30, 10)
        runs.append((dp.to_host(), diags))
    for x, y in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(x, y)
    for a, b in zip(runs[0][1], runs[1][1]):  # FP64 sums: order of binned particles may differ
        for k in ("ke", "pe", "px", "py", "pz", "wsum", "bond"):
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-30)


# ------------------------------------------------------------------ device errors
def test_device_errors_are_reported():
    grid = W.Grid(ndim=2, n=(16, 16), h=(H, H), bc=(0, 1))
    parts = random_particles(grid, 1000, 5, edge=False)
    parts.wq[:] = 1 << 20
    ctx = B.Context(grid, W.Potential(), DT, parts.n)
    banner("device error: CFL")
    bad = W.Particles(parts.cell.copy(), parts.off.copy(), parts.vel.copy(), parts.wq.copy())
    bad.vel[0, 17] = 3.0e6  # 1.5 cells per step
    dp = B.DeviceParticles.from_host(bad)
    with pytest.raises(B.PicError) as e:
        ctx.pic_step(dp, 2)
    assert e.value.code == B.PIC_ECFL
    banner("device error: cell out of range")
    bad = W.Particles(parts.cell.copy(), parts.off.copy(), parts.vel.copy(), parts.wq.copy())
    bad.cell[5] = grid.ncells + 3
    dp = B.DeviceParticles.from_host(bad)
    ctx.pic_deposit(dp)
    with pytest.raises(B.PicError) as e:
        ctx.pic_sync()
    assert e.value.code == B.PIC_ERANGE
    banner("device error: negative weight")
    bad = W.Particles(parts.cell.copy(), parts.off.copy(), parts.vel.copy(), parts.wq.copy())
    bad.wq[9] = -5
    dp = B.DeviceParticles.from_host(bad)
    with pytest.raises(B.PicError) as e:
        ctx.pic_step(dp, 1)
    assert e.value.code == B.PIC_EOVERFLOW
    # the error word was cleared: a clean run passes again
    ctx.pic_step(B.DeviceParticles.from_host(parts), 2)


def test_tile_shape_checks_keep_the_previous_tiling():
    grid = W.Grid(ndim=3, n=(24, 24, 24), h=(H, H, H), bc=(0, 0, 1))
    parts = random_particles(grid, 2000, 7, edge=False)
    ctx = B.Context(grid, W.Potential(), DT, parts.n)
    ctx.pic_set_tile_shape(8, 4, 1, 2048, -1)
    assert ctx.pic_get_tile_shape() == (8, 4) and ctx.pic_get_tiling()[:3] == (8, 1, 2048)
    for bad in ((8, 16, 1, 2048, -1),   # longer along the last axis
                (8, 2, 1, 2048, -1),    # below the smallest 3D edge
                (8, 6, 1, 2048, -1),    # not a power of two
                (16, 8, 1, 2048, -1)):  # window beyond LDS / the tile range
        with pytest.raises(B.PicError) as e:
            ctx.pic_set_tile_shape(*bad)
        assert e.value.code == B.PIC_EINVAL, bad
        assert ctx.pic_get_tile_shape() == (8, 4) and ctx.pic_get_tiling()[:3] == (8, 1, 2048)
    ctx.pic_set_tiling(4, 1, 1024, 0)
    assert ctx.pic_get_tile_shape() == (4, 4)


def test_binding_refuses_undersized_buffers():
    grid = W.Grid(ndim=2, n=(16, 16), h=(H, H), bc=(0, 1))
    parts = random_particles(grid, 100, 6, edge=False)
    ctx = B.Context(grid, W.Potential(), DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    with pytest.raises(ValueError):
        ctx.pic_deposit(dp, torch.empty(10, dtype=torch.int64, device="cuda"))
    node = ctx.pic_deposit(dp)
    with pytest.raises(ValueError):
        ctx.pic_force(dp, node, torch.empty((2, 5), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        ctx.pic_push(dp, torch.empty((2, 5), dtype=torch.float32, device="cuda"))


# ------------------------------------------------------------------ batches and graphs
def _sweep(scale=0.1, nslab=6):
    wls = W.cfg_sweep(nslab=nslab, scale=scale)
    return [(w.grid, w.parts) for w in wls]


@pytest.mark.parametrize("variant", ["lj", "morse_hcp"])
def test_batched_step_is_bit_identical_to_each_slab_alone(variant):
    """Slabs of uneven size advanced in one batched context (persistent
    launches over all slabs' items) give every slab exactly the bits it gets
    alone; per-slab diagnostics agree to FP64 summation order.  Also with the
    general kernels (Morse on the hexagonal lattice)."""
    pot = W.Potential(c_att=0.27) if variant == "lj" else W.hcp(W.morse_cu(), c_att=0.3)
    slabs = _sweep()
    banner(f"batch of {len(slabs)} slabs, N={[p.n for _, p in slabs]}")
    alone = []
    for grid, parts in slabs:
        ctx = B.Context(grid, pot, DT, parts.n)
        dp = B.DeviceParticles.from_host(parts)
        diags = ctx.pic_step(dp, 30, 10)
        alone.append((dp.to_host(), diags))
    bctx = B.BatchContext([g for g, _ in slabs], pot, DT, [p.n for _, p in slabs])
    dps = [B.DeviceParticles.from_host(p) for _, p in slabs]
    bd = bctx.pic_step_batch(dps, 30, 10)
    for k, (dp, (ref, rdiag)) in enumerate(zip(dps, alone)):
        for x, y in zip(dp.to_host(), ref):
            assert np.array_equal(x, y), f"slab {k}"
        assert len(bd[k]) == len(rdiag) == 3
        for a, b in zip(bd[k], rdiag):
            for f in ("ke", "pe", "px", "py", "pz", "wsum", "bond"):
                assert a[f] == pytest.approx(b[f], rel=1e-12, abs=1e-30), (k, f)


@pytest.mark.parametrize("variant", ["lj", "morse_hcp"])
def test_graph_replay_matches_eager_launches(variant):
    """Graph replays of 6-step blocks, interleaved with eager diagnostic steps
    and several pic_step calls (host syncs in between), reproduce the eager
    launches bit for bit on a created stream (also with the general kernels:
    Morse on the hexagonal lattice)."""
    pot = W.Potential(c_att=0.27) if variant == "lj" else W.hcp(W.morse_cu(), c_att=0.3)
    grid, parts = W.make_slab(2, (96, 64), 32, 16, H, 61, fluence_Jcm2=2.0, R_cells=20)
    stream = torch.cuda.Stream()
    banner(f"graph replay N={parts.n}")
    out = []
    for graph in (False, True):
        with torch.cuda.stream(stream):
            ctx = B.Context(grid, pot, DT, parts.n, stream=stream)
            ctx.pic_set_graph(graph)
            dp = B.DeviceParticles.from_host(parts)
            diags = []
            for _ in range(4):
                diags += ctx.pic_step(dp, 37, 10)
            stream.synchronize()
            out.append((dp.to_host(), diags))
    for x, y in zip(out[0][0], out[1][0]):
        assert np.array_equal(x, y)
    for a, b in zip(out[0][1], out[1][1]):
        assert a["ke"] == pytest.approx(b["ke"], rel=1e-12, abs=0)


def test_autotune_reads_only_and_keeps_results_identical():
    pot = W.Potential(c_att=0.27)
    grid, parts = W.make_slab(2, (96, 64), 32, 16, H, 71, fluence_Jcm2=1.0, R_cells=20)
    banner(f"autotune N={parts.n}")
    ctx = B.Context(grid, pot, DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    before = dp.to_host()
    tuning = ctx.pic_autotune(dp, 4)
    for x, y in zip(dp.to_host(), before):
        assert np.array_equal(x, y)  # probes never write the caller's arrays
    assert tuning["candidates"] >= 4 and tuning["tile"] in (8, 16, 32)
    assert ctx.pic_get_tiling()[:3] == (tuning["tile"], tuning["halo"], tuning["chunk"])
    assert ctx.pic_get_tile_shape() == (tuning["tile"], tuning["tile_last"])
    ctx.pic_step(dp, 20)
    ref_ctx = B.Context(grid, pot, DT, parts.n)
    ref = B.DeviceParticles.from_host(parts)
    ref_ctx.pic_set_path(True)
    ref_ctx.pic_step(ref, 20)
    for x, y in zip(dp.to_host(), ref.to_host()):
        assert np.array_equal(x, y)
