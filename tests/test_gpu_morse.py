"""GPU parity of the Morse pair potential (PIC_POT_MORSE) against the FP64
oracle, through the C ABI, to the same bars as the Lennard-Jones path:

* one force evaluation: |dF| <= 1e-4 |F| + 1e-5 F_scale (F_scale = 12 D / r0);
  the grid energy of the same deposit (FP64; the library integrates mu with
  a 16-point Gauss-Legendre rule, the oracle adaptively): 1e-9 relative;
* 100 FP32 steps: positions <= 1e-4 cell, velocities <= 1e-4 (relative L2),
  total energy <= 1e-4 at every diagnostic step, 2D and 3D;
* the fused tiled step equals the separate calls bit for bit;
* the host calibration of c_att equals the oracle's;
* the reverse mode of the Morse kind is tested with the Lennard-Jones one
  (test_gpu_adjoint.py, test_gpu_recorded.py).
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
POT = W.morse_cu(c_att=0.4255)


def banner(msg):
    print(f"\n[gpu-case] morse {msg}", flush=True)


def _positions(grid, cell, off):
    c = cell.astype(np.int64)
    out = []
    for d in range(grid.ndim):
        out.append(c % grid.n[d] + off[d].astype(np.float64))
        c //= grid.n[d]
    return np.stack(out)


def _pos_error(grid, ca, oa, cb, ob):
    err = np.abs(_positions(grid, ca, oa) - _positions(grid, cb, ob))
    for d in range(grid.ndim):
        if grid.bc[d] == 0:
            err[d] = np.minimum(err[d], grid.n[d] - err[d])
    return err.max()


def _case(which):
    if which == "slab2d":
        wl = W.cfg_small_slab()
        return wl.grid, wl.parts
    if which == "heated2d":
        return W.make_slab(2, (96, 64), 32, 32, H, 22, fluence_Jcm2=1.0, R_cells=20)
    return W.make_slab(3, (16, 16, 16), 8, 8, H, 21, fluence_Jcm2=1.5, R_cells=200)


@pytest.mark.parametrize("which", ["slab2d", "heated2d", "slab3d"])
def test_morse_force_and_grid_energy_match_oracle(which):
    grid, parts = _case(which)
    for pot in (POT, W.morse_cu(s_rep=2.0, c_att=0.4255)):
        banner(f"force {which} s_rep {pot.s_rep} N={parts.n}")
        ctx = B.Context(grid, pot, DT, parts.n)
        dp = B.DeviceParticles.from_host(parts)
        node = ctx.pic_deposit(dp)
        F, pe = ctx.pic_force(dp, node, want_pe=True)
        F = F.cpu().numpy().astype(np.float64)
        ref = O.forces(grid, pot, parts.cell, parts.off, parts.wq)
        scale = 12 * pot.D / pot.r0
        bad = np.abs(F - ref) > 1e-4 * np.abs(ref) + 1e-5 * scale
        print(f"max |dF|/F_scale = {np.abs(F - ref).max() / scale:.3e}, violations {bad.sum()}")
        assert not bad.any()
        _, _, _, diags = O.run(grid, pot, DT, parts.cell, parts.off, parts.vel, parts.wq, 1, diag_every=1)
        assert pe == pytest.approx(diags[0]["pe"], rel=1e-9, abs=0)


@pytest.mark.parametrize("which", ["slab2d", "heated2d", "slab3d"])
def test_morse_100_steps_match_oracle(which):
    grid, parts = _case(which)
    banner(f"100 steps {which} N={parts.n}")
    ctx = B.Context(grid, POT, DT, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    gd = ctx.pic_step(dp, 100, 10)
    v0 = O.start_leapfrog(grid, POT, DT, parts.cell, parts.off, parts.vel, parts.wq)
    c2, o2, v2, od = O.run(grid, POT, DT, parts.cell, parts.off, v0, parts.wq, 100, diag_every=10)
    cell, off, vel, _ = dp.to_host()
    perr = _pos_error(grid, cell, off, c2, o2)
    verr = np.linalg.norm(vel - v2) / np.linalg.norm(v2)
    E = np.array([d["ke"] + d["pe"] for d in gd])
    Eo = np.array([d["ke"] + d["pe"] for d in od])
    eerr = np.abs(E - Eo).max() / np.abs(Eo).max()
    print(f"position {perr:.3e} cells, velocity {verr:.3e}, energy {eerr:.3e}")
    worst = check_diagnostics(gd, od, parts, POT.mass)
    print(f"momentum {worst['p']:.3e} of sum |w m v|, bond {worst['bond']:.3e}")
    assert perr <= 1e-4 and verr <= 1e-4 and eerr <= 1e-4


def test_morse_fused_step_equals_separate_calls():
    grid, parts = W.make_slab(2, (48, 40), 20, 16, H, 31, fluence_Jcm2=2.0, R_cells=16)
    banner(f"step vs separate calls N={parts.n}")
    ctx = B.Context(grid, POT, DT, parts.n)
    a = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(a)
    b = a.clone()
    ctx.pic_step(a, 25)
    for _ in range(25):
        node = ctx.pic_deposit(b)
        ctx.pic_push(b, ctx.pic_force(b, node))
    ctx.pic_sync()
    for x, y in zip(a.to_host(), b.to_host()):
        assert np.array_equal(x, y)


def test_morse_calibration_matches_oracle():
    grid = W.Grid(ndim=2, n=(4, 64), h=(H, H, H), bc=(0, 1))
    c, w = B.pic_calibrate_catt(grid, W.morse_cu(), W.N_SOLID, 8)
    co, wo, _ = O.calibrate_catt(grid, W.morse_cu(), W.N_SOLID, 8)
    assert c == pytest.approx(co, rel=1e-9, abs=0) and w == pytest.approx(wo, rel=1e-9, abs=0)
