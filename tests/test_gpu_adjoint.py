"""GPU parity of the hand-written reverse mode (pic_force_vjp, pic_deposit_vjp,
pic_adjoint_step) against the differentiable FP64 reference
(oracle/autograd_ref.py, itself pinned to finite differences of the C oracle)
and, for whole gradients, against central finite differences of the FP64 C
oracle stored in tests/golden/adjoint_fd_16cube.json.

Tolerances.  The GPU runs the fixed-point deposit (offsets quantised to 2^-16
cells) and FP32 arithmetic; the reference is the plain FP64 CIC cycle.  The
primal quantities the derivatives are evaluated at therefore differ by about
1e-5 relative (the quantisation of node sums and of the cell-centred
differences built from them), and FP32 rounds every derivative term to 6e-8.
Per-array cotangents are compared element by element against 1e-4 of the
array's largest magnitude (their float-atomic sums carry order noise near
1e-7 relative).  Whole gradients after 400 steps are held to the 1e-4
relative target of finite differences.

Both pair potentials and both neighbour geometries run through the same
tests: Lennard-Jones and Morse (whose width alpha is a fifth parameter; its
FD fixture is tests/golden/adjoint_fd_16cube_morse.json), on the cubic and
the hexagonal close-packed lattice (tests/golden/adjoint_fd_16cube_hcp.json).
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import autograd_ref as R
from paper_1502_07722_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube.json")
GOLDEN_MORSE = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube_morse.json")
GOLDEN_HCP = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube_hcp.json")
GOLDEN_HCP_MORSE = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube_hcp_morse.json")
FREF = 1.5e4
FAMILIES = ["lj", "morse", "hcp", "hcp_morse"]


def _pot(family):
    return {"lj": lambda: W.Potential(c_att=0.27), "morse": lambda: W.morse_cu(c_att=0.43),
            "hcp": lambda: W.hcp(c_att=0.2), "hcp_morse": lambda: W.hcp(W.morse_cu(), c_att=0.3)}[family]()


def _keys(pot):
    return ("D", "r0", "s_rep", "c_att") + (("alpha",) if pot.kind == W.KIND_MORSE else ())


@pytest.fixture(scope="module")
def B():
    from paper_1502_07722_amd import binding
    return binding


def _case(nd):
    if nd == 3:
        wl = W.cfg_adjoint_3d(n=12, layers=6)
        return wl.grid, wl.parts, wl.dt
    grid, parts = W.make_slab(2, (24, 24), 12, 8, W.H_CELL, 21, fluence_Jcm2=1.5, R_cells=12.0)
    return grid, parts, W.DT


def _advance(B, ctx, dp, k):
    for _ in range(k):
        node = ctx.pic_deposit(dp)
        F = ctx.pic_force(dp, node)
        ctx.pic_push(dp, F)
    torch.cuda.synchronize()


def _host(dp):
    from types import SimpleNamespace
    cell, off, vel, wq = dp.to_host()
    return SimpleNamespace(cell=cell, off=off, vel=vel, wq=wq)


def _theta(pot, n):
    """Per-particle parameter leaves: their gradients are each particle's
    contribution, whose absolute sum bounds the rounding of the total."""
    return {k: torch.full((n,), float(getattr(pot, k)), dtype=torch.float64, requires_grad=True)
            for k in _keys(pot)}


def _check_theta(dth, th):
    if "alpha" not in th:
        assert dth[4].item() == 0.0  # no Morse width under Lennard-Jones
    for i, k in enumerate(th):
        t = th[k].grad.numpy()
        ref, l1 = t.sum(), np.abs(t).sum()
        got = dth[i].item()
        assert abs(got - ref) <= 1e-4 * abs(ref) + 2e-5 * l1, (k, got, ref, l1)


def _close(gpu, ref, rel, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref).max()
    assert err <= rel * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def _forces_at(geo, th, pot, idx, f, w, node_w):
    """Reference force with the GPU's exact node sums as values and the plain
    CIC deposit's derivative (straight-through): both sides then evaluate
    eq. (3)'s branch switch at r = r0 and the clamp of eq. (1) on the same
    side.  Solid-density particles sit at rbar ~ r0, right at the branch
    switch, so a 1e-5 difference in the densities would otherwise flip the
    derivative of a few particles."""
    N_cic = R.deposit(geo, idx, f, w)
    N_gpu = torch.as_tensor(node_w.cpu().numpy(), dtype=torch.float64) * R.WUNIT
    N = N_cic + (N_gpu - N_cic.detach())
    dens = R.density(geo, N)
    G = R.centre_gradient(geo, dens)
    n_p, Gp = R.gather(geo, dens, G, idx, f)
    return R.pair_force(th, pot.n_floor, pot.g_clamp, n_p, Gp, hcp=pot.lattice == W.LATTICE_HCP)


def _ref_state(grid, host):
    geo, idx, f = R.unpack(grid, host.cell, host.off)
    f = [t.clone().requires_grad_(True) for t in f]
    return geo, idx, f


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("nd", [2, 3])
def test_force_vjp_matches_autograd(B, nd, family):
    grid, parts, dt = _case(nd)
    pot = _pot(family)
    ctx = B.Context(grid, pot, dt, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    _advance(B, ctx, dp, 10)
    host = _host(dp)
    node = ctx.pic_deposit(dp)
    rng = np.random.default_rng(5)
    fbar = rng.standard_normal((nd, parts.n)).astype(np.float32) * np.float32(1e9)
    lam_x = torch.zeros((nd, parts.n), dtype=torch.float32, device="cuda")
    nbar, dth = ctx.pic_force_vjp(dp, node, torch.from_numpy(fbar).cuda(), lam_x)
    ctx.pic_deposit_vjp(dp, nbar, lam_x)
    ctx.pic_sync()
    geo, idx, f = _ref_state(grid, host)
    th = _theta(pot, parts.n)
    w = torch.as_tensor(host.wq, dtype=torch.float64) * R.WUNIT
    F = _forces_at(geo, th, pot, idx, f, w, node)
    L = sum((F[d] * torch.as_tensor(fbar[d], dtype=torch.float64)).sum() for d in range(nd))
    L.backward()
    for d in range(nd):
        _close(lam_x[d].cpu().numpy(), f[d].grad.numpy(), 1e-4, f"lam_x[{d}]")
    _check_theta(dth, th)


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("nd", [2, 3])
def test_adjoint_step_matches_autograd(B, nd, family):
    grid, parts, dt = _case(nd)
    pot = _pot(family)
    ctx = B.Context(grid, pot, dt, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    _advance(B, ctx, dp, 10)
    host = _host(dp)
    node = ctx.pic_deposit(dp)
    rng = np.random.default_rng(6)
    n, nnodes = parts.n, B.pic_num_nodes(grid)
    lx = rng.standard_normal((nd, n)).astype(np.float32)
    lv = (rng.standard_normal((3, n)) * 1e-3).astype(np.float32)
    nb = rng.standard_normal(nnodes).astype(np.float32)
    lam_x = torch.from_numpy(lx).cuda()
    lam_v = torch.from_numpy(lv).cuda()
    nbar, dth = ctx.pic_adjoint_step(dp, node, torch.from_numpy(nb).cuda(), lam_x, lam_v)
    ctx.pic_deposit_vjp(dp, nbar, lam_x)
    ctx.pic_sync()
    # reference: L = lx . x(n+1) + lv . v(n+1/2) + nb . (n(n+1) r0^3)
    geo, idx, f = _ref_state(grid, host)
    v = [torch.as_tensor(host.vel[d], dtype=torch.float64).requires_grad_(True) for d in range(3)]
    th = _theta(pot, parts.n)
    w = torch.as_tensor(host.wq, dtype=torch.float64) * R.WUNIT
    F = _forces_at(geo, th, pot, idx, f, w, node)
    idx2, f2, v2 = R.push(geo, dt, pot.mass, F, idx, f, v)
    dens2 = R.density(geo, R.deposit(geo, idx2, f2, w)) * pot.r0 ** 3
    L = sum((f2[d] * torch.as_tensor(lx[d], dtype=torch.float64)).sum() for d in range(nd))
    L = L + sum((v2[d] * torch.as_tensor(lv[d], dtype=torch.float64)).sum() for d in range(3))
    L = L + (dens2 * torch.as_tensor(nb, dtype=torch.float64)).sum()
    L.backward()
    for d in range(nd):
        _close(lam_x[d].cpu().numpy(), f[d].grad.numpy(), 1e-4, f"lam_x[{d}]")
    for d in range(3):
        _close(lam_v[d].cpu().numpy(), v[d].grad.numpy(), 1e-4, f"lam_v[{d}]")
    _check_theta(dth, th)


def _per_step_gradient(B, grid, parts, pot, dt, nsteps, y_s, tau):
    """Forward by pic_deposit/pic_force/pic_push with every state kept, then
    the reverse sweep by pic_adjoint_step; the start v(-1/2) = v0 - F0 dt/2m
    and the heating v0 = v_th + sigma sqrt(F/F_ref) xi are reversed here."""
    nd = grid.ndim
    ctx = B.Context(grid, pot, dt, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    v_th = torch.as_tensor(parts.v_thermal, device="cuda")
    xi = torch.as_tensor(parts.xi, device="cuda")
    sig = torch.as_tensor(parts.sigma.astype(np.float32), device="cuda")
    dp.vel.copy_((v_th + sig[None, :] * xi).reshape(dp.vel.shape))
    node0 = ctx.pic_deposit(dp)
    F0 = ctx.pic_force(dp, node0)
    ctx.pic_kick(dp, F0, -0.5)
    states = [dp.clone()]
    for _ in range(nsteps):
        _advance(B, ctx, dp, 1)
        states.append(dp.clone())
    final = _host(states[-1])
    # dJ/d(offset) of J = sum w sigmoid((y - y_s)/tau) on the normal axis
    ax = nd - 1
    cell = final.cell.astype(np.int64)
    lay = cell // int(np.prod(grid.n[:ax]))
    y = (lay + final.off[ax].astype(np.float64)) * grid.h[ax]
    s = 1.0 / (1.0 + np.exp(-(y - y_s) / tau))
    w = final.wq.astype(np.float64) * 2.0 ** -20
    J = float((w * s).sum())
    lam_x = torch.zeros((nd, parts.n), dtype=torch.float32, device="cuda")
    lam_x[ax] = torch.from_numpy((w * s * (1 - s) * grid.h[ax] / tau).astype(np.float32)).cuda()
    lam_v = torch.zeros((3, parts.n), dtype=torch.float32, device="cuda")
    dth = torch.zeros(B.NTHETA, dtype=torch.float64, device="cuda")
    nbar_next = None
    for k in range(nsteps - 1, -1, -1):
        node = ctx.pic_deposit(states[k])
        nbar, _ = ctx.pic_adjoint_step(states[k], node, nbar_next, lam_x, lam_v, dtheta=dth)
        nbar_next = nbar.clone()
    # start: v(-1/2) = v0 - (dt / 2m) F(x0): force cotangent -dt/(2m) lam_v
    fbar = (lam_v[:nd] * (-0.5 * dt / pot.mass)).contiguous()
    lam_x0 = torch.zeros_like(lam_x)
    ctx.pic_force_vjp(states[0], node0, fbar, lam_x0, dtheta=dth)
    ctx.pic_sync()
    # heating: dv0/dF = sigma xi / (2 F) at F = F_ref
    dF = float((lam_v.double() * (sig.double()[None, :] * xi.double()) / (2 * FREF)).sum().item())
    return J, dth.cpu().numpy(), dF


def test_whole_gradient_matches_oracle_finite_differences(B):
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    wl = W.cfg_adjoint_3d(n=16, layers=8)
    grid, parts = wl.grid, wl.parts
    assert parts.n == gold["particles"]
    nsteps, y_s, tau = gold["nsteps"], gold["y_s"], gold["tau"]
    alt = gold["potentials"]["altered"]
    pot = W.Potential(c_att=alt["c_att"])
    J, dth, dF = _per_step_gradient(B, grid, parts, pot, wl.dt, nsteps, y_s, tau)
    assert abs(J - alt["J"]) <= 1e-5 * abs(alt["J"]), (J, alt["J"])
    got = {"D": dth[0], "s_rep": dth[2], "c_att": dth[3], "F": dF}
    for k, v in got.items():
        fd = alt["dJ"][k]["0.0001"]
        fd_err = abs(alt["dJ"][k]["0.001"] - fd)
        print(f"dJ/d{k}: adjoint {v:.9e} finite difference {fd:.9e} rel {abs(v - fd) / abs(fd):.2e}")
        assert abs(v - fd) <= 1e-4 * abs(fd) + fd_err, (k, v, fd, fd_err)
    un = gold["potentials"]["unaltered"]
    pot1 = W.Potential(c_att=un["c_att"])
    _, dth1, _ = _per_step_gradient(B, grid, parts, pot1, wl.dt, nsteps, y_s, tau)
    fd = un["dJ"]["r0"]["0.0001"]
    fd_err = abs(un["dJ"]["r0"]["0.001"] - fd)
    print(f"dJ/dr0: adjoint {dth1[1]:.9e} finite difference {fd:.9e} rel {abs(dth1[1] - fd) / abs(fd):.2e}")
    assert abs(dth1[1] - fd) <= 1e-4 * abs(fd) + fd_err, (dth1[1], fd, fd_err)


def test_whole_morse_gradient_matches_oracle_finite_differences(B):
    """The same 400-step sweep with the Morse potential, alpha included."""
    with open(GOLDEN_MORSE) as fh:
        gold = json.load(fh)
    wl = W.cfg_adjoint_3d(n=16, layers=8)
    grid, parts = wl.grid, wl.parts
    assert parts.n == gold["particles"]
    nsteps, y_s, tau = gold["nsteps"], gold["y_s"], gold["tau"]
    for name, keys in (("altered", ("D", "s_rep", "c_att", "alpha", "F")), ("unaltered", ("r0",))):
        rec = gold["potentials"][name]
        pot = W.morse_cu(c_att=rec["c_att"])
        assert pot.alpha == rec["alpha"] and pot.D == rec["D"]
        J, dth, dF = _per_step_gradient(B, grid, parts, pot, wl.dt, nsteps, y_s, tau)
        assert abs(J - rec["J"]) <= 1e-5 * abs(rec["J"]), (J, rec["J"])
        got = dict(zip(("D", "r0", "s_rep", "c_att", "alpha"), dth))
        got["F"] = dF
        for k in keys:
            fd = rec["dJ"][k]["0.0001"]
            fd_err = abs(rec["dJ"][k]["0.001"] - fd)
            print(f"[{name}] dJ/d{k}: adjoint {got[k]:.9e} finite difference {fd:.9e} "
                  f"rel {abs(got[k] - fd) / abs(fd):.2e}")
            assert abs(got[k] - fd) <= 1e-4 * abs(fd) + fd_err, (k, got[k], fd, fd_err)


@pytest.mark.parametrize("kind", ["lj", "morse"])
def test_whole_hcp_gradient_matches_oracle_finite_differences(B, kind):
    """The same 400-step sweep on the hexagonal close-packed lattice, with the
    Lennard-Jones and with the Morse potential (alpha included)."""
    with open(GOLDEN_HCP if kind == "lj" else GOLDEN_HCP_MORSE) as fh:
        gold = json.load(fh)
    wl = W.cfg_adjoint_3d(n=16, layers=8)
    grid, parts = wl.grid, wl.parts
    nsteps, y_s, tau = gold["nsteps"], gold["y_s"], gold["tau"]
    extra = ("alpha",) if kind == "morse" else ()
    for name, keys in (("altered", ("D", "s_rep", "c_att", "F") + extra), ("unaltered", ("r0",))):
        rec = gold["potentials"][name]
        pot = W.hcp(None if kind == "lj" else W.morse_cu(), c_att=rec["c_att"])
        assert pot.r0 == rec["r0"] and rec["lattice"] == W.LATTICE_HCP
        J, dth, dF = _per_step_gradient(B, grid, parts, pot, wl.dt, nsteps, y_s, tau)
        assert abs(J - rec["J"]) <= 1e-5 * abs(rec["J"]), (J, rec["J"])
        got = dict(zip(("D", "r0", "s_rep", "c_att", "alpha"), dth))
        got["F"] = dF
        for k in keys:
            fd = rec["dJ"][k]["0.0001"]
            fd_err = abs(rec["dJ"][k]["0.001"] - fd)
            print(f"[{name}] dJ/d{k}: adjoint {got[k]:.9e} finite difference {fd:.9e} "
                  f"rel {abs(got[k] - fd) / abs(fd):.2e}")
            assert abs(got[k] - fd) <= 1e-4 * abs(fd) + fd_err, (k, got[k], fd, fd_err)
