"""GPU tests of the recorded reverse sweep (pic_forward_record /
pic_backward_record) and of the torch.autograd Functions built on it.

* The recorded forward produces the same bits as pic_step.
* The recorded sweep (checkpoints, out-of-place recompute, tiled reverse
  kernel) agrees with the chain of per-step pic_adjoint_step calls on caller
  arrays, which the adjoint parity tests pin to the FP64 references; the two
  differ only in the order of float atomic sums (nodes, centres, parameter
  partials), hence 1e-4 of each array's largest magnitude and 1e-5 relative
  on dtheta.
* The autograd crater gradient on the 16^3, 400-step case with checkpoints
  every 20 steps matches central finite differences of the FP64 C oracle
  (tests/golden/adjoint_fd_16cube.json) within the 1e-4 target; with the
  Morse potential, alpha included, against adjoint_fd_16cube_morse.json; on
  the hexagonal close-packed lattice against adjoint_fd_16cube_hcp.json.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1502_07722_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube.json")
GOLDEN_MORSE = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube_morse.json")
GOLDEN_HCP = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd_16cube_hcp.json")


@pytest.fixture(scope="module")
def B():
    from paper_1502_07722_amd import binding
    return binding


def _case(nd):
    if nd == 3:
        wl = W.cfg_adjoint_3d(n=16, layers=8)
        return wl.grid, wl.parts, wl.dt
    grid, parts = W.make_slab(2, (64, 48), 24, 12, W.H_CELL, 31, fluence_Jcm2=3.0, R_cells=20.0)
    return grid, parts, W.DT


def _seed_cotangents(grid, dp):
    """dJ/d(offset) of the crater functional at the state in dp."""
    nd = grid.ndim
    ax = nd - 1
    lateral = int(np.prod(grid.n[:ax]))
    cell = dp.cell.long()
    y = (torch.div(cell, lateral, rounding_mode="floor").double() + dp.off[ax].double()) * grid.h[ax]
    y_s = (grid.n[ax] // 2) * grid.h[ax]
    s = torch.sigmoid((y - y_s) / grid.h[ax])
    w = dp.wq.double() * 2.0 ** -20
    lam_x = torch.zeros_like(dp.off)
    lam_x[ax] = (w * s * (1 - s)).float()
    lam_v = torch.zeros_like(dp.vel)
    return lam_x, lam_v


@pytest.mark.parametrize("nd,all_states", [(2, False), (3, False), (2, True), (3, True)])
def test_recorded_forward_equals_pic_step(B, nd, all_states):
    """all_states: the record keeps every state (each step writes its output
    into the record) instead of checkpoints only."""
    grid, parts, dt = _case(nd)
    pot = W.Potential(c_att=0.27)
    ctx = B.Context(grid, pot, dt, parts.n)
    ctx.pic_set_record_states(all_states)
    a = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(a)
    b = a.clone()
    c = a.clone()
    ctx.pic_step(a, 37)
    node_a = ctx.pic_step_nodes()
    ctx.pic_forward_record(b, 37, 10)
    node_b = ctx.pic_step_nodes()
    t, h, ch, _ = ctx.pic_get_tiling()
    ctx.pic_set_tiling(t, h, ch, 3)  # re-binning at every checkpoint
    ctx.pic_forward_record(c, 37, 10)
    torch.cuda.synchronize()
    for x in (b, c):
        assert torch.equal(a.cell, x.cell) and torch.equal(a.off, x.off) and torch.equal(a.vel, x.vel)
    assert torch.equal(node_a, node_b)


@pytest.mark.parametrize("nd,rebin,family,flat,all_states",
                         [(2, False, "lj", False, False), (3, False, "lj", False, False),
                          (2, True, "lj", False, False), (3, True, "lj", False, False),
                          (2, False, "morse", False, False), (3, True, "morse", False, False),
                          (2, True, "hcp", False, False), (3, False, "hcp", False, False),
                          (3, False, "lj", True, False), (3, True, "hcp", True, False),
                          (2, True, "lj", False, True), (3, True, "lj", False, True),
                          (3, False, "morse", False, True), (3, True, "hcp", True, True)])
def test_recorded_sweep_matches_per_step_chain(B, nd, rebin, family, flat, all_states):
    """rebin: re-binning at every checkpoint (each segment has its own order,
    the cotangents are permuted between segments).  family: the pair
    potential (Morse adds the alpha slot of dtheta).  flat: tiles half as
    long along the last axis (a flatter reverse-step window).  all_states:
    the record keeps every state and node sum, and the sweep recomputes
    nothing."""
    grid, parts, dt = _case(nd)
    pot = {"lj": W.Potential(c_att=0.27), "morse": W.morse_cu(c_att=0.43), "hcp": W.hcp(c_att=0.2)}[family]
    nsteps, every = 30, 8  # a ragged last segment
    ctx = B.Context(grid, pot, dt, parts.n)
    ctx.pic_set_record_states(all_states)
    t, h, c, s = ctx.pic_get_tiling()
    ctx.pic_set_tile_shape(t, t // 2 if flat else t, h, c, 5 if rebin else s)
    assert ctx.pic_get_tile_shape() == (t, t // 2 if flat else t)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    start = dp.clone()
    # per-step chain on caller arrays
    states = [dp.clone()]
    for _ in range(nsteps):
        node = ctx.pic_deposit(dp)
        F = ctx.pic_force(dp, node)
        ctx.pic_push(dp, F)
        states.append(dp.clone())
    lam_x, lam_v = _seed_cotangents(grid, states[-1])
    lx_ref, lv_ref = lam_x.clone(), lam_v.clone()
    dth_ref = torch.zeros(B.NTHETA, dtype=torch.float64, device="cuda")
    nbar_next = None
    for k in range(nsteps - 1, -1, -1):
        node = ctx.pic_deposit(states[k])
        nbar, _ = ctx.pic_adjoint_step(states[k], node, nbar_next, lx_ref, lv_ref, dtheta=dth_ref)
        nbar_next = nbar
    ctx.pic_deposit_vjp(states[0], nbar_next, lx_ref)
    ctx.pic_sync()
    # recorded
    rec_state = start.clone()
    rec = ctx.pic_forward_record(rec_state, nsteps, every)
    assert torch.equal(rec_state.off, states[-1].off) and torch.equal(rec_state.cell, states[-1].cell)
    lx, lv = lam_x.clone(), lam_v.clone()
    dth = ctx.pic_backward_record(rec_state, rec, lx, lv)
    torch.cuda.synchronize()
    for d in range(nd):
        ref = lx_ref[d].double().cpu().numpy()
        assert np.abs(lx[d].double().cpu().numpy() - ref).max() <= 1e-4 * np.abs(ref).max(), d
    for d in range(3):
        ref = lv_ref[d].double().cpu().numpy()
        got = lv[d].double().cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-30), d
    got, ref = dth.cpu().numpy(), dth_ref.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-12), (got, ref)


def test_backward_refuses_a_foreign_record(B):
    grid, parts, dt = _case(3)
    pot = W.Potential(c_att=0.27)
    ctx = B.Context(grid, pot, dt, parts.n)
    dp = B.DeviceParticles.from_host(parts)
    rec = ctx.pic_forward_record(dp, 12, 4)
    lam_x = torch.zeros_like(dp.off)
    lam_v = torch.zeros_like(dp.vel)
    bad = dict(rec, nsteps=11)
    with pytest.raises(B.PicError):
        ctx.pic_backward_record(dp, bad, lam_x, lam_v)
    ctx.pic_set_record_states(True)  # a record replayed under the other setting
    with pytest.raises(B.PicError):
        ctx.pic_backward_record(dp, rec, lam_x, lam_v)
    ctx.pic_set_record_states(False)
    ctx.pic_set_tiling(4, 1, 2048, -1)  # a different tiling invalidates the record
    with pytest.raises(B.PicError):
        ctx.pic_backward_record(dp, rec, lam_x, lam_v)


@pytest.mark.parametrize("nsteps,every,sort_every", [(5, 8, None), (6, 1, None), (1, 1, None), (13, 4, 2)])
def test_every_state_record_matches_checkpoints(B, nsteps, every, sort_every):
    """Degenerate segment shapes of a record that keeps every state: fewer
    steps than the checkpoint interval, one step per checkpoint, a single
    step, and re-binning at every checkpoint (sort_every 2: the checkpoint
    re-bins the state the previous step wrote into the record).  The final
    state is the same bits as with checkpoints only, and the sweep agrees
    to the order of float atomic sums."""
    grid, parts, dt = _case(3)
    ctx = B.Context(grid, W.Potential(c_att=0.27), dt, parts.n)
    if sort_every is not None:
        t, h, c, _ = ctx.pic_get_tiling()
        ctx.pic_set_tiling(t, h, c, sort_every)
    dp = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(dp)
    out = {}
    for all_states in (False, True):
        ctx.pic_set_record_states(all_states)
        x = dp.clone()
        rec = ctx.pic_forward_record(x, nsteps, every)
        lam_x, lam_v = _seed_cotangents(grid, x)
        dth = ctx.pic_backward_record(x, rec, lam_x, lam_v)
        torch.cuda.synchronize()
        out[all_states] = (x, lam_x, lam_v, dth)
    (a, ax_, av, ath), (b, bx, bv, bth) = out[False], out[True]
    assert torch.equal(a.cell, b.cell) and torch.equal(a.off, b.off) and torch.equal(a.vel, b.vel)
    for u, v in ((ax_, bx), (av, bv)):
        u, v = u.double().cpu().numpy(), v.double().cpu().numpy()
        assert np.abs(u - v).max() <= 1e-4 * max(np.abs(u).max(), 1e-30)
    ath, bth = ath.cpu().numpy(), bth.cpu().numpy()
    assert np.all(np.abs(ath - bth) <= 1e-5 * np.abs(ath) + 1e-12), (ath, bth)


def test_record_sizes_of_both_settings(B):
    """A record that keeps every state holds nsteps states (one per step,
    the ragged last segment's included) and nsteps + 2 node sums; the
    backward scratch then holds the cotangents only."""
    grid, parts, dt = _case(3)
    ctx = B.Context(grid, W.Potential(c_att=0.27), dt, parts.n)
    nsteps, every = 30, 8
    ck = B.lib.pic_record_bytes(ctx.ctx, nsteps, every)
    scr = B.lib.pic_backward_bytes(ctx.ctx, every)
    ctx.pic_set_record_states(True)
    full = B.lib.pic_record_bytes(ctx.ctx, nsteps, every)
    scr_full = B.lib.pic_backward_bytes(ctx.ctx, every)
    nodes = B.pic_num_nodes(grid)
    assert full - ck >= (nsteps - 4) * 28 * parts.n + (nsteps + 2) * 8 * nodes
    assert scr - scr_full >= every * 28 * parts.n + (every + 1) * 8 * nodes


@pytest.mark.parametrize("family,all_states", [("lj", False), ("morse", False), ("hcp", False), ("lj", True)])
def test_autograd_crater_gradient_matches_oracle_finite_differences(B, family, all_states):
    from paper_1502_07722_amd import autograd as A
    with open({"lj": GOLDEN, "morse": GOLDEN_MORSE, "hcp": GOLDEN_HCP}[family]) as fh:
        gold = json.load(fh)
    wl = W.cfg_adjoint_3d(n=16, layers=8)
    grid, p = wl.grid, wl.parts
    nsteps, y_s, tau, fref = gold["nsteps"], gold["y_s"], gold["tau"], gold["fluence"]
    dev = torch.device("cuda")
    cell = torch.from_numpy(p.cell).to(dev)
    off0 = torch.from_numpy(p.off).to(dev)
    vth = torch.from_numpy(p.v_thermal).to(dev)
    xi = torch.from_numpy(p.xi).to(dev)
    sig = torch.from_numpy(p.sigma.astype(np.float32)).to(dev)
    wq = torch.from_numpy(p.wq).to(dev)
    extra = ("alpha",) if family == "morse" else ()
    for name, keys in (("altered", ("D", "s_rep", "c_att", "F") + extra), ("unaltered", ("r0",))):
        rec = gold["potentials"][name]
        pot = {"lj": lambda c: W.Potential(c_att=c), "morse": lambda c: W.morse_cu(c_att=c),
               "hcp": lambda c: W.hcp(c_att=c)}[family](rec["c_att"])
        ctx = B.Context(grid, pot, wl.dt, p.n)
        ctx.pic_set_record_states(all_states)
        theta = A.theta_of(pot).requires_grad_(True)
        fl = torch.tensor(fref, dtype=torch.float64, device=dev, requires_grad=True)
        J, _, _ = A.crater_objective(ctx, cell, off0, vth, xi, sig, fref, fl, wq, theta, nsteps, 20, y_s, tau)
        J.backward()
        assert abs(J.item() - rec["J"]) <= 1e-5 * abs(rec["J"])
        got = dict(zip(A.THETA_KEYS, theta.grad.cpu().numpy()))
        got["F"] = fl.grad.item()
        for k in keys:
            fd = rec["dJ"][k]["0.0001"]
            fd_err = abs(rec["dJ"][k]["0.001"] - fd)
            print(f"[{name}] dJ/d{k}: autograd {got[k]:.9e} finite difference {fd:.9e} "
                  f"rel {abs(got[k] - fd) / abs(fd):.2e}")
            assert abs(got[k] - fd) <= 1e-4 * abs(fd) + fd_err, (k, got[k], fd)


def test_autograd_on_a_grid_too_small_for_tiles(B):
    """A 6^3 grid has no 3D tiling: the Trajectory Function takes the
    checkpointed per-step chain; its gradient matches the differentiable FP64
    reference (oracle/autograd_ref.py) within 1e-4 relative (measured
    2.0e-6 to 5.0e-5)."""
    from oracle import autograd_ref as R
    from paper_1502_07722_amd import autograd as A
    wl = W.cfg_adjoint_3d(n=6, layers=3)
    g, p = wl.grid, wl.parts
    nsteps, y_s, tau, fref = 12, wl.slab_rows * g.h[2], g.h[2], wl.fluence
    dev = torch.device("cuda")
    # r0 on the unaltered potential: with c_att != s_rep its derivative jumps
    # where a neighbour distance crosses r0, which solid-density particles do
    for c_att, keys in ((0.27, ("D", "s_rep", "c_att")), (1.0, ("r0",))):
        pot = W.Potential(c_att=c_att)
        ctx = B.Context(g, pot, wl.dt, p.n)
        assert B.lib.pic_record_bytes(ctx.ctx, nsteps, 5) == 0  # untiled
        theta = A.theta_of(pot).requires_grad_(True)
        fl = torch.tensor(fref, dtype=torch.float64, device=dev, requires_grad=True)
        J, _, _ = A.crater_objective(ctx, torch.from_numpy(p.cell).to(dev), torch.from_numpy(p.off).to(dev),
                                     torch.from_numpy(p.v_thermal).to(dev), torch.from_numpy(p.xi).to(dev),
                                     torch.from_numpy(p.sigma.astype(np.float32)).to(dev), fref, fl,
                                     torch.from_numpy(p.wq).to(dev), theta, nsteps, 5, y_s, tau)
        J.backward()
        Jr, th, flr, _, _ = R.crater_objective(g, pot, wl.dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                               fref, p.wq, y_s, tau)
        Jr.backward()
        assert abs(J.item() - Jr.item()) <= 1e-5 * abs(Jr.item())
        for k in keys:
            i = A.THETA_KEYS.index(k)
            ref = th[k].grad.item()
            assert abs(theta.grad[i].item() - ref) <= 1e-4 * abs(ref), (k, theta.grad[i].item(), ref)
        if c_att != 1.0:
            assert abs(fl.grad.item() - flr.grad.item()) <= 1e-4 * abs(flr.grad.item())
