"""Parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (a created stream with graph replay, autotuned
tiles), on outputs the FP64 oracle can compute one by one:

* after K fused steps, the node sums of the GPU state (int64, the whole
  grid) equal the oracle's fixed-point deposit of that state bit for bit,
  and the crater measurement on them (density map, column sums, depth,
  width, eq. (5)) matches the oracle's (rules in tests/crater_check.py);
* one more GPU step, for 20,000 sampled particles, matches the oracle's
  eq. (1)-(3) force from those full node sums followed by its leapfrog push
  (FP64): positions to 1e-5 cells, velocities to 1e-5 of the largest speed;
  on the large slab and the 128^3 3D slab also with the Morse potential and
  on the hexagonal close-packed lattice (the variants bench.py times);
* on the full 128^3 adjoint workload, the autograd gradient of the crater
  functional agrees with a central difference of the GPU forward itself in
  D and in the fluence (a property that holds at any size).
"""
import numpy as np
import pytest
import torch

from oracle import crater as CR
from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

from crater_check import check_slab

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1502_07722_amd import binding
    return binding


def _abs_pos(grid, cell, off):
    nd = grid.ndim
    c = cell.astype(np.int64)
    out = []
    for d in range(nd):
        out.append((c % grid.n[d]) + off[d].astype(np.float64))
        c = c // grid.n[d]
    return np.stack(out)


POTENTIALS = {"lj": lambda: W.Potential(c_att=0.27), "morse": lambda: W.morse_cu(c_att=0.43),
              "hcp": lambda: W.hcp(c_att=0.2)}


@pytest.mark.parametrize("name,variant", [("large", "lj"), ("heated", "lj"), ("adjoint3d", "lj"),
                                          ("large", "morse"), ("large", "hcp"), ("adjoint3d", "morse"),
                                          ("adjoint3d", "hcp")])
def test_full_size_nodes_and_sampled_step_match_oracle(B, name, variant):
    """variant: the pair potential and lattice bench.py also times on the
    large slab (Morse; L-J on the hexagonal close-packed lattice)."""
    wl = W.WORKLOADS[name]()
    g, p, dt = wl.grid, wl.parts, wl.dt
    pot = POTENTIALS[variant]()
    print(f"[fullsize] {wl.name} ({variant}): {p.n} particles", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dp = B.DeviceParticles.from_host(p)
        ctx = B.Context(g, pot, dt, p.n, stream=stream)
        ctx.start_leapfrog(dp)
        probe = dp.clone()  # tuned like bench.py: on a copy advanced a few steps
        ctx.pic_step(probe, 12)
        ctx.pic_autotune(probe, 6)
        del probe
        ctx.pic_step(dp, 20)
        nodes_dev = ctx.pic_step_nodes()
        nodes = nodes_dev.cpu().numpy()
        cell, off, vel, wq = dp.to_host()
        y_s = wl.slab_rows * g.h[g.ndim - 1]
        beam_d = CR.beam_diameter(200.0 * g.h[0])
        res, col_w, rho = ctx.pic_crater(nodes_dev, W.N_SOLID, y_s, 0.01, 0.5 * g.h[g.ndim - 1], wl.fluence,
                                         beam_d, want_rho=True)
        col_w, rho = col_w.cpu().numpy(), rho.cpu().numpy()
        ctx.pic_step(dp, 1)
        cell1, off1, vel1, _ = dp.to_host()
    stream.synchronize()
    ref = O.deposit(g, cell, off.astype(np.float64), wq)
    assert np.array_equal(nodes, ref), "full-grid node sums differ from the oracle's deposit"
    check_slab(g, ref, res[0], col_w, rho, W.N_SOLID, y_s, 0.01, 0.5 * g.h[g.ndim - 1], wl.fluence, beam_d)
    rng = np.random.default_rng(12)
    s = rng.choice(p.n, 20000, replace=False)
    F = O.forces_from_nodes(g, pot, ref, cell[s], off[:, s].astype(np.float64))
    exp_c = np.empty(len(s), np.int32)
    exp_f = np.empty((g.ndim, len(s)))
    exp_v = np.empty((3, len(s)))
    for k, i in enumerate(s):
        c, f, v = O.push_one(g, pot, dt, F[:, k], cell[i], off[:, i].astype(np.float64), vel[:, i].astype(np.float64))
        exp_c[k], exp_f[:, k], exp_v[:, k] = c, f, v
    got = _abs_pos(g, cell1[s], off1[:, s])
    want = _abs_pos(g, exp_c, exp_f)
    diff = got - want
    for d in range(g.ndim):
        if not g.bc[d]:  # minimal image across the periodic seam
            diff[d] -= g.n[d] * np.round(diff[d] / g.n[d])
    perr = np.abs(diff).max()
    verr = np.abs(vel1[:, s] - exp_v).max() / np.abs(exp_v).max()
    print(f"[fullsize] {wl.name} ({variant}): position {perr:.2e} cells, velocity {verr:.2e}", flush=True)
    assert perr <= 1e-5 and verr <= 1e-5


def test_full_size_gradient_matches_gpu_central_difference(B):
    from paper_1502_07722_amd import autograd as A
    wl = W.cfg_adjoint_3d()
    g, p = wl.grid, wl.parts
    nsteps, every, h = 40, 20, 1e-3
    y_s, tau, fref = wl.slab_rows * g.h[2], g.h[2], wl.fluence
    dev = torch.device("cuda")
    cell = torch.from_numpy(p.cell).to(dev)
    off0 = torch.from_numpy(p.off).to(dev)
    vth = torch.from_numpy(p.v_thermal).to(dev)
    xi = torch.from_numpy(p.xi).to(dev)
    sig = torch.from_numpy(p.sigma.astype(np.float32)).to(dev)
    wq = torch.from_numpy(p.wq).to(dev)

    def J_of(pot, F, grad=False, all_states=False):
        ctx = B.Context(g, pot, wl.dt, p.n)
        ctx.pic_set_record_states(all_states)
        theta = A.theta_of(pot).requires_grad_(grad)
        fl = torch.tensor(F, dtype=torch.float64, device=dev, requires_grad=grad)
        J, _, _ = A.crater_objective(ctx, cell, off0, vth, xi, sig, fref, fl, wq, theta, nsteps, every, y_s, tau)
        if not grad:
            return J.item()
        J.backward()
        return J.item(), theta.grad[0].item(), fl.grad.item()

    pot = W.Potential(c_att=0.27)
    _, dJdD, dJdF = J_of(pot, fref, grad=True)
    import dataclasses
    fdD = (J_of(dataclasses.replace(pot, D=pot.D * (1 + h)), fref)
           - J_of(dataclasses.replace(pot, D=pot.D * (1 - h)), fref)) / (2 * h * pot.D)
    fdF = (J_of(pot, fref * (1 + h)) - J_of(pot, fref * (1 - h))) / (2 * h * fref)
    print(f"[fullsize] dJ/dD adjoint {dJdD:.6e} GPU central difference {fdD:.6e}; "
          f"dJ/dF adjoint {dJdF:.6e} GPU central difference {fdF:.6e}", flush=True)
    assert abs(dJdD - fdD) <= 2e-3 * abs(fdD)
    assert abs(dJdF - fdF) <= 2e-3 * abs(fdF)
    # a record that keeps every state: the same sweep without recompute, equal
    # up to the order of float atomic sums
    _, aD, aF = J_of(pot, fref, grad=True, all_states=True)
    assert abs(aD - dJdD) <= 1e-5 * abs(dJdD) and abs(aF - dJdF) <= 1e-5 * abs(dJdF), (aD, dJdD, aF, dJdF)
