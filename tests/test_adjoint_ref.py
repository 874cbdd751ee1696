"""Pins of the differentiable FP64 reference (oracle/autograd_ref.py), which in
turn pins the hand-written adjoint:

* its forward cycle reproduces the C oracle (unquantized deposit) to rounding,
  an independent restatement of the same steps;
* its reverse-mode gradients of the crater functional
  J = sum_p w_p sigmoid((y_p(T) - y_s)/tau) match central finite differences
  of the C oracle, for the potential parameters, the fluence and the initial
  offsets.

The r0 derivative is pinned with s_rep = c_att: with different branch
multipliers the force's r0-derivative jumps where a neighbour distance crosses
r0 (U'(r0) = 0 keeps the force itself continuous), so finite differences in r0
cross kinks at every step size and converge only slowly; D, s_rep, c_att and
the fluence do not move the branch point and are pinned on the altered
potential itself.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import autograd_ref as R
from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

FREF = 1.5e4  # J/m^2 (1.5 J/cm^2)


def _case3d():
    wl = W.cfg_adjoint_3d(n=6, layers=3)
    return wl.grid, wl.parts, wl.dt, wl.slab_rows * wl.grid.h[2], wl.grid.h[2]


def _case2d():
    grid, parts = W.make_slab(2, (12, 12), 6, 4, W.H_CELL, 11, fluence_Jcm2=1.5, R_cells=6.0)
    return grid, parts, W.DT, 6 * grid.h[1], grid.h[1]


CASES = {"3d": _case3d, "2d": _case2d}


def _oracle_J(grid, parts, pot, dt, nsteps, y_s, tau, fluence=FREF, off=None):
    return O.crater_objective(grid, pot, dt, nsteps, parts.cell, parts.off if off is None else off,
                              parts.v_thermal, parts.xi, parts.sigma, FREF, fluence, parts.wq, y_s, tau)


@pytest.mark.parametrize("case", sorted(CASES))
def test_reference_forward_matches_oracle(case):
    grid, p, dt, y_s, tau = CASES[case]()
    pot = W.Potential(c_att=0.27)
    nsteps = 30
    J, _, _, (idx, f, v), _ = R.crater_objective(grid, pot, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi,
                                                 p.sigma, FREF, p.wq, y_s, tau)
    v0 = O.heated_start(p.v_thermal, p.xi, p.sigma, FREF, FREF)
    vh = O.start_leapfrog(grid, pot, dt, p.cell, p.off.astype(np.float64), v0, p.wq, False)
    c, o, vv, _ = O.run(grid, pot, dt, p.cell, p.off.astype(np.float64), vh, p.wq, nsteps, quantized=False)
    nd = grid.ndim
    cell_t = idx[0] + grid.n[0] * idx[1] + (grid.n[0] * grid.n[1] * idx[2] if nd == 3 else 0)
    assert np.array_equal(cell_t.numpy(), c)
    for d in range(nd):
        assert np.abs(f[d].detach().numpy() - o[d]).max() < 1e-12
    vscale = np.abs(vv).max()
    for d in range(3):
        assert np.abs(v[d].detach().numpy() - vv[d]).max() < 1e-12 * vscale
    Jc = O.functional(grid, c, o, p.wq, y_s, tau)
    assert abs(J.item() - Jc) <= 1e-13 * abs(Jc)


def _fd(fun, x, rel):
    # J is smooth in D, s_rep, c_att and the fluence: a relative step of 1e-3
    # keeps the O(h^2) truncation near 1e-8 while staying far above the
    # rounding noise of J (about 1e-12 relative).
    h = rel * abs(x)
    return (fun(x + h) - fun(x - h)) / (2 * h)


@pytest.mark.parametrize("case", sorted(CASES))
def test_reference_gradients_match_oracle_fd(case):
    grid, p, dt, y_s, tau = CASES[case]()
    nsteps = 30
    pot = W.Potential(c_att=0.27)
    J, th, Fl, _, _ = R.crater_objective(grid, pot, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                         FREF, p.wq, y_s, tau)
    J.backward()
    for k in ("D", "s_rep", "c_att"):
        fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot, **{k: x}), dt, nsteps, y_s, tau),
                 getattr(pot, k), 1e-3)
        assert abs(th[k].grad.item() - fd) <= 2e-6 * abs(fd), (k, th[k].grad.item(), fd)
    fd = _fd(lambda x: _oracle_J(grid, p, pot, dt, nsteps, y_s, tau, fluence=x), FREF, 1e-3)
    assert abs(Fl.grad.item() - fd) <= 2e-6 * abs(fd), (Fl.grad.item(), fd)
    # r0 on the unaltered potential (no branch kink): second-order convergence
    pot1 = W.Potential(c_att=1.0)
    J1, th1, _, _, _ = R.crater_objective(grid, pot1, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                          FREF, p.wq, y_s, tau)
    J1.backward()
    fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot1, r0=x), dt, nsteps, y_s, tau), pot1.r0, 1e-4)
    assert abs(th1["r0"].grad.item() - fd) <= 2e-6 * abs(fd), (th1["r0"].grad.item(), fd)


def test_reference_offset_gradients_match_oracle_fd():
    grid, p, dt, y_s, tau = _case3d()
    nsteps = 20
    pot = W.Potential(c_att=0.27)
    J, _, _, _, f0 = R.crater_objective(grid, pot, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                        FREF, p.wq, y_s, tau, offsets_grad=True)
    J.backward()
    rng = np.random.default_rng(3)
    # particles of the top slab layer (they feel the surface gradient), away
    # from the centre-stencil switch at f = 1/2 and from the cell faces
    top = np.nonzero((p.cell // (grid.n[0] * grid.n[1]) == 2)
                     & np.all(np.abs(p.off - 0.5) > 0.02, axis=0)
                     & np.all((p.off > 0.02) & (p.off < 0.98), axis=0))[0]
    Jv = J.item()
    h = 1e-3
    for i in rng.choice(top, 6, replace=False):
        fd = np.zeros(3)
        for d in range(3):
            x0 = float(p.off[d, i])

            def J_of(x):
                off = p.off.astype(np.float64).copy()
                off[d, i] = x
                return _oracle_J(grid, p, pot, dt, nsteps, y_s, tau, off=off)

            fd[d] = (J_of(x0 + h) - J_of(x0 - h)) / (2 * h)
        ag = np.array([f0[d].grad[i].item() for d in range(3)])
        # componentwise, relative to the gradient's norm: the lateral parts are
        # three to four orders smaller than the normal one and carry the FD's
        # rounding noise (about 1e-12 |J| / h) and kinks of other particles
        assert np.abs(ag - fd).max() <= 1e-5 * np.linalg.norm(fd) + 4e-12 * abs(Jv) / h, (i, ag, fd)


# The Morse potential (the method takes any pair potential): the reference's
# forward cycle against the C oracle, and its gradients -- now including the
# Morse width alpha -- against central differences of the C oracle.
@pytest.mark.parametrize("case", sorted(CASES))
def test_reference_morse_forward_and_gradients_match_oracle(case):
    grid, p, dt, y_s, tau = CASES[case]()
    nsteps = 30
    pot = W.morse_cu(c_att=0.43)
    J, th, Fl, (idx, f, v), _ = R.crater_objective(grid, pot, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi,
                                                   p.sigma, FREF, p.wq, y_s, tau)
    Jc = _oracle_J(grid, p, pot, dt, nsteps, y_s, tau)
    assert abs(J.item() - Jc) <= 1e-13 * abs(Jc)
    J.backward()
    assert set(th) == {"D", "r0", "s_rep", "c_att", "alpha"}
    for k in ("D", "s_rep", "c_att", "alpha"):
        fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot, **{k: x}), dt, nsteps, y_s, tau),
                 getattr(pot, k), 1e-3)
        assert abs(th[k].grad.item() - fd) <= 2e-6 * abs(fd), (k, th[k].grad.item(), fd)
    fd = _fd(lambda x: _oracle_J(grid, p, pot, dt, nsteps, y_s, tau, fluence=x), FREF, 1e-3)
    assert abs(Fl.grad.item() - fd) <= 2e-6 * abs(fd), (Fl.grad.item(), fd)
    # r0 with equal branch multipliers (no kink where a distance crosses r0)
    pot1 = W.morse_cu(c_att=1.0)
    J1, th1, _, _, _ = R.crater_objective(grid, pot1, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                          FREF, p.wq, y_s, tau)
    J1.backward()
    fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot1, r0=x), dt, nsteps, y_s, tau), pot1.r0, 1e-4)
    assert abs(th1["r0"].grad.item() - fd) <= 2e-6 * abs(fd), (th1["r0"].grad.item(), fd)


# The hexagonal close-packed neighbour geometry (12 neighbours along their
# directions, the clamp on each neighbour's q): the reference's forward
# against the C oracle, its gradients against central differences of it.
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("kind", ["lj", "morse"])
def test_reference_hcp_forward_and_gradients_match_oracle(case, kind):
    grid, p, dt, y_s, tau = CASES[case]()
    nsteps = 30
    base = W.Potential() if kind == "lj" else W.morse_cu()
    pot = W.hcp(base, c_att=0.2)
    J, th, Fl, _, _ = R.crater_objective(grid, pot, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                         FREF, p.wq, y_s, tau)
    Jc = _oracle_J(grid, p, pot, dt, nsteps, y_s, tau)
    assert abs(J.item() - Jc) <= 1e-12 * abs(Jc)
    J.backward()
    keys = ("D", "s_rep", "c_att") + (("alpha",) if kind == "morse" else ())
    for k in keys:
        fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot, **{k: x}), dt, nsteps, y_s, tau),
                 getattr(pot, k), 1e-3)
        assert abs(th[k].grad.item() - fd) <= 2e-6 * abs(fd), (k, th[k].grad.item(), fd)
    # the fluence moves a few neighbours' q across the clamp within a 1e-3
    # step here (the central difference is not monotone in the step there);
    # at 3e-5 it has converged to 1e-9
    fd = _fd(lambda x: _oracle_J(grid, p, pot, dt, nsteps, y_s, tau, fluence=x), FREF, 3e-5)
    assert abs(Fl.grad.item() - fd) <= 2e-6 * abs(fd), (Fl.grad.item(), fd)
    pot1 = dataclasses.replace(pot, c_att=1.0)
    J1, th1, _, _, _ = R.crater_objective(grid, pot1, dt, nsteps, p.cell, p.off, p.v_thermal, p.xi, p.sigma,
                                          FREF, p.wq, y_s, tau)
    J1.backward()
    fd = _fd(lambda x: _oracle_J(grid, p, dataclasses.replace(pot1, r0=x), dt, nsteps, y_s, tau), pot1.r0, 1e-4)
    assert abs(th1["r0"].grad.item() - fd) <= 2e-6 * abs(fd), (th1["r0"].grad.item(), fd)


def test_reference_hcp_directions_are_the_oracles():
    """The reference builds the 12 directions its own way; as a set they are
    the C oracle's (and so the brute-force lattice's, which pins those)."""
    for nd in (2, 3):
        ref = np.array(R.hcp_neighbours(nd))[:, :nd]
        orc = O.hcp_directions()
        orc = orc if nd == 3 else orc[:, [0, 2]]
        for u in ref:
            assert np.min(np.linalg.norm(orc - u, axis=1)) < 1e-15
