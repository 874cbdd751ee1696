"""Pins of the oracle's hexagonal close-packed (HCP) neighbour geometry (the
paper notes its cubic-lattice construction adapts to HCP):

* the 12 neighbour directions are those of an ideal HCP crystal built by
  brute force (two stacked triangular layers, c/a = sqrt(8/3)): the 12
  nearest sites of an atom, all at distance a;
* they sum to zero and their second moment is 4 I (isotropic);
* uniform density feels no force; a normal gradient gives no lateral force;
* the small-gradient force is -grad mu with mu = 2 (phi(a) - a phi'(a)),
  a = 2^(1/6) rbar (finite differences of the energy density), in 2D and 3D;
* the quadrature energy density equals the Lennard-Jones closed form
  D (13/10 r0^12 n^5 - 14/3 r0^6 n^3) with the branch switch at
  n = sqrt(2) / r0^3;
* the attractive correction's calibration converges in slab thickness.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

HCP = W.hcp()
N0 = W.N_SOLID
H = 2e-9


def _brute_force_neighbours():
    a = 1.0
    c = a * math.sqrt(8.0 / 3.0)
    b1 = np.array([a, 0.0, 0.0])
    b2 = np.array([a / 2, a * math.sqrt(3) / 2, 0.0])
    sites = []
    for i, j, k in itertools.product(range(-3, 4), range(-3, 4), range(-2, 3)):
        base = i * b1 + j * b2 + np.array([0.0, 0.0, k * c])
        sites.append(base)                                               # A layer
        sites.append(base + (b1 + b2) / 3 + np.array([0.0, 0.0, c / 2]))  # B layer
    sites = np.array(sites)
    d = np.linalg.norm(sites, axis=1)
    sites, d = sites[d > 1e-9], d[d > 1e-9]
    order = np.argsort(d)
    return sites[order[:12]] / d[order[:12], None], d[order[:13]]


def test_directions_are_the_nearest_neighbours_of_an_ideal_hcp_crystal():
    U = O.hcp_directions()
    bf, dist = _brute_force_neighbours()
    assert np.allclose(dist[:12], 1.0, atol=0) and dist[12] > 1.2  # a shell of exactly 12
    assert np.allclose(np.linalg.norm(U, axis=1), 1.0, atol=1e-15)
    for u in U:
        assert np.min(np.linalg.norm(bf - u, axis=1)) < 1e-12
    assert np.allclose(U.sum(axis=0), 0.0, atol=1e-14)
    assert np.allclose(U.T @ U, 4.0 * np.eye(3), atol=1e-14)


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_density_and_normal_gradient(ndim):
    scale = 12 * HCP.D / HCP.r0
    for x in (0.7, 1.0, 1.3):
        # zero up to the rounding of the 12 directions' components
        assert np.abs(O.local_force(HCP, ndim, x * N0, [0.0] * ndim)).max() <= 1e-14 * scale
        G = [0.0] * ndim
        G[-1] = 3e35
        F = O.local_force(HCP, ndim, x * N0, G)
        assert np.abs(F[:-1]).max() <= 1e-12 * abs(F[-1])


def _mu(pot, n):
    a = W.HCP_C * n ** (-1 / 3)
    return 2 * (O.phi(pot, a) - a * O.phi_prime(pot, a))


@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 1), (3, 0), (3, 2)])
def test_small_gradient_force_is_minus_grad_mu(ndim, axis):
    for pot in (HCP, W.hcp(s_rep=2.0, c_att=0.3), W.hcp(W.morse_cu())):
        for x in (0.5, 0.9, 1.2, 1.6):
            n = x * N0
            G = [0.0] * ndim
            G[axis] = 1e-5 * n / pot.r0
            F = O.local_force(pot, ndim, n, G)[axis]
            d = 1e-4 * n
            dmu = (_mu(pot, n + d) - _mu(pot, n - d)) / (2 * d)
            assert F == pytest.approx(-dmu * G[axis], rel=2e-4, abs=0)
            # and mu is the derivative of the energy density
            e = 1e-6 * n
            fd = (O.energy_density(pot, n + e) - O.energy_density(pot, n - e)) / (2 * e)
            assert fd == pytest.approx(_mu(pot, n), rel=1e-6, abs=0)


def test_lennard_jones_energy_density_closed_form():
    for s_rep, c_att in [(1.0, 1.0), (2.5, 0.3)]:
        pot = W.hcp(s_rep=s_rep, c_att=c_att)
        r0, D = pot.r0, pot.D
        e = lambda n: D * (1.3 * r0 ** 12 * n ** 5 - 14.0 / 3.0 * r0 ** 6 * n ** 3)
        nk = math.sqrt(2.0) / r0 ** 3
        for x in (0.2, 0.6, 1.0, 1.4, 1.9):
            n = x * nk
            want = c_att * e(n) if n <= nk else c_att * e(nk) + s_rep * (e(n) - e(nk)) + 2 * (s_rep - c_att) * D * (n - nk)
            assert O.energy_density(pot, n) == pytest.approx(want, rel=1e-10, abs=0)


def test_hcp_calibration_converges():
    grid = W.Grid(ndim=2, n=(4, 64), h=(H, H, H), bc=(0, 1))
    c8, w8, _ = O.calibrate_catt(grid, HCP, W.N_SOLID, slab_layers=8)
    c16, w16, _ = O.calibrate_catt(grid, HCP, W.N_SOLID, slab_layers=16)
    assert 0 < c8 < 1 and c16 == pytest.approx(c8, rel=1e-6, abs=0)
