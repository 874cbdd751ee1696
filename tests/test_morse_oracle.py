"""Pins of the oracle's second pair potential, the Morse potential (the paper
names it among the potentials its density-to-distance map works with):

* the Morse closed forms: minimum -D at r0 with zero slope, the zero
  crossing at r0 - ln 2 / a, the e^-a(r - r0) tail, and U' the derivative
  of U (finite differences);
* the energy-density quadrature reproduces the Lennard-Jones closed form
  (so it is right before it is used where no closed form exists), and for
  Morse its derivative is the chemical potential mu(n) = phi(rbar) -
  rbar phi'(rbar), with the branch multipliers;
* the small-gradient force is -grad mu, a flat lattice feels no force and a
  compressed one pushes down its gradient;
* the attractive correction of the calibration is positive and converges
  in the slab thickness.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

MORSE = W.morse_cu()
N0 = MORSE.r0 ** -3
H = 2e-9


def test_morse_closed_forms():
    D, a, r0 = MORSE.D, MORSE.alpha, MORSE.r0
    assert O.phi(MORSE, r0) == pytest.approx(-D, rel=1e-15, abs=0)
    assert O.phi_prime(MORSE, r0) == 0.0
    assert abs(O.phi(MORSE, r0 - math.log(2) / a)) < 1e-14 * D
    for x in (3.0, 5.0, 8.0):  # far tail: U ~ -2 D e^{-a (r - r0)}
        r = r0 + x / a
        assert O.phi(MORSE, r) == pytest.approx(-2 * D * math.exp(-x) + D * math.exp(-2 * x), rel=1e-13, abs=0)
    for s_rep, c_att in [(1.0, 1.0), (3.0, 0.27)]:
        pot = W.morse_cu(s_rep=s_rep, c_att=c_att)
        for r in np.linspace(0.7, 3.0, 47) * r0:
            if abs(r - r0) < 1e-3 * r0:
                continue
            d = 1e-7 * r
            fd = (O.phi(pot, r + d) - O.phi(pot, r - d)) / (2 * d)
            assert O.phi_prime(pot, r) == pytest.approx(fd, rel=1e-6, abs=1e-9 * D / r0)
        assert O.phi(pot, r0 * (1 - 1e-12)) == pytest.approx(O.phi(pot, r0 * (1 + 1e-12)), rel=1e-9, abs=0)


def test_quadrature_reproduces_the_lennard_jones_closed_form():
    for s_rep, c_att in [(1.0, 1.0), (2.5, 0.3)]:
        pot = W.Potential(s_rep=s_rep, c_att=c_att)
        n0 = pot.r0 ** -3
        for x in (0.05, 0.4, 0.9, 1.0, 1.2, 1.8):
            n = x * n0
            assert O.energy_density_quad(pot, n) == pytest.approx(O.energy_density(pot, n), rel=1e-11, abs=0)


@pytest.mark.parametrize("s_rep,c_att", [(1.0, 1.0), (2.0, 0.3)])
def test_morse_energy_density_derivative_is_chemical_potential(s_rep, c_att):
    pot = W.morse_cu(s_rep=s_rep, c_att=c_att)
    for x in (0.2, 0.5, 0.73, 0.95, 1.05, 1.3, 1.9):
        n = x * N0
        rbar = n ** (-1 / 3)
        mu = O.phi(pot, rbar) - rbar * O.phi_prime(pot, rbar)
        d = 1e-6 * n
        fd = (O.energy_density(pot, n + d) - O.energy_density(pot, n - d)) / (2 * d)
        assert fd == pytest.approx(mu, rel=1e-6, abs=0)
    assert O.energy_density(pot, 0.0) == 0.0


@pytest.mark.parametrize("s_rep,c_att", [(1.0, 1.0), (2.0, 0.3)])
def test_morse_small_gradient_force_is_minus_grad_mu(s_rep, c_att):
    pot = W.morse_cu(s_rep=s_rep, c_att=c_att)

    def mu(n):
        rbar = n ** (-1 / 3)
        return O.phi(pot, rbar) - rbar * O.phi_prime(pot, rbar)

    for x in (0.5, 0.8, 1.1, 1.25):
        n = x * N0
        G = 1e-5 * n / pot.r0
        F = O.local_force(pot, 1, n, [G])[0]
        d = 1e-4 * n
        assert F == pytest.approx(-(mu(n + d) - mu(n - d)) / (2 * d) * G, rel=2e-4, abs=0)


def test_morse_lattice_is_static_and_compression_pushes_down_the_gradient():
    grid, p = W.make_lattice(2, (8, 8), 2, H, bc=(0, 0))
    F = O.forces(grid, MORSE, p.cell, p.off, p.wq)
    assert np.abs(F).max() == 0.0
    assert O.local_force(MORSE, 1, 1.1 * N0, [-1e36])[0] > 0
    assert O.local_force(MORSE, 1, 1.1 * N0, [+1e36])[0] < 0


def test_morse_attractive_correction_converges():
    grid = W.Grid(ndim=2, n=(4, 64), h=(H, H, H), bc=(0, 1))
    c8, w8, _ = O.calibrate_catt(grid, MORSE, W.N_SOLID, slab_layers=8)
    c16, w16, _ = O.calibrate_catt(grid, MORSE, W.N_SOLID, slab_layers=16)
    assert 0 < c8 < 1 and w8 > MORSE.D
    assert c16 == pytest.approx(c8, rel=1e-6, abs=0)
