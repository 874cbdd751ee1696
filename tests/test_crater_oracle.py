"""Pins of the crater-measurement oracle (oracle/crater.py) to closed forms.

* A flat lattice slab of L layers has every column exactly L cells thick
  (up to the 2^-20 weight quantization), no depth and no crater.
* A rectangular hole carved out of the lattice gives the closed-form
  thickness profile (full deficit inside, half on the node columns of its
  edges, a quarter on 3D corners) and hence exact column counts on either
  side of those levels.
* Gas below the 1 % cut-off does not change any column; a clump above it
  adds exactly its atoms.
* Eq. (5) inverts the Gaussian crater edge: widths built from a known
  threshold give it back, per slab and through both sweep estimates, and a
  lattice slab carved wherever a Gaussian fluence exceeds the threshold
  measures it to within the node spacing.
"""
import math

import numpy as np
import pytest

from oracle import crater as CR
from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

H = 2e-9
NS = W.N_SOLID


def _lattice(ndim, n, layers, k=2):
    bc = (0, 1) if ndim == 2 else (0, 0, 1)
    grid, p = W.make_lattice(ndim, n, k, H, fill_layers=layers, bc=bc)
    return grid, p


def _keep(p, mask):
    return p.cell[mask], p.off[:, mask], p.wq[mask]


def _cell_coords(grid, cell):
    c = cell.astype(np.int64)
    out = []
    for d in range(grid.ndim):
        out.append(c % grid.n[d])
        c = c // grid.n[d]
    return out


@pytest.mark.parametrize("ndim,n", [(2, (48, 32)), (3, (12, 10, 16))])
def test_flat_slab_is_uniformly_thick_and_uncratered(ndim, n):
    layers = 11
    grid, p = _lattice(ndim, n, layers)
    node = O.deposit(grid, p.cell, p.off, p.wq)
    t = CR.column_thickness(grid, node, NS)
    w_exact = NS * H ** 3 / 2 ** ndim
    q = p.wq[0] * 2.0 ** -20 / w_exact  # weight quantization factor
    assert np.allclose(t, layers * H * q, rtol=1e-12, atol=0)
    assert abs(q - 1) < 1e-8
    r = CR.crater(grid, node, NS, y_s=layers * H)
    assert abs(r["depth"]) < 1e-7 * H and r["ncols"] == 0 and r["width"] == 0.0
    # interior nodes of the slab are at solid density, nodes above it empty
    rho = CR.solid_density(grid, node, NS)
    cols = int(np.prod([grid.n[d] + grid.bc[d] for d in range(ndim - 1)]))
    rows = rho.reshape(-1, cols)
    assert np.allclose(rows[1:layers], q, rtol=1e-12, atol=0)
    assert np.all(rows[layers + 1:] == 0)


def test_carved_hole_2d_closed_form():
    layers, d, x0, w = 14, 6, 9, 10
    grid, p = _lattice(2, (40, 28), layers)
    i, j = _cell_coords(grid, p.cell)
    hole = (i >= x0) & (i < x0 + w) & (j >= layers - d)
    node = O.deposit(grid, *_keep(p, ~hole))
    t = CR.column_thickness(grid, node, NS)
    q = p.wq[0] * 2.0 ** -20 / (NS * H ** 3 / 4)
    want = np.full(grid.n[0], layers * H * q)
    want[x0 + 1:x0 + w] = (layers - d) * H * q
    want[[x0, x0 + w]] = (layers - d / 2) * H * q
    # the fixed-point deposit splits a weight W with a floor: each particle's
    # share of an edge column is off by at most one unit in W (~1.8e8 units)
    assert np.allclose(t, want, rtol=1e-8, atol=0)
    y_s = layers * H
    r = CR.crater(grid, node, NS, y_s, depth_min=1.0 * H)   # below the edge deficit d/2
    assert r["ncols"] == w + 1 and r["width"] == pytest.approx((w + 1) * H, rel=1e-15, abs=0)
    assert r["depth"] == pytest.approx(d * H, rel=1e-8, abs=0)
    r = CR.crater(grid, node, NS, y_s, depth_min=(d / 2 + 0.5) * H)  # above it
    assert r["ncols"] == w - 1
    r = CR.crater(grid, node, NS, y_s, depth_min=(d + 0.5) * H)  # deeper than the hole
    assert r["ncols"] == 0 and r["width"] == 0.0


def test_carved_hole_3d_closed_form():
    layers, d, x0, y0, w = 8, 4, 3, 2, 5
    grid, p = _lattice(3, (12, 11, 12), layers)
    i, j, k = _cell_coords(grid, p.cell)
    hole = (i >= x0) & (i < x0 + w) & (j >= y0) & (j < y0 + w) & (k >= layers - d)
    node = O.deposit(grid, *_keep(p, ~hole))
    t = CR.column_thickness(grid, node, NS).reshape(grid.n[1], grid.n[0])
    q = p.wq[0] * 2.0 ** -20 / (NS * H ** 3 / 8)
    # share of the hole each node column sees: product of per-axis shares
    sx = np.zeros(grid.n[0]); sx[x0 + 1:x0 + w] = 1; sx[[x0, x0 + w]] = 0.5
    sy = np.zeros(grid.n[1]); sy[y0 + 1:y0 + w] = 1; sy[[y0, y0 + w]] = 0.5
    want = (layers - d * sy[:, None] * sx[None, :]) * H * q
    assert np.allclose(t, want, rtol=1e-8, atol=0)  # fixed-point split rounding, as in 2D
    y_s = layers * H
    r = CR.crater(grid, node, NS, y_s, depth_min=0.5 * H)  # below the corner deficit d/4
    assert r["ncols"] == (w + 1) ** 2
    assert r["width"] == pytest.approx(2 * math.sqrt((w + 1) ** 2 * H * H / math.pi), rel=1e-14, abs=0)
    r = CR.crater(grid, node, NS, y_s, depth_min=1.5 * H)  # between d/4 and d/2
    assert r["ncols"] == (w - 1) ** 2 + 4 * (w - 1)
    r = CR.crater(grid, node, NS, y_s, depth_min=2.5 * H)  # between d/2 and d
    assert r["ncols"] == (w - 1) ** 2


def test_gas_below_the_cut_off_is_not_counted_and_a_clump_above_is():
    layers = 10
    grid, p = _lattice(2, (32, 30), layers)
    node0 = O.deposit(grid, p.cell, p.off, p.wq)
    t0 = CR.column_thickness(grid, node0, NS)
    rng = np.random.default_rng(3)
    ngas = 200
    gcell = (rng.integers(0, 32, ngas) + 32 * rng.integers(layers + 3, 28, ngas)).astype(np.int32)
    goff = rng.random((2, ngas)).astype(np.float32)
    # each gas particle alone is far below 1 % of solid density on any node
    gw = np.full(ngas, W.weight_q(0.001 * NS * H ** 3 * 0.25), dtype=np.int32)
    node1 = O.deposit(grid, np.concatenate([p.cell, gcell]), np.concatenate([p.off, goff], axis=1),
                      np.concatenate([p.wq, gw]))
    assert CR.solid_density(grid, node1, NS).max() > 0
    rho_gas = O.density(grid, node1 - node0) / NS
    assert rho_gas.max() < 0.01  # and the gas nodes hold nothing else
    assert np.array_equal(CR.column_thickness(grid, node1, NS), t0)
    # a dense clump (one lattice cell's atoms, well above the cut) high in column 7's cells
    ccell = np.full(4, 7 + 32 * 24, dtype=np.int32)
    coff = np.array([[0.25, 0.75, 0.25, 0.75], [0.25, 0.25, 0.75, 0.75]], dtype=np.float32)
    cw = np.full(4, p.wq[0], dtype=np.int32)
    node2 = O.deposit(grid, np.concatenate([p.cell, ccell]), np.concatenate([p.off, coff], axis=1),
                      np.concatenate([p.wq, cw]))
    t2 = CR.column_thickness(grid, node2, NS)
    added = 4 * p.wq[0] * 2.0 ** -20 / (NS * H * grid.depth2d)  # atoms / (n_s x column cross-section)
    assert t2.sum() - t0.sum() == pytest.approx(added, rel=1e-12, abs=0)
    assert np.array_equal(t2[:7], t0[:7]) and np.array_equal(t2[9:], t0[9:])


def test_eq5_inverts_gaussian_crater_widths():
    a, F_th = 600e-9, 0.15e4
    F = np.array([0.1, 0.2, 0.5, 1.0, 2.0, 5.0]) * 1e4
    G = np.where(F > F_th, a * np.sqrt(np.log(np.maximum(F / F_th, 1.0))), 0.0)
    for f, g in zip(F[G > 0], G[G > 0]):
        assert CR.threshold_fluence(f, g, a) == pytest.approx(F_th, rel=1e-13, abs=0)
    fixed, fit, a_fit = CR.sweep_threshold(F, G, a)
    assert fixed == pytest.approx(F_th, rel=1e-13, abs=0)
    assert fit == pytest.approx(F_th, rel=1e-10, abs=0) and a_fit == pytest.approx(a, rel=1e-12, abs=0)
    assert math.isnan(CR.sweep_threshold(F[:1], G[:1], a)[0])


def test_carved_gaussian_crater_measures_its_threshold():
    """Remove the top d layers wherever the local fluence F exp(-2 x^2/R^2)
    exceeds F_th: the measured width through eq. (5) with a = sqrt(2) R gives
    F_th back to within the node spacing."""
    nx, layers, d = 256, 12, 6
    R = 60 * H
    F, F_th = 2.0e4, 0.5e4
    grid, p = _lattice(2, (nx, 24), layers)
    i, j = _cell_coords(grid, p.cell)
    xc = (i + 0.5 - nx / 2) * H
    local = F * np.exp(-2 * xc ** 2 / R ** 2)
    node = O.deposit(grid, *_keep(p, ~((local > F_th) & (j >= layers - d))))
    a = CR.beam_diameter(R)
    r = CR.crater(grid, node, NS, layers * H, depth_min=1.0 * H, fluence=F, beam_d=a)
    g_true = a * math.sqrt(math.log(F / F_th))
    assert abs(r["width"] - g_true) <= 2 * H
    lo = F * math.exp(-((g_true + 2 * H) / a) ** 2)
    hi = F * math.exp(-((g_true - 2 * H) / a) ** 2)
    assert lo <= r["f_th"] <= hi
