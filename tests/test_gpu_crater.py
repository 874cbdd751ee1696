"""GPU parity of the crater measurement (pic_crater) against the FP64 oracle
(oracle/crater.py), through the C ABI:

* a laser-heated slab after 300 fused steps (ejecta above the surface, some
  of it under the 1 % cut-off), ragged grid sizes (columns not a multiple of
  the 256-column block, rows not a multiple of the 32-row chunk), 2D and 3D;
* a carved lattice slab with gas and a clump, and lateral reflecting walls
  (half-measure wall columns);
* a batch of 18 slabs of different sizes and fluences (two launches of the
  16-slab table), and the sweep's threshold fit against the oracle's;
* degenerate inputs: an empty grid (every column cratered at depth y_s), a
  cut-off of zero, and invalid arguments rejected on the host.
The comparison rules are in tests/crater_check.py.
"""
import math

import numpy as np
import pytest
import torch

from oracle import crater as CR
from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

from crater_check import check_slab

pytestmark = pytest.mark.gpu

NS = W.N_SOLID
H = W.H_CELL


@pytest.fixture(scope="module")
def B():
    from paper_1502_07722_amd import binding
    return binding


def _measure(B, ctx, nodes_dev, y_s, cut=0.01, depth_min=None, fluence=None, beam_d=None):
    res, col_w, rho = ctx.pic_crater(nodes_dev, NS, y_s, cut, depth_min, fluence, beam_d, want_rho=True)
    return res, col_w.cpu().numpy(), rho.cpu().numpy()


@pytest.mark.parametrize("ndim,n,layers,fluence", [(2, (300, 77), 40, 6.0), (3, (20, 13, 24), 12, 8.0)])
def test_heated_slab_after_fused_steps(B, ndim, n, layers, fluence):
    grid, p = W.make_slab(ndim, n, layers, 16 if ndim == 2 else 8, H, 41, fluence_Jcm2=fluence, R_cells=40.0)
    print(f"[crater] heated {ndim}D {n}: {p.n} particles", flush=True)
    pot = W.Potential(c_att=0.27)
    ctx = B.Context(grid, pot, W.DT, p.n)
    dp = B.DeviceParticles.from_host(p)
    ctx.start_leapfrog(dp)
    ctx.pic_step(dp, 300)
    nodes_dev = ctx.pic_deposit(dp)
    cell, off, _, wq = dp.to_host()
    nodes = O.deposit(grid, cell, off.astype(np.float64), wq)
    assert np.array_equal(nodes_dev.cpu().numpy(), nodes)
    y_s = layers * H
    R = 40.0 * H
    for cut, dmin in ((0.01, 0.25 * H), (0.2, 1.0 * H), (0.0, 0.5 * H)):
        res, col_w, rho = _measure(B, ctx, nodes_dev, y_s, cut, dmin, fluence * 1e4, CR.beam_diameter(R))
        ref = check_slab(grid, nodes, res[0], col_w, rho, NS, y_s, cut, dmin, fluence * 1e4, CR.beam_diameter(R))
        print(f"[crater] cut {cut} depth_min {dmin:.1e}: depth {res[0]['depth']:.3e} width {res[0]['width']:.3e} "
              f"cols {res[0]['ncols']} (oracle {ref['ncols']})", flush=True)


def test_carved_slab_with_gas_clump_and_lateral_walls(B):
    layers = 20
    grid, p = W.make_lattice(2, (70, 45), 2, H, fill_layers=layers, bc=(1, 1))
    c = p.cell.astype(np.int64)
    i, j = c % 70, c // 70
    keep = ~((i >= 30) & (i < 47) & (j >= layers - 7))
    rng = np.random.default_rng(5)
    ng = 500
    gcell = (rng.integers(0, 70, ng) + 70 * rng.integers(layers + 2, 45, ng)).astype(np.int32)
    goff = rng.random((2, ng)).astype(np.float32)
    gw = rng.integers(1, W.weight_q(40.0), ng).astype(np.int32)
    cell = np.concatenate([p.cell[keep], gcell])
    off = np.concatenate([p.off[:, keep], goff], axis=1)
    wq = np.concatenate([p.wq[keep], gw])
    vel = np.zeros((3, len(cell)), np.float32)
    ctx = B.Context(grid, W.Potential(c_att=0.27), W.DT, len(cell))
    dp = B.DeviceParticles(*(torch.from_numpy(a).cuda() for a in (cell, off, vel, wq)))
    nodes_dev = ctx.pic_deposit(dp)
    nodes = O.deposit(grid, cell, off.astype(np.float64), wq)
    assert np.array_equal(nodes_dev.cpu().numpy(), nodes)
    for dmin in (1.0 * H, 4.0 * H):
        res, col_w, rho = _measure(B, ctx, nodes_dev, layers * H, 0.01, dmin)
        ref = check_slab(grid, nodes, res[0], col_w, rho, NS, layers * H, 0.01, dmin)
        assert ref["ncols"] > 0


def test_batch_of_18_slabs_and_threshold_fit(B):
    rng = np.random.default_rng(9)
    grids, parts, ys, Fs = [], [], [], []
    for k in range(18):
        w = int(rng.integers(40, 330))
        d = int(rng.integers(8, 40))
        F = 0.5 * 10 ** (k / 17)
        g, p = W.make_slab(2, (w, 2 * d), d, 8, H, 100 + k, fluence_Jcm2=F, R_cells=30.0)
        grids.append(g)
        parts.append(p)
        ys.append(d * H)
        Fs.append(F * 1e4)
    pot = W.Potential(c_att=0.27)
    ctx = B.BatchContext(grids, pot, W.DT, [p.n for p in parts])
    dps = [B.DeviceParticles.from_host(p) for p in parts]
    ctx.pic_step_batch(dps, 60)
    nodes_dev = ctx.pic_step_nodes()
    a = CR.beam_diameter(30.0 * H)
    res, col_w, rho = _measure(B, ctx, nodes_dev, ys, 0.01, 0.25 * H, Fs, [a] * 18)
    nodes_all = nodes_dev.cpu().numpy()
    no = co = 0
    refs = []
    for k, g in enumerate(grids):
        nn = g.nnodes
        nc = B.pic_num_columns(g)
        cell, off, _, wq = dps[k].to_host()
        nodes = O.deposit(g, cell, off.astype(np.float64), wq)
        assert np.array_equal(nodes_all[no:no + nn], nodes), k
        refs.append(check_slab(g, nodes, res[k], col_w[co:co + nc], rho[no:no + nn], NS, ys[k], 0.01, 0.25 * H,
                               Fs[k], a))
        no += nn
        co += nc
    widths = [r["width"] for r in res]
    got = B.pic_threshold_fit(Fs, widths, a)
    want = CR.sweep_threshold(Fs, widths, a)
    print(f"[crater] sweep: widths {np.round(np.array(widths) / H, 1)} cells; threshold {got} oracle {want}",
          flush=True)
    for x, y in zip(got, want):
        assert (math.isnan(x) and math.isnan(y)) or abs(x - y) <= 1e-10 * abs(y)


def test_empty_grid_and_invalid_arguments(B):
    grid = W.Grid(ndim=3, n=(9, 7, 5), h=(H, H, H), bc=(0, 0, 1))
    ctx = B.Context(grid, W.Potential(c_att=0.27), W.DT, 16)
    nodes_dev = torch.zeros(grid.nnodes, dtype=torch.int64, device="cuda")
    res, col_w, rho = _measure(B, ctx, nodes_dev, 3 * H, 0.01, 0.5 * H)
    assert res[0]["ncols"] == 63 and res[0]["depth"] == 3 * H and res[0]["t_max"] == 0.0
    assert res[0]["width"] == pytest.approx(2 * math.sqrt(63 * H * H / math.pi), rel=1e-15, abs=0)
    assert not col_w.any() and not rho.any()
    check_slab(grid, np.zeros(grid.nnodes, np.int64), res[0], col_w, rho, NS, 3 * H, 0.01, 0.5 * H)
    with pytest.raises(B.PicError):
        ctx.pic_crater(nodes_dev, -1.0, 3 * H)
    with pytest.raises(B.PicError):
        ctx.pic_crater(nodes_dev, NS, 3 * H, depth_min=0.0)
    with pytest.raises(B.PicError):
        ctx.pic_crater(nodes_dev, NS, 3 * H, fluence=1e4)  # fluence without a beam diameter
    with pytest.raises(ValueError):
        ctx.pic_crater(nodes_dev[:-1], NS, 3 * H)
