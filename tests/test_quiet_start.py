"""Quiet-start loading (the convergence studies' lattice-jittered slabs):
exact sub-lattice positions, jitter bounds, and the uniform deposit of the
unjittered sub-lattice (every interior node of the slab at solid density)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1502_07722_amd import workloads as W

H = 4e-9


@pytest.mark.parametrize("ndim,ppc", [(2, 16), (2, 64), (3, 8)])
def test_unjittered_sub_lattice_deposits_uniform_density(ndim, ppc):
    n = (12, 10) if ndim == 2 else (6, 5, 8)
    layers = 5
    grid, p = W.make_slab(ndim, n, layers, ppc, H, 3, quiet=0.0, depth2d=1e-9)
    k = round(ppc ** (1 / ndim))
    sub = np.sort(np.unique(p.off[0]))
    assert np.allclose(sub, (np.arange(k) + 0.5) / k, rtol=0, atol=1e-7)
    dens = O.density(grid, O.deposit(grid, p.cell, p.off, p.wq)).reshape(-1, int(np.prod(
        [grid.n[d] + grid.bc[d] for d in range(ndim - 1)])))
    w_exact = W.N_SOLID * (H ** 3 if ndim == 3 else H * H * 1e-9) / ppc
    q = p.wq[0] * 2.0 ** -20 / w_exact
    assert np.allclose(dens[1:layers], W.N_SOLID * q, rtol=1e-7, atol=0)  # the split's floor: < 1 unit in W


def test_jitter_stays_inside_the_sub_cell_and_bad_ppc_is_refused():
    ppc, k = 36, 6
    grid, p = W.make_slab(2, (16, 16), 8, ppc, H, 5, quiet=0.8, depth2d=1e-9)
    base = np.tile(np.stack(np.meshgrid(np.arange(k), np.arange(k), indexing="ij")).reshape(2, ppc),
                   (1, p.n // ppc))
    dev = p.off.astype(np.float64) * k - (base + 0.5)
    assert np.abs(dev).max() <= 0.4 + 1e-6 and np.abs(dev).max() > 0.3
    assert p.off.min() >= 0 and p.off.max() < 1
    with pytest.raises(ValueError):
        W.make_slab(2, (8, 8), 4, 10, H, 1, quiet=0.5)
