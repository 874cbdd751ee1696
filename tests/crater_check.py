"""Comparison of the library's crater measurement with the FP64 oracle
(oracle/crater.py), shared by the GPU tests.

* density map: zero exactly where the oracle's FP64 density is below the
  cut-off, elsewhere within 2e-7 of it (the library scales the integer
  node sum in float: three roundings of 2^-24);
* column sums: bit-exact against the integer sum of the node weights the
  oracle keeps;
* thickness, depth, t_min, t_max, eq. (5): 1e-12 relative (the oracle sums
  rho * length per node, the library divides the exact integer sum once);
* cratered columns and width: exact, except for columns whose deficit lies
  within 1e-12 of depth_min (there the two roundings may decide apart).
"""
import numpy as np

from oracle import crater as CR
from oracle import oracle as O

REL = 1e-12


def lateral_measures(grid):
    return CR._lateral_measures(grid)


def check_slab(grid, node_sums, got, col_w, rho, n_solid, y_s, cut, depth_min, fluence=0.0, beam_d=0.0):
    """got: the library's result dict for this slab; col_w, rho: its host
    arrays (rho may be None)."""
    ref = CR.crater(grid, node_sums, n_solid, y_s, cut, depth_min, fluence, beam_d)
    dens = O.density(grid, node_sums) / n_solid
    keep = dens >= cut
    if rho is not None:
        assert np.array_equal(rho == 0, ~keep | (node_sums == 0)), "density map cut differs"
        assert np.allclose(rho, np.where(keep, dens, 0.0), rtol=2e-7, atol=0), "density map differs"
    cols = len(ref["thickness"])
    S = np.where(keep, node_sums, 0).reshape(-1, cols).sum(axis=0)
    assert np.array_equal(col_w, S), "column sums differ"
    m = lateral_measures(grid)
    area = (grid.h[0] * (grid.depth2d if grid.ndim == 2 else grid.h[1])) * (m / m.max())
    t = col_w * 2.0 ** -20 / (n_solid * area)
    assert np.allclose(t, ref["thickness"], rtol=REL, atol=REL * max(abs(y_s), grid.h[grid.ndim - 1]))
    scale = max(abs(y_s), grid.h[grid.ndim - 1])
    for k in ("depth", "t_min", "t_max"):
        assert abs(got[k] - ref[k]) <= REL * scale, (k, got[k], ref[k])
    deficit = y_s - ref["thickness"]
    tie = np.abs(deficit - depth_min) <= REL * scale
    n_ties = int(tie.sum())
    assert abs(got["ncols"] - ref["ncols"]) <= n_ties, (got["ncols"], ref["ncols"], n_ties)
    if n_ties == 0:
        assert got["ncols"] == ref["ncols"]
        assert abs(got["width"] - ref["width"]) <= REL * max(ref["width"], grid.h[0])
        if fluence > 0 and beam_d > 0:
            assert abs(got["f_th"] - ref["f_th"]) <= REL * fluence
    if not (fluence > 0 and beam_d > 0):
        assert got["f_th"] == 0.0
    return ref
