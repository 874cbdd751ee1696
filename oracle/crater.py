"""FP64 oracle of the crater measurement that follows the particle cycle, and
of the threshold-fluence relation eq. (5).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's checks,
never by the library.  Plain numpy on the node sums the oracle's deposit
produces; every quantity is written out as its definition.

What the paper gives (results section, Figs. 3-4 and eq. 5): density maps in
units of the solid density with nothing drawn below 1 % of it (the thin gas
there does not change the crater), the crater's width and depth measured
once the surface has settled, and a threshold fluence from eq. (5),
F_th = F exp(-(Gamma / a)^2), with Gamma the crater diameter and a the beam
diameter.  The paper does not say how width and depth are read off the map;
the readings below are this module's:

* Column thickness.  A column is the set of nodes that share their lateral
  indices; the normal (last) axis runs along it.  Its equivalent solid
  thickness is t = sum_j rho_j l_j over the nodes kept by the cut-off, with
  rho_j the node density in solid-density units and l_j the node's length
  along the normal (a cell edge, half of it on a reflecting wall), i.e. the
  thickness the column's atoms would have at solid density.
* Depth: the largest deficit y_s - t over the columns, y_s the initial
  surface height.
* Width: columns whose deficit is at least ``depth_min`` are cratered.  In
  2D, Gamma is their total lateral length; in 3D, the diameter of the circle
  of their total lateral area.  Each column's lateral extent is its node's
  (a cell edge, half of it on a reflecting lateral wall).
* Beam diameter in eq. (5): the diameter at which the Gaussian fluence falls
  to 1/e of its peak.  For a profile F exp(-2 x^2 / R^2) (R the 1/e^2
  radius) that is a = sqrt(2) R, and eq. (5) then states exactly that the
  crater edge sits where the local fluence equals F_th.
* Over a sweep of fluences: the fixed-diameter estimate is the geometric
  mean of the per-slab eq. (5) values (the least-squares value of ln F_th
  with a held fixed); the free fit regresses Gamma^2 on ln F (slope a^2,
  intercept -a^2 ln F_th) and also returns the diameter it implies.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def node_shape(grid):
    """Nodes per axis (periodic: n, reflecting: n + 1), fastest axis first."""
    return [grid.n[d] + grid.bc[d] for d in range(grid.ndim)]


def solid_density(grid, node_sums, n_solid: float, cut: float = 0.01):
    """Node density in units of n_solid, set to zero below ``cut``
    (float64, one value per node in the deposit's node order)."""
    rho = O.density(grid, node_sums) / n_solid
    return np.where(rho >= cut, rho, 0.0)


def _normal_lengths(grid):
    ax = grid.ndim - 1
    rows = grid.n[ax] + grid.bc[ax]
    ell = np.full(rows, grid.h[ax], dtype=np.float64)
    if grid.bc[ax]:
        ell[0] *= 0.5
        ell[-1] *= 0.5
    return ell


def _lateral_measures(grid):
    """Lateral length (2D) or area (3D) of each column's node."""
    m = np.ones(1, dtype=np.float64)
    for d in range(grid.ndim - 1):
        e = np.full(grid.n[d] + grid.bc[d], grid.h[d], dtype=np.float64)
        if grid.bc[d]:
            e[0] *= 0.5
            e[-1] *= 0.5
        m = (e[None, :] * m[:, None]).reshape(-1) if d else e.copy()
    return m


def column_thickness(grid, node_sums, n_solid: float, cut: float = 0.01):
    """Equivalent solid thickness of every column, m (columns in lateral node
    order, x fastest)."""
    rho = solid_density(grid, node_sums, n_solid, cut)
    shape = node_shape(grid)
    rows = shape[-1]
    cols = int(np.prod(shape[:-1]))
    ell = _normal_lengths(grid)
    t = np.zeros(cols, dtype=np.float64)
    for j in range(rows):
        t += rho[j * cols:(j + 1) * cols] * ell[j]
    return t


def crater(grid, node_sums, n_solid: float, y_s: float, cut: float = 0.01, depth_min: float | None = None,
           fluence: float = 0.0, beam_d: float = 0.0):
    """Depth, width and (when fluence and beam_d are given) the eq. (5)
    threshold of the crater in one slab's node sums."""
    if depth_min is None:
        depth_min = grid.h[grid.ndim - 1]
    t = column_thickness(grid, node_sums, n_solid, cut)
    deficit = y_s - t
    hit = deficit >= depth_min
    m = _lateral_measures(grid)
    measure = float(m[hit].sum())
    width = measure if grid.ndim == 2 else 2.0 * math.sqrt(measure / math.pi)
    out = dict(depth=float(deficit.max()), width=width, t_min=float(t.min()), t_max=float(t.max()),
               ncols=int(hit.sum()), thickness=t, cratered=hit)
    out["f_th"] = threshold_fluence(fluence, width, beam_d) if fluence > 0 and beam_d > 0 else 0.0
    return out


def threshold_fluence(fluence: float, width: float, beam_d: float) -> float:
    """Eq. (5)."""
    return fluence * math.exp(-((width / beam_d) ** 2))


def beam_diameter(R: float) -> float:
    """1/e diameter of the fluence profile exp(-2 x^2 / R^2)."""
    return math.sqrt(2.0) * R


def sweep_threshold(fluences, widths, beam_d: float):
    """Threshold over a sweep: (fixed-diameter estimate, free-fit estimate,
    free-fit diameter); slabs without a crater are left out; NaN where too
    few slabs remain (one for the first, two for the fit)."""
    F = np.asarray(fluences, dtype=np.float64)
    G = np.asarray(widths, dtype=np.float64)
    sel = G > 0
    fixed = fit = a_fit = float("nan")
    if sel.sum() >= 1:
        each = [threshold_fluence(f, g, beam_d) for f, g in zip(F[sel], G[sel])]
        fixed = math.exp(float(np.mean(np.log(each))))
    if sel.sum() >= 2:
        x = np.log(F[sel])
        y = G[sel] ** 2
        xm, ym = x.mean(), y.mean()
        sxx = float(((x - xm) ** 2).sum())
        if sxx > 0:
            slope = float(((x - xm) * (y - ym)).sum()) / sxx
            icpt = ym - slope * xm
            if slope > 0:
                a_fit = math.sqrt(slope)
                fit = math.exp(-icpt / slope)
    return fixed, fit, a_fit
