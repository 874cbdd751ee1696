"""Differentiable FP64 reference of the PIC pair-potential cycle (arXiv 1502.07722)
in plain PyTorch CPU ops, for tiny cases.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU baseline of
the benchmark may import this module; the library never does.  It shares no
code with the C oracle or with the HIP path: it restates the same steps of the
paper independently, with the deposit in plain (unquantized) CIC form so that
every step is differentiable, and lets torch.autograd supply the reverse mode.

Its gradients pin the hand-written adjoint: they are themselves pinned against
central finite differences of the C oracle (tests/test_adjoint_ref.py).

Steps, in the paper's order (Sec. 2, Fig. 1):
  deposit   weights to the 2^d surrounding nodes, linear (CIC) shares
  density   n = weight / node volume (half volume on reflecting walls)
  gradient  at the cell centres: mean of the 2^(d-1) edge differences / h
  gather    n from the 2^d nodes, G from the 2^d nearest centres (mirror
            ghosts on reflecting walls: normal component negated)
  eq. (1)   rbar = n^(-1/3), g = d rbar/dx = -(1/3) G n^(-4/3), clamped
  eq. (2)   r(+d) = rbar / (1 - g/2), r(-d) = rbar / (1 + g/2)
  eq. (3)   F = Phi'(r+) - Phi'(r-), Phi' = s_rep U' (r < r0), c_att U' (r >= r0);
            U is Lennard-Jones, or Morse D (e^2 - 2e), e = exp(-alpha (r - r0))
            (the paper's method takes any pair potential; only U' changes);
            on the hexagonal close-packed lattice the 12 neighbours' pair
            forces along their directions replace the per-axis pairs
  push      leapfrog: v += F/m dt, x += v dt, carry / wrap / mirror
Functional: J = sum_p w_p sigmoid((y_p - y_s) / tau) on the normal axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

WUNIT = 2.0 ** -20  # atoms per weight unit of wq


@dataclass
class Geometry:
    ndim: int
    n: tuple       # cells per axis (3 entries)
    h: tuple       # cell size per axis, m
    bc: tuple      # 0 periodic, 1 reflecting
    depth2d: float

    @staticmethod
    def of(grid) -> "Geometry":
        d2 = grid.depth2d if grid.ndim == 2 else 0.0
        return Geometry(grid.ndim, tuple(int(v) for v in grid.n), tuple(float(v) for v in grid.h),
                        tuple(int(v) for v in grid.bc), float(d2))

    def nodes_on(self, d: int) -> int:
        return self.n[d] + (1 if self.bc[d] else 0)

    @property
    def nnodes(self) -> int:
        return math.prod(self.nodes_on(d) for d in range(self.ndim))

    @property
    def ncells(self) -> int:
        return math.prod(self.n[: self.ndim])


def _node_linear(geo: Geometry, a):
    """a: list of per-axis node coordinates (LongTensor), already in range."""
    k = torch.zeros_like(a[0])
    stride = 1
    for d in range(geo.ndim):
        k = k + a[d] * stride
        stride *= geo.nodes_on(d)
    return k


def _node_coord(geo: Geometry, d: int, a):
    # periodic axes store node n as node 0; reflecting axes keep 0..n
    return torch.remainder(a, geo.n[d]) if not geo.bc[d] else a


def _corners(geo: Geometry):
    return [[(k >> d) & 1 for d in range(geo.ndim)] for k in range(1 << geo.ndim)]


def deposit(geo: Geometry, idx, f, w):
    """Node weight sums (atoms): each particle's weight w split over its 2^d
    nodes with weights prod_d (f_d or 1 - f_d).  Differentiable in f and w."""
    N = torch.zeros(geo.nnodes, dtype=torch.float64)
    for bits in _corners(geo):
        s = w
        a = []
        for d in range(geo.ndim):
            s = s * (f[d] if bits[d] else 1.0 - f[d])
            a.append(_node_coord(geo, d, idx[d] + bits[d]))
        N = N.index_add(0, _node_linear(geo, a), s)
    return N


def node_volumes(geo: Geometry):
    V = geo.h[0] * geo.h[1] * (geo.h[2] if geo.ndim == 3 else geo.depth2d)
    shape = [geo.nodes_on(d) for d in range(geo.ndim)]
    vol = torch.full(shape[::-1], V, dtype=torch.float64)  # index order [..., a1, a0]
    for d in range(geo.ndim):
        if geo.bc[d]:
            ax = geo.ndim - 1 - d
            sl = [slice(None)] * geo.ndim
            sl[ax] = 0
            vol[tuple(sl)] *= 0.5
            sl[ax] = geo.n[d]
            vol[tuple(sl)] *= 0.5
    return vol.reshape(-1)


def density(geo: Geometry, N):
    return N / node_volumes(geo)


def centre_gradient(geo: Geometry, dens):
    """G[d] at every cell centre: mean of the edge differences along d over the
    cell's 2^(d-1) edges, divided by h_d."""
    nd = geo.ndim
    cells = torch.arange(geo.ncells)
    ci = []
    r = cells
    for d in range(nd):
        ci.append(r % geo.n[d])
        r = r // geo.n[d]
    corner_vals = {}
    for bits in _corners(geo):
        a = [_node_coord(geo, d, ci[d] + bits[d]) for d in range(nd)]
        corner_vals[tuple(bits)] = dens[_node_linear(geo, a)]
    G = []
    for d in range(nd):
        acc = torch.zeros(geo.ncells, dtype=torch.float64)
        for bits, v in corner_vals.items():
            acc = acc + (v if bits[d] else -v)
        G.append(acc / (2 ** (nd - 1) * geo.h[d]))
    return torch.stack(G)  # [nd, ncells]


def gather(geo: Geometry, dens, G, idx, f):
    """n at the particle from its 2^d nodes; G from the 2^d nearest cell
    centres, reflecting walls mirrored (normal component negated)."""
    nd = geo.ndim
    n_p = 0.0
    for bits in _corners(geo):
        s = 1.0
        a = []
        for d in range(nd):
            s = s * (f[d] if bits[d] else 1.0 - f[d])
            a.append(_node_coord(geo, d, idx[d] + bits[d]))
        n_p = n_p + s * dens[_node_linear(geo, a)]
    # centre stencil: centres at c + 1/2; lower one c0 = idx (f >= 1/2) or idx - 1
    c0, t = [], []
    for d in range(nd):
        hi = f[d] >= 0.5
        c0.append(torch.where(hi, idx[d], idx[d] - 1))
        t.append(torch.where(hi, f[d] - 0.5, f[d] + 0.5))
    Gp = []
    for comp in range(nd):
        acc = 0.0
        for bits in _corners(geo):
            s = 1.0
            m = []
            sign = torch.ones_like(f[0])
            for d in range(nd):
                s = s * (t[d] if bits[d] else 1.0 - t[d])
                md = c0[d] + bits[d]
                if geo.bc[d]:
                    lo, hi = md < 0, md >= geo.n[d]
                    if d == comp:
                        sign = torch.where(lo | hi, -sign, sign)
                    md = torch.where(lo, torch.zeros_like(md), torch.where(hi, torch.full_like(md, geo.n[d] - 1), md))
                else:
                    md = torch.remainder(md, geo.n[d])
                m.append(md)
            lin = torch.zeros_like(m[0])
            stride = 1
            for d in range(nd):
                lin = lin + m[d] * stride
                stride *= geo.n[d]
            acc = acc + s * sign * G[comp][lin]
        Gp.append(acc)
    return n_p, Gp


def hcp_neighbours(ndim: int):
    """Unit vectors to the 12 nearest neighbours of an ideal hexagonal
    close-packed site (c/a = sqrt(8/3)), in grid axes: the basal plane holds
    six at 60 degree steps from the x axis; three sit a height sqrt(2/3) above
    it and three below, over the centres of alternate basal triangles (in-plane
    distance 1/sqrt(3), at 30 + 120 j degrees).  The c axis is the normal
    (last) grid axis; in 2D the second basal axis is not resolved and its
    component is dropped."""
    out = []
    for k in range(6):
        a = math.radians(60.0 * k)
        out.append((math.cos(a), math.sin(a), 0.0))
    for h in (1.0, -1.0):
        for j in range(3):
            a = math.radians(30.0 + 120.0 * j)
            out.append((math.cos(a) / math.sqrt(3.0), math.sin(a) / math.sqrt(3.0), h * math.sqrt(2.0 / 3.0)))
    return [u if ndim == 3 else (u[0], u[2], 0.0) for u in out]


def pair_force(theta: dict, n_floor: float, g_clamp: float, n_p, Gp, hcp: bool = False):
    """Eq. (1)-(3) per atom, in newtons; zero where n <= n_floor.  theta holds
    D, r0, s_rep, c_att and, for the Morse potential, alpha.  hcp: the 12
    neighbours of the hexagonal close-packed lattice instead of one pair per
    axis, each at the midpoint-rule distance 2^(1/6) rbar / (1 - q/2) along
    its direction u, q = 2^(1/6) grad(rbar).u (clamped); force = sum of the
    pair forces along u."""
    D, r0, s_rep, c_att = theta["D"], theta["r0"], theta["s_rep"], theta["c_att"]
    live = n_p > n_floor
    n_safe = torch.where(live, n_p, torch.ones_like(n_p) * max(n_floor, 1.0))
    rbar = n_safe ** (-1.0 / 3.0)

    def dphi(r):
        if "alpha" in theta:  # Morse: U' = 2 D alpha (e - e^2)
            e = torch.exp(-theta["alpha"] * (r - r0))
            du = 2.0 * D * theta["alpha"] * (e - e * e)
        else:
            x6 = (r0 / r) ** 6
            du = -(12.0 * D / r) * (x6 * x6 - x6)
        return torch.where(r < r0, s_rep * du, c_att * du)

    if hcp:
        c6 = 2.0 ** (1.0 / 6.0)
        grad = [(-1.0 / 3.0) * Gd * n_safe ** (-4.0 / 3.0) for Gd in Gp]  # eq. (1), unclamped
        F = [torch.zeros_like(rbar) for _ in Gp]
        for u in hcp_neighbours(len(Gp)):
            q = torch.clamp(c6 * sum(grad[d] * u[d] for d in range(len(Gp))), -g_clamp, g_clamp)
            f = dphi(c6 * rbar / (1.0 - 0.5 * q))
            F = [F[d] + f * u[d] for d in range(len(Gp))]
        return [torch.where(live, Fd, torch.zeros_like(Fd)) for Fd in F]
    F = []
    for Gd in Gp:
        g = (-1.0 / 3.0) * Gd * n_safe ** (-4.0 / 3.0)
        g = torch.clamp(g, -g_clamp, g_clamp)
        rp = rbar / (1.0 - 0.5 * g)
        rm = rbar / (1.0 + 0.5 * g)
        F.append(torch.where(live, dphi(rp) - dphi(rm), torch.zeros_like(rp)))
    return F


def forces(geo: Geometry, theta, n_floor, g_clamp, idx, f, w, hcp: bool = False):
    N = deposit(geo, idx, f, w)
    dens = density(geo, N)
    G = centre_gradient(geo, dens)
    n_p, Gp = gather(geo, dens, G, idx, f)
    return pair_force(theta, n_floor, g_clamp, n_p, Gp, hcp)


def push(geo: Geometry, dt: float, mass: float, F, idx, f, v):
    """Leapfrog kick and drift with carry, periodic wrap and mirror walls.
    v: list of 3 components; returns new (idx, f, v)."""
    nd = geo.ndim
    v = [v[d] + F[d] * (dt / mass) if d < nd else v[d] for d in range(3)]
    idx_new, f_new = [], []
    for d in range(nd):
        x = f[d] + v[d] * (dt / geo.h[d])
        xd = x.detach()
        n = geo.n[d]
        if geo.bc[d]:
            lo = (idx[d] == 0) & (xd < 0.0)
            hi = (idx[d] == n - 1) & (xd >= 1.0)
        else:
            lo = hi = torch.zeros_like(xd, dtype=torch.bool)
        up = (xd >= 1.0) & ~hi
        down = (xd < 0.0) & ~lo
        xn = torch.where(lo, -x, torch.where(hi, 2.0 - x, torch.where(up, x - 1.0, torch.where(down, x + 1.0, x))))
        i = idx[d] + up.long() - down.long()
        tie = down & (xn.detach() >= 1.0)  # x + 1 rounded to 1: the particle is on the node
        xn = torch.where(tie, torch.zeros_like(xn), xn)
        i = torch.where(tie, idx[d], i)
        hi_top = hi & (xn.detach() >= 1.0)
        xn = torch.where(hi_top, torch.full_like(xn, math.nextafter(1.0, 0.0)), xn)
        if not geo.bc[d]:
            i = torch.remainder(i, n)
        wall = lo | hi
        v[d] = torch.where(wall, -v[d], v[d])
        idx_new.append(i)
        f_new.append(xn)
    return idx_new, f_new, v


def step(geo, theta, n_floor, g_clamp, dt, mass, idx, f, v, w, hcp: bool = False):
    F = forces(geo, theta, n_floor, g_clamp, idx, f, w, hcp)
    return push(geo, dt, mass, F, idx, f, v)


def functional(geo: Geometry, idx, f, w, y_s: float, tau: float):
    ax = geo.ndim - 1
    y = (idx[ax].double() + f[ax]) * geo.h[ax]
    return (w * torch.sigmoid((y - y_s) / tau)).sum()


def unpack(grid, cell, off):
    """(cell ids, offsets [ndim, n]) -> per-axis index tensors and offset tensors."""
    geo = Geometry.of(grid)
    c = torch.as_tensor(cell, dtype=torch.int64)
    idx = []
    for d in range(geo.ndim):
        idx.append(c % geo.n[d])
        c = c // geo.n[d]
    f = [torch.as_tensor(off[d], dtype=torch.float64) for d in range(geo.ndim)]
    return geo, idx, f


def crater_objective(grid, pot, dt, nsteps, cell, off, v_thermal, xi, sigma_ref, fluence_ref, wq, y_s, tau,
                     theta=None, fluence=None, offsets_grad=False):
    """J after nsteps from the heated initial state v0 = v_th + sigma(F) xi with
    sigma proportional to sqrt(F); v(-1/2) = v0 - F(x0)/m dt/2.  Returns (J,
    theta dict, fluence tensor, final state, initial offsets); theta and
    fluence (and the initial offsets with offsets_grad) are leaves with grad."""
    hcp = getattr(pot, "lattice", 0) == 1
    geo, idx, f = unpack(grid, cell, off)
    if offsets_grad:
        f = [t.clone().requires_grad_(True) for t in f]
    f0 = f
    if theta is None:
        keys = ("D", "r0", "s_rep", "c_att") + (("alpha",) if pot.kind == 1 else ())
        theta = {k: torch.tensor(float(getattr(pot, k)), dtype=torch.float64, requires_grad=True) for k in keys}
    if fluence is None:
        fluence = torch.tensor(float(fluence_ref), dtype=torch.float64, requires_grad=True)
    w = torch.as_tensor(wq, dtype=torch.float64) * WUNIT
    scale = torch.sqrt(fluence / fluence_ref)
    sig = torch.as_tensor(sigma_ref, dtype=torch.float64) * scale
    v = [torch.as_tensor(v_thermal[d], dtype=torch.float64) + sig * torch.as_tensor(xi[d], dtype=torch.float64)
         for d in range(3)]
    F0 = forces(geo, theta, pot.n_floor, pot.g_clamp, idx, f, w, hcp)
    v = [v[d] - 0.5 * F0[d] * (dt / pot.mass) if d < geo.ndim else v[d] for d in range(3)]
    for _ in range(nsteps):
        idx, f, v = step(geo, theta, pot.n_floor, pot.g_clamp, dt, pot.mass, idx, f, v, w, hcp)
    J = functional(geo, idx, f, w, y_s, tau)
    return J, theta, fluence, (idx, f, v), f0
