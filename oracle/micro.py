"""Arbitrary-precision micro-oracle for one to three macroparticles.

TEST INFRASTRUCTURE ONLY.  A second, literal transcription of the PIC
pair-potential cycle in pure Python with ``mpmath`` at 50 significant digits,
written independently of the C oracle (dictionaries of node and centre values,
no shared helpers), for brute-force checks on tiny inputs: it enumerates the
nodes each particle touches, the node densities, the cell-centre gradients
around each particle, and evaluates eq. (1)-(3) of the paper directly.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50


class Micro:
    """grid: dict(ndim, n, h, bc, depth2d); pot: dict(D, r0, s_rep, c_att,
    g_clamp, n_floor, mass).  Particles: lists of (cell_index_tuple, offsets,
    velocity3, wq)."""

    def __init__(self, grid, pot, quantized=True):
        self.nd = grid["ndim"]
        self.n = list(grid["n"])[: self.nd]
        self.h = [mp.mpf(x) for x in list(grid["h"])[: self.nd]]
        self.bc = list(grid["bc"])[: self.nd]
        depth = mp.mpf(grid.get("depth2d", 0.0)) if self.nd == 2 else self.h[2]
        self.vol = self.h[0] * self.h[1] * depth
        self.pot = {k: mp.mpf(v) for k, v in pot.items()}
        self.quantized = quantized

    # --- node and centre bookkeeping -------------------------------------
    def wrap_node(self, a):
        out = []
        for d in range(self.nd):
            n, i = self.n[d], a[d]
            if self.bc[d] == 0:
                i = i % n
            else:
                if i < 0:
                    i = -i
                if i > n:
                    i = 2 * n - i
            out.append(i)
        return tuple(out)

    def node_volume(self, a):
        v = self.vol
        for d in range(self.nd):
            if self.bc[d] == 1 and a[d] in (0, self.n[d]):
                v = v / 2
        return v

    def corners(self):
        for k in range(2 ** self.nd):
            yield tuple((k >> d) & 1 for d in range(self.nd))

    # --- deposit -----------------------------------------------------------
    def shares(self, f, wq):
        """Weight units each of the 2^nd corner nodes receives."""
        out = {}
        if self.quantized:
            u = [min(65535, max(0, int(mp.floor(mp.mpf(fd) * 65536)))) for fd in f]
            parts = {(): int(wq)}
            for d in range(self.nd):
                nxt = {}
                for key, val in parts.items():
                    up = (val * u[d]) // 65536
                    nxt[key + (0,)] = val - up
                    nxt[key + (1,)] = up
                parts = nxt
            for key, val in parts.items():
                out[key] = mp.mpf(val)
        else:
            for b in self.corners():
                w = mp.mpf(int(wq))
                for d in range(self.nd):
                    w *= mp.mpf(f[d]) if b[d] else 1 - mp.mpf(f[d])
                out[b] = w
        return out

    def densities(self, parts):
        sums = {}
        for cell, f, _v, wq in parts:
            for b, val in self.shares(f, wq).items():
                a = self.wrap_node(tuple(cell[d] + b[d] for d in range(self.nd)))
                sums[a] = sums.get(a, mp.mpf(0)) + val
        unit = mp.mpf(2) ** -20
        return {a: s * unit / self.node_volume(a) for a, s in sums.items()}

    def dens_at(self, dens, a):
        return dens.get(self.wrap_node(a), mp.mpf(0))

    def centre_grad(self, dens, c, d):
        """Gradient component d at the centre of cell c (ghost centres beyond
        reflecting walls mirror the first interior centre, normal part negated)."""
        c = list(c)
        sign = 1
        for e in range(self.nd):
            if self.bc[e] == 1:
                if c[e] < 0:
                    c[e] = -1 - c[e]
                    sign = -sign if e == d else sign
                elif c[e] >= self.n[e]:
                    c[e] = 2 * self.n[e] - 1 - c[e]
                    sign = -sign if e == d else sign
        total = mp.mpf(0)
        cnt = 0
        for b in self.corners():
            if b[d]:
                continue
            lo = [c[e] + b[e] for e in range(self.nd)]
            hi = list(lo)
            hi[d] += 1
            total += self.dens_at(dens, tuple(hi)) - self.dens_at(dens, tuple(lo))
            cnt += 1
        return sign * total / (cnt * self.h[d])

    def gather(self, dens, cell, f):
        f = [mp.mpf(x) for x in f]
        n_p = mp.mpf(0)
        for b in self.corners():
            w = mp.mpf(1)
            for d in range(self.nd):
                w *= f[d] if b[d] else 1 - f[d]
            n_p += w * self.dens_at(dens, tuple(cell[d] + b[d] for d in range(self.nd)))
        base, t = [], []
        for d in range(self.nd):
            if f[d] >= mp.mpf("0.5"):
                base.append(cell[d])
                t.append(f[d] - mp.mpf("0.5"))
            else:
                base.append(cell[d] - 1)
                t.append(f[d] + mp.mpf("0.5"))
        G = []
        for d in range(self.nd):
            s = mp.mpf(0)
            for b in self.corners():
                w = mp.mpf(1)
                for e in range(self.nd):
                    w *= t[e] if b[e] else 1 - t[e]
                s += w * self.centre_grad(dens, tuple(base[e] + b[e] for e in range(self.nd)), d)
            G.append(s)
        return n_p, G

    # --- eq. (1)-(3) -------------------------------------------------------
    def dphi(self, r):
        P = self.pot
        u = -12 * P["D"] / r * ((P["r0"] / r) ** 12 - (P["r0"] / r) ** 6)
        return (P["s_rep"] if r < P["r0"] else P["c_att"]) * u

    def force(self, n_p, G):
        P = self.pot
        if not n_p > P["n_floor"]:
            return [mp.mpf(0)] * self.nd
        rbar = n_p ** (-mp.mpf(1) / 3)
        F = []
        for d in range(self.nd):
            g = -G[d] * n_p ** (-mp.mpf(4) / 3) / 3
            g = max(-P["g_clamp"], min(P["g_clamp"], g))
            F.append(self.dphi(rbar / (1 - g / 2)) - self.dphi(rbar / (1 + g / 2)))
        return F

    def forces(self, parts):
        dens = self.densities(parts)
        out = []
        for cell, f, _v, _w in parts:
            n_p, G = self.gather(dens, cell, f)
            out.append(self.force(n_p, G))
        return out

    def step(self, parts, dt):
        """One leapfrog cycle; returns the new particle list."""
        dt = mp.mpf(dt)
        Fs = self.forces(parts)
        new = []
        for (cell, f, v, wq), F in zip(parts, Fs):
            cell, f, v = list(cell), [mp.mpf(x) for x in f], [mp.mpf(x) for x in v]
            for d in range(self.nd):
                v[d] += F[d] / self.pot["mass"] * dt
            for d in range(self.nd):
                x = f[d] + v[d] * dt / self.h[d]
                n = self.n[d]
                if self.bc[d] == 1 and cell[d] == 0 and x < 0:
                    x, v[d] = -x, -v[d]
                elif self.bc[d] == 1 and cell[d] == n - 1 and x >= 1:
                    x, v[d] = 2 - x, -v[d]
                else:
                    k = int(mp.floor(x))
                    x -= k
                    cell[d] += k
                    if self.bc[d] == 0:
                        cell[d] %= n
                f[d] = x
            new.append((tuple(cell), f, v, wq))
        return new
