"""Writes the stored expected values under tests/golden/ from the 50-digit
micro-oracle only (oracle/micro.py).  Run: python tests/golden/make_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.micro import Micro  # noqa: E402

H = 2e-9
GRID = dict(ndim=2, n=(5, 4), h=(H, 1.25 * H, H), bc=(0, 1, 0), depth2d=H)
POT = dict(D=0.4093 * 1.602176634e-19, r0=8.49e28 ** (-1.0 / 3.0), s_rep=2.0, c_att=0.4,
           g_clamp=1.0, n_floor=8.49e22, mass=63.546 * 1.66053906660e-27)
PARTS = [((1, 0), ["0.3125", "0.0625"], ["150.0", "-420.0", "33.0"], 44511724),
         ((2, 1), ["0.8125", "0.5"], ["-90.0", "210.0", "-5.0"], 22255862),
         ((4, 3), ["0.0", "0.96875"], ["310.0", "95.0", "0.0"], 33554432)]


def main():
    out = {}
    for q in (True, False):
        m = Micro(GRID, POT, quantized=q)
        parts = [(c, [float(x) for x in f], [float(x) for x in v], w) for c, f, v, w in PARTS]
        F = m.forces(parts)
        new = m.step(parts, 1e-15)
        out["quantized" if q else "exact"] = dict(
            force=[[str(x) for x in Fi] for Fi in F],
            cell=[list(p[0]) for p in new],
            off=[[str(x) for x in p[1]] for p in new],
            vel=[[str(x) for x in p[2]] for p in new])
    doc = dict(source="oracle/micro.py at 50 significant digits (brute force, 3 particles)",
               grid=GRID, pot=POT, dt=1e-15,
               particles=[dict(cell=list(c), off=f, vel=v, wq=w) for c, f, v, w in PARTS],
               result=out)
    with open(os.path.join(HERE, "micro_three_particles_2d.json"), "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
