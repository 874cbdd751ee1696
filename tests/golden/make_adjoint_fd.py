"""Writes adjoint_fd_16cube.json: central finite differences of the crater
functional J = sum_p w_p sigmoid((y_p(T) - y_s)/tau) computed by the FP64 C
oracle alone (unquantized deposit), on the 16^3-cell copy of the 3D adjoint
workload (x, y periodic, z reflecting, slab in the lower 8 layers, 8 ppc,
1.5 J/cm^2 heating, 400 steps of 1 fs).

Two potentials: the altered one (s_rep = 1, c_att = 0.27) for D, s_rep, c_att
and the fluence, and the unaltered one (s_rep = c_att = 1) for r0, whose
derivative jumps where a neighbour distance crosses r0 when the two branch
multipliers differ.  Each derivative is recorded at relative steps 1e-3 and
1e-4; their difference bounds the FD's own error.

With the argument `morse` it writes adjoint_fd_16cube_morse.json instead:
the same case with the Morse copper potential (altered: c_att = 0.43, for
D, s_rep, c_att, the Morse width alpha and the fluence; unaltered: c_att = 1,
for r0).  With `hcp`, adjoint_fd_16cube_hcp.json: L-J on the hexagonal
close-packed lattice (altered: c_att = 0.2; unaltered: c_att = 1); with
`hcp_morse`, adjoint_fd_16cube_hcp_morse.json: Morse on that lattice
(altered: c_att = 0.3, alpha included; unaltered: c_att = 1).

    python tests/golden/make_adjoint_fd.py [lj|morse|hcp|hcp_morse]
"""
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1502_07722_amd import workloads as W  # noqa: E402

NSTEPS = 400
FREF = 1.5e4


FAMILIES = {
    "lj": ("adjoint_fd_16cube.json",
           (("altered", W.Potential(c_att=0.27), ("D", "s_rep", "c_att", "F")),
            ("unaltered", W.Potential(c_att=1.0), ("r0",)))),
    "morse": ("adjoint_fd_16cube_morse.json",
              (("altered", W.morse_cu(c_att=0.43), ("D", "s_rep", "c_att", "alpha", "F")),
               ("unaltered", W.morse_cu(c_att=1.0), ("r0",)))),
    "hcp": ("adjoint_fd_16cube_hcp.json",
            (("altered", W.hcp(c_att=0.2), ("D", "s_rep", "c_att", "F")),
             ("unaltered", W.hcp(c_att=1.0), ("r0",)))),
    "hcp_morse": ("adjoint_fd_16cube_hcp_morse.json",
                  (("altered", W.hcp(W.morse_cu(), c_att=0.3), ("D", "s_rep", "c_att", "alpha", "F")),
                   ("unaltered", W.hcp(W.morse_cu(), c_att=1.0), ("r0",)))),
}


def main(family="lj"):
    fname, cases = FAMILIES[family]
    wl = W.cfg_adjoint_3d(n=16, layers=8)
    g, p = wl.grid, wl.parts
    y_s = wl.slab_rows * g.h[2]
    tau = g.h[2]

    def J_of(pot, F=FREF):
        return O.crater_objective(g, pot, wl.dt, NSTEPS, p.cell, p.off, p.v_thermal, p.xi, p.sigma, FREF, F,
                                  p.wq, y_s, tau)

    out = {"case": "cfg_adjoint_3d(n=16, layers=8)", "particles": int(p.n), "nsteps": NSTEPS, "dt": wl.dt,
           "fluence": FREF, "y_s": y_s, "tau": tau, "potentials": {}}
    t0 = time.time()
    for name, pot, keys in cases:
        rec = {"D": pot.D, "r0": pot.r0, "s_rep": pot.s_rep, "c_att": pot.c_att}
        if pot.kind == W.KIND_MORSE:
            rec.update(kind=pot.kind, alpha=pot.alpha)
        if pot.lattice == W.LATTICE_HCP:
            rec.update(lattice=pot.lattice)
        rec.update(J=J_of(pot), dJ={})
        for k in keys:
            vals = {}
            for rel in (1e-3, 1e-4):
                if k == "F":
                    h = rel * FREF
                    vals[str(rel)] = (J_of(pot, FREF + h) - J_of(pot, FREF - h)) / (2 * h)
                else:
                    x = getattr(pot, k)
                    h = rel * x
                    vals[str(rel)] = (J_of(dataclasses.replace(pot, **{k: x + h}))
                                      - J_of(dataclasses.replace(pot, **{k: x - h}))) / (2 * h)
                print(name, k, rel, vals[str(rel)], f"{time.time() - t0:.0f}s", flush=True)
            rec["dJ"][k] = vals
        out["potentials"][name] = rec
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), fname), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "lj")
