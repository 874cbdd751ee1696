"""Shared checks of the FP64 diagnostics of a GPU run against the oracle's
(imported by the GPU parity tests; holds no arithmetic of the method).

Bars, per diagnostic step (the norms of the 100-step state bar):
  - kinetic, grid potential and bond energy: 1e-4 relative;
  - momentum per component: 1e-4 of sum |w m v_d| (momentum itself may be
    near zero, so its scale is the sum of the magnitudes it is made of);
  - weight sum: 1e-12 relative (the same integers on both sides).
"""
import numpy as np

W_UNIT = 2.0 ** -20


def momentum_scale(parts, mass):
    w = parts.wq.astype(np.float64) * W_UNIT
    return (w * mass * np.abs(parts.vel.astype(np.float64))).sum(axis=1)


def check_diagnostics(gd, od, parts, mass, tol=1e-4):
    assert len(gd) == len(od) and len(gd) > 0
    ps = momentum_scale(parts, mass)
    worst = {"p": 0.0, "bond": 0.0}
    for a, b in zip(gd, od):
        assert a["step"] == b["step"]
        assert abs(a["wsum"] - b["wsum"]) <= 1e-12 * abs(b["wsum"])
        for k in ("ke", "pe", "bond"):
            assert abs(a[k] - b[k]) <= tol * abs(b[k]), (k, a["step"], a[k], b[k])
        worst["bond"] = max(worst["bond"], abs(a["bond"] - b["bond"]) / abs(b["bond"]))
        for d, k in enumerate(("px", "py", "pz")):
            err = abs(a[k] - b[k])
            assert err <= tol * ps[d], (k, a["step"], a[k], b[k], ps[d])
            worst["p"] = max(worst["p"], err / ps[d])
    return worst
