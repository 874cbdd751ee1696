"""Checkpoint and resume of a run's particle state.

The paper reuses the structure a finished run leaves behind to start another
one (results section: a few-shot study initialises the next laser-target
simulation from the resulting target).  A checkpoint holds what pic_step
carries between calls: cell, offsets, half-step velocities v(n - 1/2) and
fixed-point weights, plus the grid, the potential, the time step and the
step count, in a NumPy ``.npz`` file of plain arrays (no pickled objects:
it loads with ``allow_pickle=False``).

Because node sums are exact integers and each particle is advanced from its
own state, N steps in one call and K steps, save, load, N - K steps give the
same bits (the internal binning is rebuilt on import and does not affect
results).  Resume with pic_step directly; the state is already leapfrogged.
"""
from __future__ import annotations

import dataclasses
import json

import numpy as np

from . import workloads as W

FORMAT = "pic-checkpoint-1"


def _host_arrays(parts):
    if hasattr(parts, "to_host"):  # DeviceParticles
        return parts.to_host()
    return parts.cell, parts.off, parts.vel, parts.wq


def save_state(path, parts, grid: W.Grid, pot: W.Potential, dt: float, step: int, meta: dict | None = None):
    """Write the particle state (device or host arrays) and its run settings."""
    cell, off, vel, wq = _host_arrays(parts)
    header = {"format": FORMAT, "grid": dataclasses.asdict(grid), "potential": dataclasses.asdict(pot),
              "dt": float(dt), "step": int(step), "meta": meta or {}}
    np.savez(path, cell=np.ascontiguousarray(cell, dtype=np.int32), off=np.ascontiguousarray(off, dtype=np.float32),
             vel=np.ascontiguousarray(vel, dtype=np.float32), wq=np.ascontiguousarray(wq, dtype=np.int32),
             header=np.array(json.dumps(header)))


def load_state(path):
    """(host Particles, grid, potential, dt, step, meta) from a checkpoint."""
    with np.load(path, allow_pickle=False) as z:
        header = json.loads(str(z["header"]))
        if header.get("format") != FORMAT:
            raise ValueError(f"{path}: not a {FORMAT} file")
        parts = W.Particles(cell=z["cell"].copy(), off=z["off"].copy(), vel=z["vel"].copy(), wq=z["wq"].copy())
    g = header["grid"]
    grid = W.Grid(ndim=g["ndim"], n=tuple(g["n"]), h=tuple(g["h"]), bc=tuple(g["bc"]), depth2d=g["depth2d"])
    pot = W.Potential(**header["potential"])
    return parts, grid, pot, header["dt"], header["step"], header["meta"]


def write_diagnostics(path, diags, step0: int = 0, every: int = 1, meta: dict | None = None):
    """Append pic_step's FP64 diagnostics to a JSON-lines log, one line per
    diagnostic step (the step index of the run, energies, momentum, weight)."""
    with open(path, "a") as fh:
        for i, d in enumerate(diags):
            rec = {"step": step0 + i * every, **{k: d[k] for k in d if k != "step"}}
            if meta:
                rec.update(meta)
            fh.write(json.dumps(rec) + "\n")
