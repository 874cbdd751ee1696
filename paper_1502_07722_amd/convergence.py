"""Convergence of the method in particles per cell and in cell size, and the
large-s_rep limit of the altered potential with quiet-start loading.

The paper states (results section) that its transport runs at 10 nm cells,
12 fs steps and 3600 particles per cell were numerically converged, and it
takes the repulsive branch of eq. (3) to an unbounded wall below r0.  These
studies run the same laser-heated copper slab (same physical box, slab,
heating and time) through the library at several resolutions and report how
much each observable still moves against the finest setting:

* ke_ratio   kinetic energy at the end over that after the heating kick;
* drift      (E_end - E_start) / KE_start, E = KE + grid energy (the
             paper's energy-conservation claim);
* deficit_nm mean missing thickness (y_s minus the column's equivalent
             solid thickness, 1 % cut-off) over the columns within the
             beam's 1/e^2 radius;
* rho_max    largest node density at the end, units of solid density.

Every step of every run is the library's fused step (pic_step); the
observables come from its FP64 diagnostics and from pic_crater.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import binding as B
from . import workloads as W


@dataclasses.dataclass
class Case:
    h_nm: float                  # cell edge
    ppc: int                     # macroparticles per slab cell
    box_nm: tuple = (640.0, 320.0)
    slab_nm: float = 160.0
    fluence_Jcm2: float = 3.0
    R_nm: float = 200.0          # 1/e^2 radius of the heating profile
    steps: int = 2000
    dt: float = 1e-15
    s_rep: float = 1.0
    quiet: float = -1.0          # quiet-start jitter (-1: uniform-random offsets)
    depth_nm: float = 0.5        # 2D thickness the plane stands for: keeps a macroparticle's
                                 # weight below the 2^11 atoms of the fixed-point format at
                                 # 10 nm cells and 4 ppc (the density does not depend on it)
    seed: int = 7

    @property
    def label(self):
        q = f", quiet {self.quiet:g}" if self.quiet >= 0 else ""
        t = f", dt {self.dt * 1e15:.3g} fs" if self.dt != 1e-15 else ""
        return f"h {self.h_nm:g} nm, {self.ppc} ppc, s_rep {self.s_rep:g}{q}{t}"


def _cells(case):
    nx = int(round(case.box_nm[0] / case.h_nm))
    ny = int(round(case.box_nm[1] / case.h_nm))
    layers = int(round(case.slab_nm / case.h_nm))
    return nx, ny, layers


def run_case(case: Case, device="cuda:0", stream=None, log_fn=None) -> dict:
    nx, ny, layers = _cells(case)
    h = case.h_nm * 1e-9
    t0 = time.perf_counter()
    grid, parts = W.make_slab(2, (nx, ny), layers, case.ppc, h, case.seed, fluence_Jcm2=case.fluence_Jcm2,
                              R_cells=case.R_nm / case.h_nm, quiet=case.quiet, depth2d=case.depth_nm * 1e-9)
    t_gen = time.perf_counter() - t0
    base = W.Potential(s_rep=case.s_rep)
    c_att, _ = B.pic_calibrate_catt(grid, base, W.N_SOLID, 8)
    pot = dataclasses.replace(base, c_att=c_att)
    stream = stream or torch.cuda.Stream(device=device)
    with torch.cuda.stream(stream):
        ctx = B.Context(grid, pot, case.dt, parts.n, device=device, stream=stream)
        dp = B.DeviceParticles.from_host(parts, device)
        ctx.start_leapfrog(dp)
        every = max(case.steps // 10, 1)
        stream.synchronize()
        t1 = time.perf_counter()
        diags = ctx.pic_step(dp, case.steps, every)
        stream.synchronize()
        elapsed = time.perf_counter() - t1
        nodes = ctx.pic_step_nodes()
        y_s = layers * h
        res, col_w, rho = ctx.pic_crater(nodes, W.N_SOLID, y_s, 0.01, 0.5 * h, want_rho=True)
        col = col_w.cpu().numpy()
        rho_max = float(rho.max().item())
    t = col * 2.0 ** -20 / (W.N_SOLID * h * grid.depth2d)
    x = (np.arange(nx) - nx / 2.0) * h
    spot = np.abs(x) <= case.R_nm * 1e-9
    out = {
        "case": case.label, "h_nm": case.h_nm, "ppc": case.ppc, "s_rep": case.s_rep, "quiet": case.quiet,
        "cells": [nx, ny], "particles": parts.n, "steps": case.steps, "c_att": c_att,
        "ke_ratio": diags[-1]["ke"] / diags[0]["ke"],
        "drift": (diags[-1]["ke"] + diags[-1]["pe"] - diags[0]["ke"] - diags[0]["pe"]) / diags[0]["ke"],
        "deficit_nm": float(np.mean(y_s - t[spot])) * 1e9,
        "rho_max": rho_max, "crater_depth_nm": res[0]["depth"] * 1e9,
        "particle_steps_per_s": parts.n * case.steps / elapsed, "generate_s": t_gen,
    }
    if log_fn:
        log_fn(f"convergence {case.label}: {parts.n} particles, ke_ratio {out['ke_ratio']:.5f}, drift "
               f"{out['drift']:.2e}, deficit {out['deficit_nm']:.3f} nm, rho_max {rho_max:.3f}, "
               f"{out['particle_steps_per_s']:.2e} particle-steps/s")
    del ctx, dp
    return out


OBSERVABLES = ("ke_ratio", "drift", "deficit_nm", "rho_max")


def _against_finest(rows: List[dict], finest: int) -> None:
    ref = rows[finest]
    for r in rows:
        r["diff_vs_finest"] = {k: r[k] - ref[k] for k in OBSERVABLES}


def study_ppc(ppcs=(4, 16, 64, 256, 1024, 3600), h_nm=10.0, steps=2000, log_fn=None) -> List[dict]:
    """Particles per cell at the paper's 10 nm cells, up to its 3600."""
    rows = [run_case(Case(h_nm=h_nm, ppc=p, steps=steps), log_fn=log_fn) for p in ppcs]
    _against_finest(rows, len(rows) - 1)
    return rows


def study_cell(hs=(10.0, 8.0, 5.0, 4.0, 2.0), ppc=64, steps=2000, log_fn=None) -> List[dict]:
    """Cell size at fixed particles per cell (the calibration of c_att
    follows the cell size)."""
    rows = [run_case(Case(h_nm=h, ppc=ppc, steps=steps), log_fn=log_fn) for h in hs]
    _against_finest(rows, len(rows) - 1)
    return rows


def study_srep(s_reps=(1.0, 2.0, 4.0, 8.0, 16.0, 32.0), h_nm=4.0, ppc=64, quiet=0.5, steps=2000,
               log_fn=None, scale_dt=False) -> List[dict]:
    """The repulsive multiplier towards the paper's unbounded wall, with
    quiet-start loading (8 x 8 sub-lattice, half a sub-spacing of jitter).
    scale_dt: the time step shrinks as 1 / sqrt(s_rep) (the stiffer branch's
    oscillation period) over the same physical time."""
    rows = []
    for s in s_reps:
        k = math.sqrt(s) if scale_dt else 1.0
        case = Case(h_nm=h_nm, ppc=ppc, s_rep=s, quiet=quiet, steps=int(round(steps * k)), dt=1e-15 / k)
        rows.append(run_case(case, log_fn=log_fn))
        rows[-1]["dt"] = case.dt
    _against_finest(rows, len(rows) - 1)
    return rows


def run_all(steps=2000, log_fn=None, small: Optional[bool] = False) -> dict:
    if small:  # a quick pass with the same structure
        return {"ppc": study_ppc((4, 16), steps=steps, log_fn=log_fn),
                "cell": study_cell((10.0, 5.0), steps=steps, log_fn=log_fn),
                "s_rep": study_srep((1.0, 4.0), steps=steps, log_fn=log_fn),
                "s_rep_dt": study_srep((1.0, 4.0), steps=steps, log_fn=log_fn, scale_dt=True)}
    return {"ppc": study_ppc(steps=steps, log_fn=log_fn), "cell": study_cell(steps=steps, log_fn=log_fn),
            "s_rep": study_srep(steps=steps, log_fn=log_fn),
            "s_rep_dt": study_srep((1.0, 4.0, 16.0, 32.0), steps=steps, log_fn=log_fn, scale_dt=True)}
