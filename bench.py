"""Benchmark of the PIC pair-potential cycle on one MI355X.

One "step" is one full pass of the method over all particles: deposit ->
density and gradient -> gather -> eq. (1)-(3) force -> leapfrog push (plus
the FP64 diagnostics reductions every 100 steps, and on the first and the
last step of shorter runs).  The timed region is one pic_step(K) call with
the particles already resident in HBM: import into the binned store, K
steps, export back to the caller's arrays.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload large|heated|small]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one launch of the dominant (fused) kernel: each
# particle's state read once and written once -- reads cell 4 + offsets
# 4*ndim + velocity 12 + weight 4, writes cell 4 + offsets 4*ndim + velocity
# 12: 52 B in 2D, 60 B in 3D -- plus 16 B per node (int64 sums written once
# and read once).
DEFAULTS = {"large": (2000, 20), "large_morse": (500, 20), "convergence": (5000, 0), "heated": (5000, 20), "small": (200, 20), "sweep": (1000, 12), "adjoint": (400, 1)}


COUNTERS = {"large": "profiles/k_step_tiled_slab2d_4096x2048_32ppc.counters.json"}


def measured_traffic(workload):
    """HBM bytes per launch of the fused kernel from the committed FETCH_SIZE /
    WRITE_SIZE runs (scaled by a plain copy kernel), or None when there are no
    counters for this workload or the kernel's sources changed since."""
    import hashlib
    name = COUNTERS.get(workload)
    if name is None or not os.path.exists(os.path.join(ROOT, name)):
        return None
    with open(os.path.join(ROOT, name)) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(f.encode())
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def diag_period(steps):
    """FP64 diagnostics every 100 steps, and at least on the first and the
    last step of a run (a 20-step run has them on steps 0 and 19)."""
    return max(1, min(100, steps - 1))


TUNE_AFTER = 12  # steps a copy of the start state runs before the autotuner probes it


def tune(ctx, state):
    """pic_autotune on a copy of the state advanced TUNE_AFTER steps: a freshly
    loaded slab has the same particle count in every tile, and the first
    moves change that (a chunk equal to the count then splits half the
    tiles into two items).  state: DeviceParticles, or a list for a batch."""
    if isinstance(state, list):
        probe = [s.clone() for s in state]
        ctx.pic_step_batch(probe, TUNE_AFTER)
    else:
        probe = state.clone()
        ctx.pic_step(probe, TUNE_AFTER)
    return ctx.pic_autotune(probe, 6)


def _finite(x):
    """JSON has no NaN: undetermined figures are reported as null."""
    return x if x == x and abs(x) != float("inf") else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """Host cores and CPU model (the CPU baseline's machine)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _time_oracle(g, pot, dt, cell, off, vel, wq, threads, seconds):
    """Particle-steps/s of the oracle's run on prepared arrays (advanced in
    place): one step to size the run, then as many steps as fit `seconds`."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    O.run(g, pot, dt, cell, off, vel, wq, 1, threads=threads, copy=False)
    t1 = time.perf_counter() - t0
    steps = max(1, min(20, int(seconds / max(t1, 1e-3))))
    t0 = time.perf_counter()
    O.run(g, pot, dt, cell, off, vel, wq, steps, threads=threads, copy=False)
    return cell.shape[0] * steps / (time.perf_counter() - t0), steps


def cpu_baseline(wl, pot, seconds_hint=10.0):
    """The FP64 oracle as it stands, timed on this host's cores: on all usable
    cores (its OpenMP build: particles and grid loops split over threads,
    integer node sums, so the state is the serial one's) on the whole slab,
    and single-threaded (the serial build the tests use) on a 256-column strip
    of the same slab through the beam centre, periodic in x.  Each leg runs
    about `seconds_hint` seconds after a one-step sizing run."""
    import numpy as np
    from paper_1502_07722_amd import workloads as W

    g, p = wl.grid, wl.parts
    host = host_info()
    threads = int(host["omp_num_threads"] or host["nproc"] or 1)
    full = (p.cell.copy(), p.off.astype(np.float64), p.vel.astype(np.float64))
    rate_all, steps_all = _time_oracle(g, pot, wl.dt, *full, p.wq, threads, seconds_hint)
    del full
    nx = g.n[0]
    width = min(256, nx)
    x0 = nx // 2 - width // 2
    i = p.cell.astype(np.int64) % nx
    rest = p.cell.astype(np.int64) // nx
    sel = (i >= x0) & (i < x0 + width)
    cell = ((i[sel] - x0) + width * rest[sel]).astype(np.int32)
    gs = W.Grid(ndim=g.ndim, n=(width,) + tuple(g.n[1:]), h=g.h, bc=g.bc, depth2d=g.depth2d)
    nsample = int(cell.shape[0])
    rate_1, steps_1 = _time_oracle(gs, pot, wl.dt, cell, np.ascontiguousarray(p.off[:, sel], dtype=np.float64),
                                   np.ascontiguousarray(p.vel[:, sel], dtype=np.float64),
                                   np.ascontiguousarray(p.wq[sel]), 0, seconds_hint)
    return {"value": rate_all, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole slab ({p.n} particles), {steps_all} FP64 steps, {threads} OpenMP threads",
            "host": host,
            "single_thread": {"value": rate_1, "unit": "particle-steps/s", "cores": 1,
                              "sample": f"{width}x{g.n[1]}-cell strip of the same slab through the beam centre "
                                        f"({nsample} particles), {steps_1} FP64 steps"}}


def run_sweep(steps, warmup, log_fn=log):
    """The intensity sweep: 24 slabs of uneven size (0.2-5 J/cm^2).  Plain: a
    loop over the slabs, one context each, per-step launches, default tiles,
    no graph.  Batched: one context over all slabs, autotuned tiles, graph
    replay on a created stream.  Both start from the same state; their final
    states must be bit-identical."""
    import torch
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import workloads as W

    t0 = time.perf_counter()
    wls = W.cfg_sweep()
    N = sum(w.parts.n for w in wls)
    log_fn(f"sweep: {len(wls)} slabs, {N} particles, generated in {time.perf_counter() - t0:.1f} s")
    c_att, _ = B.pic_calibrate_catt(wls[0].grid, wls[0].pot, W.N_SOLID, 8)
    pot = W.Potential(c_att=c_att)
    dt = wls[0].dt
    # starting states: v(-1/2) from each slab's own force
    starts = []
    for w in wls:
        ctx = B.Context(w.grid, pot, dt, w.parts.n)
        dp = B.DeviceParticles.from_host(w.parts)
        ctx.start_leapfrog(dp)
        starts.append(dp)
        del ctx
    torch.cuda.synchronize()
    # plain loop
    plain_ctx = [B.Context(w.grid, pot, dt, w.parts.n) for w in wls]
    plain = [s.clone() for s in starts]
    for c, p in zip(plain_ctx, plain):
        c.pic_step(p, warmup)
    plain = [s.clone() for s in starts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, p in zip(plain_ctx, plain):
        c.pic_step(p, steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    del plain_ctx
    log_fn(f"plain loop: {steps} steps x {len(wls)} slabs in {t_plain:.3f} s")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bctx = B.BatchContext([w.grid for w in wls], pot, dt, [w.parts.n for w in wls], stream=stream)
        tuning = tune(bctx, starts)
        log_fn(f"autotuned tiling {tuning}")
        # plain loop with the batched run's tiling and graph replay on a created
        # stream: the gain from batching alone
        tctx = [B.Context(w.grid, pot, dt, w.parts.n, stream=stream) for w in wls]
        for c in tctx:
            c.pic_set_tile_shape(tuning["tile"], tuning["tile_last"], tuning["halo"], tuning["chunk"], -1)
        tuned = [s.clone() for s in starts]
        for c, p in zip(tctx, tuned):
            c.pic_step(p, warmup)
        tuned = [s.clone() for s in starts]
        stream.synchronize()
        t0 = time.perf_counter()
        for c, p in zip(tctx, tuned):
            c.pic_step(p, steps)
        stream.synchronize()
        t_tuned = time.perf_counter() - t0
        del tctx
        log_fn(f"plain loop, tuned tiles and graphs: {steps} steps x {len(wls)} slabs in {t_tuned:.3f} s")
        # batched
        batch = [s.clone() for s in starts]
        bctx.pic_step_batch(batch, warmup)
        batch = [s.clone() for s in starts]
        stream.synchronize()
        t0 = time.perf_counter()
        bctx.pic_step_batch(batch, steps)
        stream.synchronize()
        t_batch = time.perf_counter() - t0
        # crater of every slab at the end of the run and the threshold over the sweep
        ys = [w.slab_rows * w.grid.h[1] for w in wls]
        Fs = [w.fluence for w in wls]
        a = 2.0 ** 0.5 * 200.0 * W.H_CELL
        cr, _, _ = bctx.pic_crater(bctx.pic_step_nodes(), W.N_SOLID, ys, 0.01, 0.5 * W.H_CELL, Fs, [a] * len(wls))
        fixed, fit, a_fit = B.pic_threshold_fit(Fs, [r["width"] for r in cr], a)
    log_fn(f"batched: {steps} steps in {t_batch:.3f} s")
    same = all(torch.equal(a.cell, b.cell) and torch.equal(a.off, b.off) and torch.equal(a.vel, b.vel)
               for a, b in zip(plain, batch))
    same = same and all(torch.equal(a.cell, b.cell) and torch.equal(a.off, b.off) and torch.equal(a.vel, b.vel)
                        for a, b in zip(tuned, batch))
    roof = 1.0 / (52 * N + 16 * sum(B.pic_num_nodes(w.grid) for w in wls)) * HBM_PEAK_GBS * 1e9 * N
    return {"workload": f"sweep of {len(wls)} slabs, widths 256-2048, depths 128-512 rows, 16-32 ppc, "
                        f"0.2-5 J/cm^2, {steps} steps",
            "particles": N, "steps": steps,
            "plain_particle_steps_per_s": N * steps / t_plain,
            "plain_tuned_particle_steps_per_s": N * steps / t_tuned,
            "batched_particle_steps_per_s": N * steps / t_batch,
            "speedup": t_plain / t_batch, "speedup_over_tuned_plain": t_tuned / t_batch,
            "roofline_particle_steps_per_s": roof,
            "speedup_bound": {"value": roof / (N * steps / t_plain),
                              "note": "batched at 100 % of the 8 TB/s roofline (52 B per particle + 16 B per "
                                      "node per step) over the measured plain loop: no batching can pass it"},
            "plain": "one context per slab, per-step launches, default tiles, no graph",
            "plain_tuned": "one context per slab on a created stream, the batched run's tiling, graph replay",
            "bit_identical": bool(same), "tuning": tuning,
            "slab_particles": [w.parts.n for w in wls],
            "crater_end_of_run": {"note": f"after {steps} fs the surface has not settled: the measurement path, "
                                          "not a threshold claim",
                                  "width_m": [r["width"] for r in cr], "depth_m": [r["depth"] for r in cr],
                                  "f_th_fixed_Jm2": _finite(fixed), "f_th_fit_Jm2": _finite(fit),
                                  "beam_d_fit_m": _finite(a_fit)}}


def run_adjoint(log_fn=log, every=20, steps=None, potential="lj", all_states=None):
    """The 3D adjoint workload: 128^3 cells of 2 nm, slab in the lower 64
    layers, 8 ppc, 1.5 J/cm^2, 400 steps.  Forward = pic_step over the 400
    steps from v(-1/2).  Gradient = torch.autograd through the crater
    functional: recorded forward (checkpoints every 20 steps, where the run
    may re-bin) + reverse sweep + the start and heating terms.
    all_states: the record keeps every state and node sum (each recorded step
    writes its output there; the sweep is the reverse steps alone, no segment
    recompute); None = when the record fits the free device memory with
    16 GiB to spare (the 400-step record is about 100 GB).
    potential: "lj" (eq. (3)), "morse" (Morse copper, alpha a parameter) or
    "hcp" (eq. (3) on the hexagonal close-packed lattice)."""
    import numpy as np
    import torch
    from paper_1502_07722_amd import autograd as A
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import workloads as W

    t0 = time.perf_counter()
    wl = W.cfg_adjoint_3d()
    g, p = wl.grid, wl.parts
    log_fn(f"adjoint workload {wl.name}: {p.n} particles, generated in {time.perf_counter() - t0:.1f} s")
    base = {"lj": wl.pot, "morse": W.morse_cu(), "hcp": W.hcp()}[potential]
    c_att, _ = B.pic_calibrate_catt(g, base, W.N_SOLID, 8)
    pot = dataclasses.replace(base, c_att=c_att)
    nsteps = wl.steps if steps is None else steps
    dev = torch.device("cuda:0")
    cell = torch.from_numpy(p.cell).to(dev)
    off0 = torch.from_numpy(p.off).to(dev)
    vth = torch.from_numpy(p.v_thermal).to(dev)
    xi = torch.from_numpy(p.xi).to(dev)
    sig = torch.from_numpy(p.sigma.astype(np.float32)).to(dev)
    wq = torch.from_numpy(p.wq).to(dev)
    # both the forward and the gradient run on a created stream (the forward
    # replays plain steps as HIP graphs there) with autotuned tiles
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = B.Context(g, pot, wl.dt, p.n, device=dev, stream=stream)
    y_s = wl.slab_rows * g.h[2]
    tau = g.h[2]
    fref = wl.fluence
    # plain forward: the same start state, pic_step over nsteps
    dp = B.DeviceParticles(cell.clone(), off0.clone(), (vth + sig[None, :] * xi).contiguous(), wq)
    ctx.start_leapfrog(dp)
    tuning = tune(ctx, dp)
    log_fn(f"adjoint workload: autotuned tiling {tuning}")
    if all_states is None:
        ctx.pic_set_record_states(True)
        need = B.lib.pic_record_bytes(ctx.ctx, nsteps, every) + B.lib.pic_backward_bytes(ctx.ctx, every)
        free, _ = torch.cuda.mem_get_info(dev)
        all_states = need + (16 << 30) <= free
        log_fn(f"adjoint workload: a record of every state needs {need / 1e9:.1f} GB, {free / 1e9:.1f} GB free")
    ctx.pic_set_record_states(all_states)
    record_bytes = B.lib.pic_record_bytes(ctx.ctx, nsteps, every)
    warm = dp.clone()
    ctx.pic_step(warm, nsteps)  # the same run once untimed: every graph captured
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.pic_step(dp, nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del warm

    def grad_once():
        theta = A.theta_of(pot).requires_grad_(True)
        fl = torch.tensor(fref, dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        J, _, _ = A.crater_objective(ctx, cell, off0, vth, xi, sig, fref, fl, wq, theta, nsteps, every, y_s, tau)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        return J.item(), theta.grad.cpu().numpy(), fl.grad.item(), tb - ta, tc - tb

    grad_once()  # warm-up (allocations, code objects)
    J, gth, gF, t_rec, t_bwd = grad_once()
    log_fn(f"adjoint: forward {t_fwd * 1e3:.1f} ms, recorded forward {t_rec * 1e3:.1f} ms, "
           f"backward {t_bwd * 1e3:.1f} ms")
    step_bytes = 60 * p.n + 16 * B.pic_num_nodes(g)  # 3D algorithmic bytes per step
    fwd_gbs = step_bytes * nsteps / t_fwd / 1e9
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream(dev))
    del ctx
    torch.cuda.empty_cache()
    return {"workload": f"{wl.name}: 128^3 cells, slab 64 layers, 8 ppc, 1.5 J/cm^2, {nsteps} steps, "
                        f"checkpoint every {every}" + {"lj": "", "morse": ", Morse potential",
                                                       "hcp": ", hexagonal lattice"}[potential],
            "potential": {"lj": "lennard-jones", "morse": "morse", "hcp": "lennard-jones, hcp"}[potential],
            "c_att": c_att,
            "particles": int(p.n), "steps": nsteps, "checkpoint_every": every,
            "record": ("every state and node sum (no recompute)" if all_states
                       else "checkpoints (segments recomputed)") + f", {record_bytes / 1e9:.1f} GB",
            "tiling": tuning, "forward_s": t_fwd, "recorded_forward_s": t_rec, "backward_s": t_bwd,
            "adjoint_over_forward": t_bwd / t_fwd, "gradient_over_forward": (t_rec + t_bwd) / t_fwd,
            "forward_particle_steps_per_s": p.n * nsteps / t_fwd,
            "forward_roofline": {"achieved_gbs": fwd_gbs, "frac": fwd_gbs / HBM_PEAK_GBS,
                                 "basis": "60 B/particle + 16 B/node per step, whole step"},
            "J": J, "dJ_dtheta": {k: float(v) for k, v in zip(A.THETA_KEYS, gth)}, "dJ_dfluence": gF}


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (read + write bytes per second) of a plain
    1 GiB copy on this GPU: the practical HBM ceiling beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def measure_crater(ctx, wl, stream, log_fn=log, calls=20):
    """Crater measurement (density map with the 1 % cut-off, column sums,
    depth, width, eq. 5) on the node sums of the last pic_step, timed with
    HIP events on the context's stream over back-to-back calls."""
    import torch
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import workloads as W

    g = wl.grid
    ax = g.ndim - 1
    nodes = ctx.pic_step_nodes()
    bufs = ctx.crater_buffers(want_rho=True)
    y_s = wl.slab_rows * g.h[ax]
    beam_d = 2.0 ** 0.5 * 200.0 * g.h[0]  # 1/e diameter of the heating profile (1/e^2 radius 200 cells)
    args = (nodes, W.N_SOLID, y_s, 0.01, 0.5 * g.h[ax], wl.fluence or None, beam_d if wl.fluence else None, bufs)
    for _ in range(3):
        ctx.pic_crater_launch(*args)
    # the calls are captured into one graph so that host-side argument
    # marshalling does not leave the GPU idle between them
    graph = torch.cuda.CUDAGraph()
    stream.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(calls):
            ctx.pic_crater_launch(*args)
    graph.replay()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    graph.replay()
    b.record(stream)
    b.synchronize()
    us = a.elapsed_time(b) / calls * 1e3
    ctx.pic_crater_launch(*args)  # eager call: the results below come from it
    res = ctx.crater_results(bufs[2])[0]
    nn, nc = B.pic_num_nodes(g), B.pic_num_columns(g)
    nbytes = 12 * nn + 24 * nc  # node sums read, float map written; column sums cleared, added, read
    gbs = nbytes / (us * 1e-6) / 1e9
    log_fn(f"crater: {us:.1f} us per call, {gbs:.0f} GB/s; {res}")
    return {"result": res, "us_per_call": us, "bytes_per_call": nbytes, "achieved_gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "basis": "12 B per node + 24 B per column; clear + column pass + reduction",
            "y_s": y_s, "beam_d": beam_d}


def run_slab(name, steps, warmup, log_fn=log, variant="lj"):
    """One single-slab workload through pic_step: (result, workload, potential,
    diagnostics).  The timed region is one pic_step call of `steps` steps
    with diagnostics every 100 steps, particles resident in HBM.  variant:
    "lj" (eq. (3), cubic lattice), "morse" (the Morse copper potential) or
    "hcp" (eq. (3) on the hexagonal close-packed lattice)."""
    import numpy as np
    import torch
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import workloads as W

    t0 = time.perf_counter()
    wl = W.WORKLOADS[name]()
    log_fn(f"generated {wl.name}: {wl.parts.n} particles in {time.perf_counter() - t0:.1f} s")
    base = {"lj": wl.pot, "morse": W.morse_cu(), "hcp": W.hcp()}[variant]
    c_att, _ = B.pic_calibrate_catt(wl.grid, base, W.N_SOLID, 8)
    pot = dataclasses.replace(base, c_att=c_att)
    N = wl.parts.n
    diag_every = diag_period(steps)
    dev = torch.device("cuda:0")
    # a created stream: plain steps replay as HIP graphs there
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        dp = B.DeviceParticles.from_host(wl.parts, dev)
        ctx = B.Context(wl.grid, pot, wl.dt, N, device=dev, stream=stream)
        ctx.start_leapfrog(dp)
        tuning = tune(ctx, dp)
        log_fn(f"{wl.name}: autotuned tiling {tuning}")
        start = dp.clone()
        if warmup:
            ctx.pic_step(dp, warmup, diag_every)
        dp = start.clone()
        stream.synchronize()
        log_fn(f"{wl.name}: timing {steps} steps")
        t0 = time.perf_counter()
        diags = ctx.pic_step(dp, steps, diag_every)
        stream.synchronize()
        elapsed = time.perf_counter() - t0
        # the same run again with HIP events on every launch (no graphs):
        # the fused kernel's average duration for the roofline
        dp = start.clone()
        ctx.pic_set_timing(True)
        stream.synchronize()
        t1 = time.perf_counter()
        ctx.pic_step(dp, steps, diag_every)
        stream.synchronize()
        elapsed_events = time.perf_counter() - t1
        timing = ctx.pic_get_timing()
        ctx.pic_set_timing(False)
        crater = measure_crater(ctx, wl, stream, log_fn)
    log_fn(f"{steps} steps in {elapsed:.3f} s (with per-launch events {elapsed_events:.3f} s); phases {timing}")
    nd = wl.grid.ndim
    bytes_per_particle = 4 + 4 * nd + 12 + 4 + 4 + 4 * nd + 12
    nnodes = B.pic_num_nodes(wl.grid)
    launch_bytes = bytes_per_particle * N + 16 * nnodes
    ms_fp, nfp = timing.get("force_push", (0.0, 0))
    avg_s = ms_fp / 1e3 / max(nfp, 1)
    achieved = launch_bytes / avg_s / 1e9 if nfp else None
    traffic = measured_traffic(name)
    roofline = {"bound": "hbm", "kernel": "k_step_tiled (fused gather+force+push+deposit)", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                "traffic": traffic,
                "traffic_gbs": traffic / avg_s / 1e9 if (traffic and nfp) else None,
                "bytes_per_launch": launch_bytes, "bytes_per_particle": bytes_per_particle,
                "bytes_per_node": 16, "avg_launch_ms": avg_s * 1e3,
                "phases_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in timing.items() if isinstance(v, tuple)},
                "drifters_last_step": timing.get("drifters_last"), "items_last_step": timing.get("items_last")}
    one_time_ms = sum(timing.get(k, (0.0, 0))[0] for k in ("import_export", "deposit"))
    roofline["whole_call"] = {
        "achieved": launch_bytes * steps / elapsed / 1e9, "frac": launch_bytes * steps / elapsed / 1e9 / HBM_PEAK_GBS,
        "unit": "GB/s", "one_time_ms": one_time_ms,
        "steady_particle_steps_per_s": N * steps / max(elapsed - one_time_ms * 1e-3, 1e-9),
        "basis": "algorithmic bytes x steps / the timed pic_step call (import into the binned store, first "
                 "deposit, steps, diagnostics, export); one_time_ms: import/export and first deposit (events)"}
    res = {"workload": wl.name + ("" if variant == "lj" else "_" + variant), "particles": N,
           "value": N * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
           "potential": {"lj": "lennard-jones, cubic", "morse": "morse, cubic", "hcp": "lennard-jones, hcp"}[variant],
           "elapsed_s": elapsed, "roofline": roofline, "c_att": c_att, "tiling": tuning,
           "ms_per_step_with_events": elapsed_events / steps * 1e3, "crater": crater, "diag_every": diag_every}
    del ctx, dp, start
    torch.cuda.empty_cache()
    return res, wl, pot, diags


def energy_check(diags):
    """Total energy KE + PE on the first and the last diagnostic step of the
    timed run, and its change relative to the first step's kinetic energy."""
    if len(diags) < 2:
        return None
    a, b = diags[0], diags[-1]
    Ea, Eb = a["ke"] + a["pe"], b["ke"] + b["pe"]
    return {"step_first": int(a["step"]), "step_last": int(b["step"]), "E_first": Ea, "E_last": Eb,
            "dE_over_KE0": (Eb - Ea) / a["ke"], "KE_first": a["ke"], "KE_last": b["ke"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="large",
                    choices=["large", "heated", "small", "sweep", "adjoint", "convergence"])
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the batched intensity sweep (plain loop vs batched) reported in the same line")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the 3D adjoint timing (gradient vs forward cost) reported in the same line")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the small and heated single-slab configs reported in the same line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the design notes describe how it would shard).", file=sys.stderr)
        sys.exit(2)
    steps = args.steps if args.steps is not None else DEFAULTS[args.workload][0]
    warmup = args.warmup if args.warmup is not None else DEFAULTS[args.workload][1]

    import numpy as np
    import torch
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import workloads as W

    if args.workload == "adjoint":
        res = run_adjoint(steps=args.steps)
        res["morse"] = run_adjoint(steps=args.steps, potential="morse")
        res["hcp"] = run_adjoint(steps=args.steps, potential="hcp")
        rec = "every state recorded" if res["record"].startswith("every") else "checkpoint every 20"
        out = {"metric": f"adjoint time / forward time ({res['steps']} steps, {rec})",
               "value": res["adjoint_over_forward"], "unit": "ratio", "n_gpus": 1, "steps": res["steps"],
               "warmup": 1, "ms_per_step": res["backward_s"] / res["steps"] * 1e3, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": res["workload"]}, "adjoint": res}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "convergence":
        from paper_1502_07722_amd import convergence as CV
        t0 = time.perf_counter()
        res = CV.run_all(steps=steps, log_fn=log)
        wall = time.perf_counter() - t0
        rows = [r for v in res.values() for r in v]
        ps = sum(r["particles"] * r["steps"] for r in rows)
        t_run = sum(r["particles"] * r["steps"] / r["particle_steps_per_s"] for r in rows)
        out = {"metric": "particle-steps/s (deposit+force+push), convergence studies",
               "value": ps / t_run, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": 0,
               "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32", "data": "synthetic",
               "config": {"workload": "convergence studies: ppc 4-3600 at 10 nm cells; cells 10-2 nm at 64 ppc; "
                                      "s_rep 1-32 with quiet start; 640x320 nm box, 160 nm slab, 3 J/cm^2"},
               "wall_s": wall, "convergence": res}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "sweep":
        res = run_sweep(steps, warmup)
        out = {"metric": "particle-steps/s (deposit+force+push), batched intensity sweep",
               "value": res["batched_particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
               "steps": steps, "warmup": warmup, "ms_per_step": None, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": res["workload"]}, "sweep": res}
        print(json.dumps(out), flush=True)
        return

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    res, wl, pot, diags = run_slab(args.workload, steps, warmup)
    value, N, nd, c_att = res["value"], wl.parts.n, wl.grid.ndim, res["c_att"]
    roofline = res["roofline"]
    ceiling = copy_ceiling()
    log(f"device copy ceiling {ceiling:.0f} GB/s")
    roofline["copy_ceiling_gbs"] = ceiling
    roofline["frac_of_copy"] = roofline["achieved"] / ceiling if roofline["achieved"] else None
    elapsed = res["elapsed_s"]
    out = {
        "metric": "particle-steps/s (deposit+force+push)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "particles": N, "cells": list(wl.grid.n[:nd]),
                   "ppc": int(round(N / (wl.slab_rows * np.prod(wl.grid.n[: nd - 1])))),
                   "dt_s": wl.dt, "diag_every": res["diag_every"], "c_att": c_att, "tiling": res["tiling"],
                   "state": "int32 cell + f32 offsets/velocities, int64 fixed-point deposit"},
        "roofline": roofline,
        "energy_check": energy_check(diags),
    }
    if args.workload == "large" and not args.no_configs:
        # the other single-slab configs, each with its own roofline fraction
        out["configs"] = {}
        for name in ("small", "heated"):
            r, _, _, _ = run_slab(name, *DEFAULTS[name])
            out["configs"][name] = {k: r[k] for k in ("workload", "particles", "value", "ms_per_step")}
            out["configs"][name]["roofline_frac"] = r["roofline"]["frac"]
            out["configs"][name]["roofline_achieved_gbs"] = r["roofline"]["achieved"]
        # the same large slab with the Morse pair potential and on the hexagonal
        # lattice (the paper names both as alternatives)
        for variant in ("morse", "hcp"):
            r, _, _, _ = run_slab("large", *DEFAULTS["large_morse"], variant=variant)
            key = "large_" + variant
            out["configs"][key] = {k: r[k] for k in ("workload", "particles", "value", "ms_per_step", "potential",
                                                      "c_att")}
            out["configs"][key]["roofline_frac"] = r["roofline"]["frac"]
            out["configs"][key]["roofline_achieved_gbs"] = r["roofline"]["achieved"]
    if not args.no_sweep and args.workload == "large":
        out["sweep"] = run_sweep(*DEFAULTS["sweep"])
    if not args.no_adjoint and args.workload == "large":
        out["adjoint"] = run_adjoint()
        out["adjoint"]["morse"] = run_adjoint(potential="morse")
        out["adjoint"]["hcp"] = run_adjoint(potential="hcp")
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, pot)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
