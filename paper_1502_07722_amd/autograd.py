"""torch.autograd bindings of the hand-written reverse mode.

Four Functions, all thin wrappers of the C ABI (every step of the cycle and
of its reverse runs in the library's kernels):

  Force       off(0), theta -> per-atom force (pic_deposit + pic_force);
              backward by pic_force_vjp + pic_deposit_vjp.
  Kick        v, F -> v + frac F/m dt on the evolved components (pic_kick);
              the map is the identity in v and a scalar multiple of F, so
              its VJP onto F is pic_kick itself applied to zero velocities
              with the velocity cotangent in place of the force.
  Trajectory  off(0), v(-1/2), theta -> off(T), v(T - 1/2) over nsteps
              cycles (pic_forward_record, checkpoints every `every` steps);
              backward by pic_backward_record, which recomputes each segment
              between checkpoints and sweeps it in reverse.  Grids too small
              for tiles take the same checkpointed scheme through the
              per-step calls (pic_deposit / pic_force / pic_push forward,
              pic_adjoint_step backward).
  StartedTrajectory  off(0), v(0), theta -> off(T), v(T - 1/2): the leapfrog
              start v(-1/2) = v(0) - F(0)/m dt/2 (pic_deposit, pic_force,
              pic_kick) and a recorded run; backward by pic_backward_record
              with the start kick's VJP folded into its last reverse step
              (the force VJP of the initial state is then not a pass of its
              own).  Tiled contexts; others compose Force, Kick, Trajectory.

theta is a float64 tensor (D, r0, s_rep, c_att, alpha) holding the
context's potential (alpha: the Morse width; its gradient is zero under
Lennard-Jones); it is there to receive dJ/dtheta.  Cell indices are integer
outputs without gradient.

crater_objective() composes them into the paper's experiment (Sec. 3): a
slab heated by an absorbed fluence F (kick std proportional to sqrt(F)),
the leapfrog start v(-1/2) = v(0) - F(0)/m dt/2, nsteps cycles, and the
smooth crater functional J = sum_p w_p sigmoid((y_p(T) - y_s) / tau) (the
weight no longer below the initial surface, on the normal axis).
"""
from __future__ import annotations

import torch

from . import binding as B

THETA_KEYS = ("D", "r0", "s_rep", "c_att", "alpha")


def theta_of(pot, device="cuda"):
    return torch.tensor([float(getattr(pot, k)) for k in THETA_KEYS], dtype=torch.float64, device=device)


def _check_theta(ctx: B.Context, theta):
    want = theta_of(ctx.pot, "cpu")
    if not torch.equal(theta.detach().cpu(), want):
        raise ValueError("theta must hold the context's potential (D, r0, s_rep, c_att, alpha)")


class Force(torch.autograd.Function):
    @staticmethod
    def forward(fctx, off, theta, ctx: B.Context, cell, wq):
        _check_theta(ctx, theta)
        n = cell.shape[0]
        vel = torch.zeros((3, n), dtype=torch.float32, device=off.device)
        dp = B.DeviceParticles(cell, off.detach().contiguous(), vel, wq)
        node = ctx.pic_deposit(dp)
        F = ctx.pic_force(dp, node)
        fctx.pic = (ctx, dp, node)
        fctx.theta_dev = theta.device
        return F

    @staticmethod
    def backward(fctx, gF):
        ctx, dp, node = fctx.pic
        lam_x = torch.zeros_like(dp.off)
        nbar, dth = ctx.pic_force_vjp(dp, node, gF.contiguous().float(), lam_x)
        ctx.pic_deposit_vjp(dp, nbar, lam_x)
        return lam_x, dth.to(fctx.theta_dev), None, None, None


class Kick(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vel, force, ctx: B.Context, cell, wq, frac: float):
        n = cell.shape[0]
        dp = B.DeviceParticles(cell, torch.zeros((ctx.grid.ndim, n), dtype=torch.float32, device=vel.device),
                               vel.detach().contiguous().clone(), wq)
        ctx.pic_kick(dp, force.detach().contiguous(), frac)
        fctx.pic = (ctx, cell, wq, float(frac))
        return dp.vel

    @staticmethod
    def backward(fctx, g_vel):
        ctx, cell, wq, frac = fctx.pic
        nd, n = ctx.grid.ndim, cell.shape[0]
        g_vel = g_vel.contiguous().float()
        dp = B.DeviceParticles(cell, torch.zeros((nd, n), dtype=torch.float32, device=g_vel.device),
                               torch.zeros((3, n), dtype=torch.float32, device=g_vel.device), wq)
        ctx.pic_kick(dp, g_vel[:nd].contiguous(), frac)
        return g_vel, dp.vel[:nd].contiguous(), None, None, None, None


def _step_untiled(ctx: B.Context, dp):
    node = ctx.pic_deposit(dp)
    F = ctx.pic_force(dp, node)
    ctx.pic_push(dp, F)


class Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, off0, vel0, theta, ctx: B.Context, cell0, wq, nsteps: int, every: int):
        _check_theta(ctx, theta)
        dp = B.DeviceParticles(cell0.clone(), off0.detach().contiguous().clone(),
                               vel0.detach().contiguous().clone(), wq)
        if B.lib.pic_record_bytes(ctx.ctx, int(nsteps), int(every)):
            rec = ctx.pic_forward_record(dp, nsteps, every)
        else:  # untiled context: checkpoints in the caller's order
            rec = []
            for s in range(nsteps):
                if s % every == 0:
                    rec.append(dp.clone())
                _step_untiled(ctx, dp)
        # the outputs go through save_for_backward: kept on fctx they would
        # form a reference cycle that holds the record until the next
        # garbage collection
        fctx.save_for_backward(dp.off, dp.vel, dp.cell)
        fctx.pic = (ctx, wq, rec, int(nsteps), int(every))
        fctx.theta_dev = theta.device
        fctx.mark_non_differentiable(dp.cell)
        return dp.off, dp.vel, dp.cell

    @staticmethod
    def backward(fctx, g_off, g_vel, _g_cell):
        ctx, wq, rec, nsteps, every = fctx.pic
        fctx.pic = None  # the record is released as soon as the sweep has run
        off, vel, cell = fctx.saved_tensors
        dp = B.DeviceParticles(cell, off, vel, wq)
        lam_x = torch.zeros_like(dp.off) if g_off is None else g_off.contiguous().float().clone()
        lam_v = torch.zeros_like(dp.vel) if g_vel is None else g_vel.contiguous().float().clone()
        if isinstance(rec, dict):
            dth = ctx.pic_backward_record(dp, rec, lam_x, lam_v)
        else:
            dth = torch.zeros(B.NTHETA, dtype=torch.float64, device=dp.off.device)
            nbar_next = None
            for j in range(len(rec) - 1, -1, -1):
                s0 = j * every
                states = [rec[j].clone()]
                for _ in range(min(every, nsteps - s0) - 1):
                    nxt = states[-1].clone()
                    _step_untiled(ctx, nxt)
                    states.append(nxt)
                for st in reversed(states):
                    node = ctx.pic_deposit(st)
                    nbar_next, _ = ctx.pic_adjoint_step(st, node, nbar_next, lam_x, lam_v, dtheta=dth)
            ctx.pic_deposit_vjp(rec[0], nbar_next, lam_x)
        return lam_x, lam_v, dth.to(fctx.theta_dev), None, None, None, None, None


class StartedTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, off0, v0, theta, ctx: B.Context, cell0, wq, nsteps: int, every: int):
        _check_theta(ctx, theta)
        dp = B.DeviceParticles(cell0.clone(), off0.detach().contiguous().clone(), v0.detach().contiguous().clone(),
                               wq)
        ctx.start_leapfrog(dp)  # v(0) -> v(-1/2): pic_deposit, pic_force, pic_kick(-1/2)
        rec = ctx.pic_forward_record(dp, nsteps, every)
        fctx.save_for_backward(dp.off, dp.vel, dp.cell)  # no reference cycle (see Trajectory)
        fctx.pic = (ctx, wq, rec)
        fctx.theta_dev = theta.device
        fctx.mark_non_differentiable(dp.cell)
        return dp.off, dp.vel, dp.cell

    @staticmethod
    def backward(fctx, g_off, g_vel, _g_cell):
        ctx, wq, rec = fctx.pic
        fctx.pic = None
        off, vel, cell = fctx.saved_tensors
        dp = B.DeviceParticles(cell, off, vel, wq)
        lam_x = torch.zeros_like(dp.off) if g_off is None else g_off.contiguous().float().clone()
        lam_v = torch.zeros_like(dp.vel) if g_vel is None else g_vel.contiguous().float().clone()
        dth = ctx.pic_backward_record(dp, rec, lam_x, lam_v, start_kick=-0.5)
        return lam_x, lam_v, dth.to(fctx.theta_dev), None, None, None, None, None


def crater_objective(ctx: B.Context, cell, off0, v_thermal, xi, sigma_ref, fluence_ref, fluence, wq, theta,
                     nsteps: int, every: int, y_s: float, tau: float):
    """J(theta, F) on device tensors (cell int32 [n], off0 float32 [ndim][n],
    v_thermal / xi float32 [3][n], sigma_ref float32 [n], wq int32 [n]);
    fluence is a float64 scalar tensor.  Returns (J, final offsets, cells)."""
    grid = ctx.grid
    nd = grid.ndim
    scale = torch.sqrt(fluence / fluence_ref).float()
    v0 = v_thermal + (sigma_ref * scale)[None, :] * xi
    if B.lib.pic_record_bytes(ctx.ctx, int(nsteps), int(every)):
        offT, velT, cellT = StartedTrajectory.apply(off0, v0, theta, ctx, cell, wq, nsteps, every)
    else:  # untiled context: the start kick and the run as separate Functions
        F0 = Force.apply(off0, theta, ctx, cell, wq)
        vh = Kick.apply(v0, F0, ctx, cell, wq, -0.5)
        offT, velT, cellT = Trajectory.apply(off0, vh, theta, ctx, cell, wq, nsteps, every)
    ax = nd - 1
    lateral = 1
    for d in range(ax):
        lateral *= grid.n[d]
    layer = torch.div(cellT.long(), lateral, rounding_mode="floor").double()
    y = (layer + offT[ax].double()) * grid.h[ax]
    w = wq.double() * 2.0 ** -20
    J = (w * torch.sigmoid((y - y_s) / tau)).sum()
    return J, offT, cellT
