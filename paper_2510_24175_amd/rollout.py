"""Time loop over the C ABI: one CFL read-back per step.

Per step: dt and c_h come from the CFL reduction of the current state (the
standalone reduction for the first step, afterwards the maxima the previous
step already reduced on its output), dt is clipped so that t does not pass
t_end, the GLM decay factor exp(-alpha c_h dt / dh_min) is formed on the
host in FP64, and one Runge-Kutta step (SSP-RK2 or SSP-RK3, as the
context is configured) runs on the device.
"""
import torch

from .mhd import Context


def advance(ctx: Context, U0, nsteps=None, t_end=None, t0=0.0, history=None, keep_u1=None):
    """Advance the state U0 (not modified).  Returns (U, t, hist) with hist
    the list of (dt, c_h, damp) per step.  If ``history`` is given the
    recorded (dt, c_h, damp) are replayed instead of the CFL values.
    ``keep_u1`` (a list) receives (Un, U1) device copies of every step, for
    the adjoint."""
    a = U0.clone()
    b = torch.empty_like(a)
    t = t0
    hist = []
    s = 0
    have_info = False
    while True:
        if history is not None:
            if s >= len(history):
                break
            dt, ch, dmp = history[s]
        else:
            if nsteps is not None and s >= nsteps:
                break
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            if have_info:
                dt, ch, _ = ctx.step_info()
            else:
                dt, ch = ctx.cfl_dt(a)
            if t_end is not None and t + dt > t_end:
                dt = t_end - t
            dmp = ctx.damp(dt, ch)
        u1 = torch.empty_like(a) if keep_u1 is not None else None
        ctx.step(a, b, dt, ch, dmp, U1_out=u1)
        if keep_u1 is not None:
            keep_u1.append((a, u1))
            a = b
            b = torch.empty_like(a)
        else:
            a, b = b, a
        have_info = True
        t += dt
        hist.append((dt, ch, dmp))
        s += 1
    return a, t, hist
