"""Gradients of functionals of a rollout through the hand-written adjoint.

``Rollout.apply(V0, ctx, history, checkpoint_every)`` maps FP64 primitive
initial fields V0 (on the device) to the final conserved state U_T of a
rollout that replays ``history`` (the (dt, c_h, damp) list of a forward run,
frozen: the adjoint does not differentiate the CFL choice).  Its backward:

* receives dJ/dU_T from autograd and carries it in FP64;
* walks the checkpoint segments backwards: re-runs each segment from its
  stored state (keeping U^n and the stage-1 state U1 of every step) and
  applies ``mhd_step_adjoint`` step by step in reverse;
* maps dJ/dU_0 to dJ/dV0 with ``mhd_prim_to_cons_adjoint``.

Memory: one state per checkpoint plus 2 states per step of one segment.
All arithmetic runs in the library's kernels; this module only orders the
calls and holds the buffers.
"""
import torch

from .mhd import Context
from .rollout import advance


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V0, mctx, history, checkpoint_every=20):
        if not mctx.adjoint:
            raise ValueError("the context needs adjoint=True")
        U = mctx.prim_to_cons(V0.detach().contiguous())
        ckpts = []
        a, b = U, torch.empty_like(U)
        for s, (dt, ch, dmp) in enumerate(history):
            if s % checkpoint_every == 0:
                ckpts.append(a.clone())
            mctx.step(a, b, dt, ch, dmp)
            a, b = b, a
        fctx.mctx = mctx
        fctx.history = list(history)
        fctx.every = int(checkpoint_every)
        fctx.ckpts = ckpts
        fctx.save_for_backward(V0)
        return a

    @staticmethod
    def backward(fctx, gT):
        (V0,) = fctx.saved_tensors
        mctx, hist, every = fctx.mctx, fctx.history, fctx.every
        lam = gT.detach().to(torch.float64).contiguous()
        lam_n = torch.empty_like(lam)
        nsteps = len(hist)
        for seg in reversed(range(len(fctx.ckpts))):
            s0, s1 = seg * every, min(seg * every + every, nsteps)
            states = []
            a = fctx.ckpts[seg]
            for s in range(s0, s1):
                dt, ch, dmp = hist[s]
                b = torch.empty_like(a)
                u1 = torch.empty_like(a)
                mctx.step(a, b, dt, ch, dmp, U1_out=u1)
                states.append((a, u1))
                a = b
            for s in reversed(range(s0, s1)):
                dt, ch, dmp = hist[s]
                Un, U1 = states[s - s0]
                mctx.step_adjoint(Un, U1, lam, lam_n, dt, ch, dmp)
                lam, lam_n = lam_n, lam
            del states
        gV = mctx.prim_to_cons_adjoint(V0.detach().contiguous(), lam)
        return gV, None, None, None


def forward_history(mctx: Context, V0, nsteps=None, t_end=None):
    """Run the forward once to fix the (dt, c_h, damp) list."""
    U0 = mctx.prim_to_cons(V0.contiguous())
    _, _, hist = advance(mctx, U0, nsteps=nsteps, t_end=t_end)
    return hist


def kinetic_energy(U, cell_volume):
    """J = sum over cells of |m|^2 / (2 rho) times the cell volume (FP64)."""
    Ud = U.double()
    return 0.5 * ((Ud[1] ** 2 + Ud[2] ** 2 + Ud[3] ** 2) / Ud[0]).sum() * cell_volume
