"""Adjoint step and checkpointed rollout gradients on the GPU.

* one mhd_step_adjoint against the FP64 PyTorch reference gradient (itself
  pinned to central differences of the C oracle): FP64 <= 1e-10, FP32
  <= 2e-4 relative L2, on generic states (1D/2D/3D, HLL/HLLD, minmod/MC,
  periodic/outflow, with and without GLM);
* the rollout gradient of the final kinetic energy with respect to the
  initial density and velocity against central differences of the GPU
  FP64 forward with the frozen (dt, c_h) list, at the turbulence workload
  (128^3, 200 steps, checkpoints every 20, 8 smooth directions, eps 1e-3)
  and at 24^3;
* the same gradient against the reference gradient of the PyTorch step at
  32^3 (the workload's 200 steps, checkpoints every 20).
"""

import numpy as np
import pytest
import torch

from oracle import coracle as C
from oracle import torch_ref as R
from paper_2510_24175_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _generic_cases():
    s, V = W.turbulence((21, 13, 9))
    V[0] = 1.0 + 0.1 * V[2]
    V[4] = 1.0 + 0.1 * V[3]
    V[8] = 0.03 * V[1]
    yield "turb3d-hlld", s, V
    yield "turb3d-hll-mc", dict(s, riemann="hll", limiter="mc"), V
    yield "turb3d-outflow", dict(s, bc=(("outflow", "outflow"), ("periodic", "periodic"),
                                        ("outflow", "outflow"))), V
    yield "turb3d-noglm", dict(s, glm=False), V
    s1, V1 = W.cpa_wave((70,), amplitude=0.2)
    s1["bc"] = W.OUTFLOW_X
    noise = np.random.default_rng(11).normal(size=(9, 70))
    for q in range(9):
        V1[q, 0, 0] += 0.01 * np.convolve(noise[q], np.ones(5) / 5, mode="same")
    yield "1d-outflow-hlld", s1, V1
    yield "1d-outflow-hll", dict(s1, riemann="hll"), V1
    s2, V2 = W.orszag_tang((66, 10))
    V2 += 0.01 * np.random.default_rng(12).normal(size=V2.shape) * \
        np.array([1, 1, 1, 1, 1, 0.3, 0.3, 0.3, 1.0])[:, None, None, None]
    yield "2d-ot", s2, V2
    # (the turbulence start itself is not a case here: there p = 1 is only
    # uniform up to rounding, so limiter branches of p follow rounding noise
    # that differs between implementations; the rollout tests below cover it
    # through the gradients with respect to density and velocity, on which
    # the p branches have no effect)


CASES = list(_generic_cases())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,setup,V", CASES, ids=[c[0] for c in CASES])
def test_step_adjoint_matches_reference(name, setup, V, dtype):
    from paper_2510_24175_amd.mhd import Context
    _say(f"[gpu-adjoint] step {name} {dtype}")
    o = C.Oracle(setup)
    Uo = o.prim_to_cons(V)
    dt, ch = o.cfl(Uo)
    dmp = o.damp(dt, ch)
    ctx = Context(setup, dtype, adjoint=True)
    # both sides start from the oracle's conserved state, rounded to the
    # state type on the host for FP32
    Us = Uo if dtype == "f64" else Uo.astype(np.float32)
    Ug = torch.from_numpy(Us).cuda()
    lamp = np.random.default_rng(5).normal(size=Ug.shape)
    lamn = torch.empty(Ug.shape, dtype=torch.float64, device="cuda")
    ctx.step_adjoint(Ug, None, torch.from_numpy(lamp).cuda(), lamn, dt, ch, dmp)
    torch.cuda.synchronize()
    g_gpu = lamn.cpu().numpy()
    # reference gradient at that same state
    Ut = torch.from_numpy(Us.astype(np.float64)).requires_grad_(True)
    J = (torch.from_numpy(lamp) * R.step(Ut, setup, dt, ch, dmp)).sum()
    (g_ref,) = torch.autograd.grad(J, Ut)
    g_ref = g_ref.numpy()
    err = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    _say(f"    rel L2 {err:.2e}")
    assert err <= (1e-10 if dtype == "f64" else 2e-4), err
    # passing the stage-1 state from the forward gives the same result
    out = torch.empty_like(Ug)
    u1 = torch.empty_like(Ug)
    ctx.step(Ug, out, dt, ch, dmp, U1_out=u1)
    lamn2 = torch.empty_like(lamn)
    ctx.step_adjoint(Ug, u1, torch.from_numpy(lamp).cuda(), lamn2, dt, ch, dmp)
    torch.cuda.synchronize()
    assert torch.equal(lamn, lamn2)


def _smooth_dirs(n, seeds):
    return [W.smooth_direction(n, s) for s in seeds]


def _fd_check(n, nsteps, every, dtype, seeds, tol):
    from paper_2510_24175_amd.adjoint import Rollout, forward_history, kinetic_energy
    from paper_2510_24175_amd.mhd import Context
    from paper_2510_24175_amd.rollout import advance
    _say(f"[gpu-adjoint] rollout FD {n}^3 {nsteps} steps every {every} {dtype}")
    s, V = W.turbulence(n)
    Vd = torch.from_numpy(V).cuda()
    ctx64 = Context(s, "f64", adjoint=True)
    hist = forward_history(ctx64, Vd, nsteps=nsteps)
    ctx = ctx64 if dtype == "f64" else Context(s, "f32", adjoint=True)
    V0 = Vd.clone().requires_grad_(True)
    UT = Rollout.apply(V0, ctx, hist, every)
    J = kinetic_energy(UT, ctx.cell_volume)
    (g,) = torch.autograd.grad(J, V0)
    g = g.cpu().numpy()

    def J64(Vx):
        U, _, _ = advance(ctx64, ctx64.prim_to_cons(Vx), history=hist)
        return float(kinetic_energy(U, ctx64.cell_volume))

    eps = 1e-3
    dirs = _smooth_dirs(n, seeds)
    for k, d in enumerate(dirs):
        dV = np.zeros_like(V)
        dV[0] = 0.1 * d[0]          # density
        dV[1:4] = 0.1 * d           # velocity
        dVd = torch.from_numpy(dV).cuda()
        fd = (J64(Vd + eps * dVd) - J64(Vd - eps * dVd)) / (2 * eps)
        ad = float((g * dV).sum())
        rel = abs(fd - ad) / abs(fd)
        _say(f"    dir {k}: fd {fd:.10e} adjoint {ad:.10e} rel {rel:.2e}")
        assert rel <= tol, (fd, ad)


def test_adjoint_turbulence_workload_vs_finite_differences():
    """128^3 turbulence, FP32 forward and adjoint, 200 steps, checkpoints
    every 20; 8 seeded smooth directions (seeds 100-107), central
    differences of the FP64 forward with eps = 1e-3."""
    _fd_check(128, 200, 20, "f32", list(range(100, 108)), 1e-3)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rollout_gradient_vs_finite_differences_coarse(dtype):
    # At 24^3 the first step's limiter kink at the uniform initial density
    # (measured 2.8e-4 for one step, shrinking fast with resolution) bounds
    # the agreement; the exact FP64 comparison is against the reference
    # gradient below.
    _fd_check(24, 20, 5, dtype, [100, 101, 102], 5e-4 if dtype == "f64" else 1e-3)


def test_rollout_gradient_vs_reference_gradient():
    from paper_2510_24175_amd.adjoint import Rollout, kinetic_energy
    from paper_2510_24175_amd.mhd import Context
    n = 32
    nsteps = 200
    _say(f"[gpu-adjoint] rollout vs reference {n}^3 {nsteps} steps")
    s, V = W.turbulence(n)
    o = C.Oracle(s)
    hist = o.run(o.prim_to_cons(V), nsteps=nsteps)[2]
    Vt = torch.from_numpy(V.copy()).requires_grad_(True)
    UT = R.rollout(R.prim_to_cons(Vt, s["gamma"]), s, hist)
    Jr = R.kinetic_energy(UT, 1.0 / n ** 3)
    (g_ref,) = torch.autograd.grad(Jr, Vt)
    g_ref = g_ref.numpy()
    for dtype, tol in [("f64", 1e-10), ("f32", 1e-4)]:
        ctx = Context(s, dtype, adjoint=True)
        V0 = torch.from_numpy(V).cuda().requires_grad_(True)
        J = kinetic_energy(Rollout.apply(V0, ctx, hist, 20), ctx.cell_volume)
        (g,) = torch.autograd.grad(J, V0)
        g = g.cpu().numpy()
        sel = [0, 1, 2, 3]  # density and velocity
        err = np.linalg.norm(g[sel] - g_ref[sel]) / np.linalg.norm(g_ref[sel])
        _say(f"    {dtype}: rel L2 vs reference {err:.2e}")
        assert err <= tol, (dtype, err)
