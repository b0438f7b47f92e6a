"""GPU path at the workloads' full sizes, in the launch configuration the
benchmark uses.

* 512^3 turbulence, FP32: one step compared cell by cell at sampled cells
  (corners, tile and z-chunk boundaries, random) with the FP64 oracle run on
  an 11^3 periodic window around each cell (a step at a cell depends only on
  cells within 4 along each axis; the window reproduces the full-grid value,
  pinned in the oracle tests); dt and c_h from the oracle's full-grid CFL;
  the GPU's own CFL against it; FP64 conservation sums over two steps.
* 128^3 turbulence, FP64: full-grid comparison after 10 steps (100 steps
  with MHD_FULL_CHECKS=1).
* 1024^2 Orszag-Tang: 10 FP32 steps against the oracle on the full grid;
  a run to t = 0.4 (Courant number 0.15) in FP64 and FP32 checked for
  conservation and for the 180-degree rotation symmetry of the setup.
"""
import os

import numpy as np
import pytest
import torch

from oracle import coracle as C
from paper_2510_24175_amd import workloads as W
from tests.helpers import rel_l1

pytestmark = pytest.mark.gpu
FULL = os.environ.get("MHD_FULL_CHECKS") == "1"


def _say(msg):
    print(msg, flush=True)


def _sample_cells(n, rng, count=40):
    cells = [(0, 0, 0), (n - 1, n - 1, n - 1), (63, 64, 3), (64, 63, 4), (127, 4, 63),
             (128, 3, 64), (n - 1, 0, 64), (0, n - 1, 63), (255, 256, 255), (511, 300, 448)]
    while len(cells) < count:
        cells.append(tuple(int(v) for v in rng.integers(0, n, 3)))
    return [(k, j, i) for (i, j, k) in cells]


def test_turbulence_512_fp32_one_step_sampled():
    from paper_2510_24175_amd.mhd import Context
    n = 512
    _say("[gpu-fullsize] turbulence 512^3 FP32, generating fields")
    s, V = W.turbulence(n)
    o = C.Oracle(s)
    Uo = o.prim_to_cons(V)
    dt, ch = o.cfl(Uo)
    dmp = o.damp(dt, ch)
    _say(f"    oracle CFL dt={dt:.6e} c_h={ch:.6e}")
    ctx = Context(s, "f32")
    Ug = ctx.prim_to_cons(torch.from_numpy(V).cuda())
    del V
    dtg, chg = ctx.cfl_dt(Ug)
    assert abs(dtg / dt - 1) < 1e-6 and abs(chg / ch - 1) < 1e-6, (dtg, dt, chg, ch)
    out = torch.empty_like(Ug)
    ctx.step(Ug, out, dt, ch, dmp)
    _, _, sums1 = ctx.step_info()
    out2 = torch.empty_like(Ug)
    dt2, ch2, _ = ctx.step_info()
    ctx.step(out, out2, dt2, ch2, ctx.damp(dt2, ch2))
    _, _, sums2 = ctx.step_info()
    torch.cuda.synchronize()
    # periodic: rho, m, E, B conserved up to the FP32 rounding of the stored state
    scale = np.array([np.abs(Uo[q]).sum() for q in range(9)]) * o.cell_volume
    dsum = np.abs(np.array(sums2) - np.array(sums1))[:8] / scale[:8]
    _say(f"    conservation over one FP32 step (FP64 sums): {dsum.max():.2e}")
    assert dsum.max() <= 1e-6
    # sampled cells against the oracle on an 11^3 window
    r = 5
    sub = W.make_setup("window", 3, (2 * r + 1,) * 3, gamma=s["gamma"], cfl=s["cfl"],
                       riemann=s["riemann"], bc=(("outflow", "outflow"),) * 3,
                       hi=tuple((2 * r + 1) / n for _ in range(3)))
    ow = C.Oracle(sub)
    rng = np.random.default_rng(9)
    comp_scale = np.maximum(np.abs(Uo).max(axis=(1, 2, 3)), 1e-2)
    worst = 0.0
    for (k, j, i) in _sample_cells(n, rng):
        idx = np.ix_(range(9), [(k + a) % n for a in range(-r, r + 1)],
                     [(j + a) % n for a in range(-r, r + 1)], [(i + a) % n for a in range(-r, r + 1)])
        ref = ow.step(Uo[idx], dt, ch, dmp)[:, r, r, r]
        got = out[:, k, j, i].double().cpu().numpy()
        err = (np.abs(got - ref) / comp_scale).max()
        worst = max(worst, err)
        assert err <= 1e-5, ((k, j, i), got, ref)
    _say(f"    worst sampled-cell error (per-component scaled): {worst:.2e}")


def test_turbulence_128_fp64_full_grid():
    from paper_2510_24175_amd.mhd import Context
    from paper_2510_24175_amd.rollout import advance
    nsteps = 100 if FULL else 10
    _say(f"[gpu-fullsize] turbulence 128^3 FP64, {nsteps} steps, full grid")
    s, V = W.turbulence(128)
    ctx = Context(s, "f64")
    U, _, hg = advance(ctx, ctx.prim_to_cons(torch.from_numpy(V).cuda()), nsteps=nsteps)
    Ug = U.cpu().numpy()
    o = C.Oracle(s)
    Uo, _, ho = o.run(o.prim_to_cons(V), nsteps=nsteps)
    err = rel_l1(Ug, Uo, ch=ho[-1][1])
    _say(f"    rel L1 per component {np.array2string(err, precision=2)}")
    assert err.max() <= 1e-10


def _rot_asym(U):
    R = U[:, :, ::-1, ::-1].copy()
    R[[1, 2, 5, 6]] *= -1
    return max(np.abs(U[q] - R[q]).sum() / np.abs(U[q]).sum() for q in (0, 1, 2, 4, 5, 6))


def test_orszag_tang_1024():
    from paper_2510_24175_amd.mhd import Context
    from paper_2510_24175_amd.rollout import advance
    s, V = W.orszag_tang(1024)
    _say("[gpu-fullsize] Orszag-Tang 1024^2: 10 FP32 steps vs oracle")
    ctx = Context(s, "f32")
    U0 = ctx.prim_to_cons(torch.from_numpy(V).cuda())
    U, _, hg = advance(ctx, U0, nsteps=10)
    o = C.Oracle(s)
    Uo, _, ho = o.run(o.prim_to_cons(V), nsteps=10)
    err = rel_l1(U.double().cpu().numpy(), Uo, ch=ho[-1][1])
    _say(f"    rel L1 per component {np.array2string(err, precision=2)}")
    assert err.max() <= 1e-5
    o_sums0 = o.sums(o.prim_to_cons(V))
    scale = np.array([np.abs(Uo[q]).sum() for q in range(9)]) * o.cell_volume
    # Without floors this scheme (PLM minmod + HLLD + GLM, SSP-RK2) loses
    # pressure positivity on this setup at 1024^2 before t = 0.5 for Courant
    # numbers 0.2 - 0.3 in FP64 (the FP64 oracle at 0.3 fails at t = 0.398, as
    # the GPU path does).  At 0.15 the run is on the edge near t = 0.44: the
    # FP64 oracle reaches t = 0.5, while two GPU builds whose steps agree to
    # 3e-16 on the same input (the HLLD flux written with and without terms
    # that are exactly zero) follow trajectories that agree to 1e-15 through
    # step 6500 and then part, one reaching t = 0.5 and the other stopping at
    # t = 0.4386.  The long run therefore ends at t = 0.4 (Courant number 0.15).  The point symmetry
    # holds up to rounding differences that the shock interactions amplify:
    # the FP64 oracle's own asymmetry on this setup at 512^2 (4372 steps) is
    # 4.3e-6, and the GPU FP64 state there differs from the oracle's by 6e-6
    # (rel L1).  Conservation: FP64 to rounding (3e-16 measured); the FP32
    # state is rounded at every cell update, and over the 8795 steps to
    # t = 0.5 the FP64 sums of the FP32 states drifted by 2.3e-6 of sum |q|
    # (measured), so 1e-5.
    s_long = dict(s, cfl=0.15)
    t_long = 0.4
    for dtype, sym_tol, cons_tol in [("f64", 5e-5, 1e-12), ("f32", 5e-5, 1e-5)]:
        _say(f"[gpu-fullsize] Orszag-Tang 1024^2 {dtype} to t = {t_long} (Courant 0.15)")
        ctx = Context(s_long, dtype)
        U0 = ctx.prim_to_cons(torch.from_numpy(V).cuda())
        U, t, hist = advance(ctx, U0, t_end=t_long)
        _, _, sums = ctx.step_info()
        Ug = U.double().cpu().numpy()
        asym = _rot_asym(Ug)
        dcons = (np.abs(np.array(sums) - o_sums0)[[0, 1, 2, 4, 5, 6]] / scale[[0, 1, 2, 4, 5, 6]]).max()
        _say(f"    steps {len(hist)} t={t:.6f} asymmetry {asym:.2e} conservation {dcons:.2e}")
        assert abs(t - t_long) < 1e-12
        assert asym <= sym_tol
        assert dcons <= cons_tol
