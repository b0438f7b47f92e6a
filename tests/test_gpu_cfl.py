"""The CFL maxima fused into the last stage against mhd_cfl_dt, which forms
the FP64 speeds of every cell of the same state: with FP32 states the fused
reduction takes FP64 speeds only of the cells an FP32 estimate picks (one
per maximum and thread), which can differ from the all-FP64 maxima by twice
the estimate's error; on these workloads (ragged 3D turbulence and 256^3 in
the benchmark's launch shape, WENO-Z + SSP-RK3, 2D and 1D, a uniform state
whose every cell ties) every step's dt and c_h are those of the all-FP64
reduction bit for bit.  FP64 states take every cell's FP64 speeds in both."""
import pytest

from paper_2510_24175_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    ("turbulence 70x37x45", lambda: W.turbulence((70, 37, 45))),
    ("turbulence 256^3", lambda: W.turbulence(256)),
    ("3D Orszag-Tang 70x37x45 WENO-Z RK3", lambda: W.orszag_tang_3d((70, 37, 45))),
    ("Orszag-Tang 130x66", lambda: W.orszag_tang((130, 66))),
    ("Brio-Wu 400", lambda: W.brio_wu(400)),
    ("uniform 70x37x45", lambda: W.uniform((70, 37, 45), ndim=3)),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fused_cfl_equals_standalone(name, make, dtype):
    import torch
    from paper_2510_24175_amd.mhd import Context
    print(f"[gpu-cfl] {name} {dtype}", flush=True)
    s, V = make()
    ctx = Context(s, dtype)
    a = ctx.prim_to_cons(torch.from_numpy(V).cuda())
    b = torch.empty_like(a)
    dt, ch = ctx.cfl_dt(a)
    for _ in range(10):
        ctx.step(a, b, dt, ch, ctx.damp(dt, ch))
        a, b = b, a
        dti, chi, _ = ctx.step_info()
        dtc, chc = ctx.cfl_dt(a)
        assert (dti, chi) == (dtc, chc), (dti, dtc, chi, chc)
        dt, ch = dti, chi
    ctx.close()
