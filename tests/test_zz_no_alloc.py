"""mhd_step_noalloc (the step for callers that cannot allocate: static
device scratch, no context) against mhd_step on the same inputs, through
the C ABI: identical outputs (bit for bit: the same kernels) and identical
reductions, on two calls in a row, the second on a smaller grid (the static
partials and flag keep the first call's contents, which must not leak into
the second).  Also: the limit and argument checks."""
import ctypes
import sys

import pytest

from paper_2510_24175_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _reference(setup, dtype, V):
    """mhd_step through a context: (Un, U1, U_next, info) on the device."""
    import torch
    from paper_2510_24175_amd.mhd import Context
    ctx = Context(setup, dtype)
    Un = ctx.prim_to_cons(torch.from_numpy(V).cuda())
    dt, ch = ctx.cfl_dt(Un)
    dmp = ctx.damp(dt, ch)
    U1 = torch.empty_like(Un)
    Ux = torch.empty_like(Un)
    ctx.step(Un, Ux, dt, ch, dmp, U1_out=U1)
    info = ctx.step_info()
    torch.cuda.synchronize()
    return ctx, Un, U1, Ux, (dt, ch, dmp), info


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_step_matches_context_step(dtype):
    import torch
    from paper_2510_24175_amd import mhd
    lib = mhd.load_library()
    cases = [("turbulence 70x40x36", *W.turbulence((70, 40, 36))),
             ("Orszag-Tang 3D 37x21x9 WENO-Z", *W.orszag_tang_3d((37, 21, 9), time_order=2))]
    for name, setup, V in cases:
        _say(f"[gpu-noalloc] {name} {dtype}")
        ctx, Un, U1, Ux, (dt, ch, dmp), info = _reference(setup, dtype, V)
        cfg = mhd.make_config(setup, dtype)
        U1n = torch.full_like(Un, float("nan"))
        Uxn = torch.full_like(Un, float("nan"))
        out = (ctypes.c_double * 11)()
        st = lib.mhd_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.c_void_p(Un.data_ptr()), ctypes.c_void_p(Uxn.data_ptr()),
                                  ctypes.c_void_p(U1n.data_ptr()), dt, ch, dmp, out)
        assert st == mhd.MHD_OK, st
        torch.cuda.synchronize()
        assert torch.equal(U1n, U1) and torch.equal(Uxn, Ux)
        assert list(out) == [info[0], info[1], *info[2]]
        _say(f"    identical state and reductions (dt_next {out[0]:.6e})")
        # async form (no info): same result
        Uxa = torch.full_like(Un, float("nan"))
        st = lib.mhd_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.c_void_p(Un.data_ptr()), ctypes.c_void_p(Uxa.data_ptr()),
                                  ctypes.c_void_p(U1n.data_ptr()), dt, ch, dmp, None)
        assert st == mhd.MHD_OK, st
        torch.cuda.synchronize()
        assert torch.equal(Uxa, Ux)
        ctx.close()


def test_noalloc_reports_nonphysical_and_then_recovers():
    import torch
    from paper_2510_24175_amd import mhd
    lib = mhd.load_library()
    s, V = W.turbulence((40, 24, 20))
    _say("[gpu-noalloc] non-physical flag")
    ctx, Un, U1, Ux, (dt, ch, dmp), info = _reference(s, "f32", V)
    cfg = mhd.make_config(s, "f32")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    bad = Un.clone()
    bad[4, 3, 5, 7] = 0.01  # E below kinetic + magnetic energy: p < 0
    out = (ctypes.c_double * 11)()
    a, b = torch.empty_like(Un), torch.empty_like(Un)
    st = lib.mhd_step_noalloc(ctypes.byref(cfg), stream, ctypes.c_void_p(bad.data_ptr()),
                              ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), dt, ch, dmp, out)
    assert st == mhd.MHD_ERR_NONPHYSICAL
    # the next call clears the flag: a good state steps cleanly
    st = lib.mhd_step_noalloc(ctypes.byref(cfg), stream, ctypes.c_void_p(Un.data_ptr()),
                              ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), dt, ch, dmp, out)
    assert st == mhd.MHD_OK
    torch.cuda.synchronize()
    assert torch.equal(a, Ux)
    ctx.close()


def test_noalloc_argument_checks():
    import torch
    from paper_2510_24175_amd import mhd
    lib = mhd.load_library()
    s, V = W.turbulence((16, 8, 8))
    cfg = mhd.make_config(s, "f32")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    U = torch.zeros((9, 8, 8, 16), device="cuda")
    A, B = torch.empty_like(U), torch.empty_like(U)
    p = lambda x: ctypes.c_void_p(x.data_ptr())  # noqa: E731
    call = lambda c, u, a, b, dt=1e-3, ch=1.0, dm=1.0: lib.mhd_step_noalloc(  # noqa: E731
        ctypes.byref(c), stream, u, a, b, dt, ch, dm, None)
    assert call(cfg, p(U), p(A), None) == mhd.MHD_ERR_ARG          # U1_out is required
    assert call(cfg, p(U), p(U), p(B)) == mhd.MHD_ERR_ARG          # aliasing
    assert call(cfg, p(U), p(A), p(B), dt=0.0) == mhd.MHD_ERR_ARG
    assert call(cfg, p(U), p(A), p(B), dm=1.5) == mhd.MHD_ERR_ARG
    c3 = mhd.make_config(dict(s, time_order=3), "f32")
    assert call(c3, p(U), p(A), p(B)) == mhd.MHD_ERR_UNSUPPORTED
    cad = mhd.make_config(s, "f32", adjoint=True)
    assert call(cad, p(U), p(A), p(B)) == mhd.MHD_ERR_ARG
    # beyond the static partials: 2048 x 2048 x 2048 cells (not allocated:
    # refused before any device work)
    big = mhd.make_config(W.turbulence((16, 8, 8))[0], "f32")
    for d in range(3):
        big.n[d] = 2048
    assert call(big, p(U), p(A), p(B)) == mhd.MHD_ERR_ARG
