"""C ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects invalid arguments before touching a
device."""
import ctypes
import os
import re

import pytest

from paper_2510_24175_amd import mhd, workloads as W
from tests.helpers import ROOT, have_gpu


def header_functions():
    text = open(os.path.join(ROOT, "include", "mhd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mhd.load_library()
    names = header_functions()
    assert len(names) >= 11, names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mhd.h but not exported"


def test_status_strings():
    lib = mhd.load_library()
    for st in range(-5, 1):
        assert lib.mhd_status_string(st)
    assert lib.mhd_status_string(0) == b"ok"


def _init(cfg):
    lib = mhd.load_library()
    h = ctypes.c_void_p()
    st = lib.mhd_init(ctypes.byref(cfg), None, ctypes.byref(h))
    if h:
        lib.mhd_destroy(h)
    return st


def _base():
    s, _ = W.turbulence(8)
    return mhd.make_config(s, "f32")


@pytest.mark.parametrize("field,value", [
    ("ndim", 0), ("ndim", 4), ("dtype", 7), ("riemann", 3), ("limiter", 9), ("glm", 2),
    ("flags", 2), ("gamma", 1.0), ("cfl", 0.0), ("cfl", 1.5), ("glm_alpha", -0.1),
    ("limiter", 3), ("time_order", 1), ("time_order", 4), ("ct", 3), ("ct", -1),
])
def test_invalid_config_is_rejected_before_device_use(field, value):
    cfg = _base()
    setattr(cfg, field, value)
    assert _init(cfg) == mhd.MHD_ERR_ARG


def test_config_layout_matches_the_header():
    # two int32 fields appended after the three doubles keep 8-byte alignment
    # (sizes of the C struct on x86-64 / LP64)
    assert ctypes.sizeof(mhd.mhd_config) == 152
    assert mhd.mhd_config.time_order.offset == 144
    assert mhd.mhd_config.ct.offset == 148


def test_constrained_transport_config_checks():
    s, _ = W.orszag_tang_3d_ct(8)
    cfg = mhd.make_config(s, "f32")
    assert cfg.ct == 1 and cfg.glm == 0
    cfg.glm = 1
    assert _init(cfg) == mhd.MHD_ERR_ARG  # CT replaces GLM
    cfg = mhd.make_config(s, "f32", adjoint=True)
    assert _init(cfg) == mhd.MHD_ERR_UNSUPPORTED
    cfg = mhd.make_config(s, "f32")
    cfg.bc[2][0] = cfg.bc[2][1] = mhd.MHD_OUTFLOW
    assert _init(cfg) == mhd.MHD_ERR_UNSUPPORTED
    s2, _ = W.orszag_tang(8)
    cfg = mhd.make_config(s2, "f32")
    cfg.ct, cfg.glm = 1, 0
    assert _init(cfg) == mhd.MHD_ERR_UNSUPPORTED  # 2D


@pytest.mark.parametrize("limiter,time_order", [("wenoz", 2), ("wenoz", 3), ("minmod", 3)])
def test_adjoint_of_weno_or_rk3_is_unsupported(limiter, time_order):
    s, _ = W.turbulence(8)
    s["limiter"], s["time_order"] = limiter, time_order
    assert _init(mhd.make_config(s, "f32", adjoint=True)) == mhd.MHD_ERR_UNSUPPORTED
    assert mhd.make_config(s, "f32").time_order == time_order


def test_invalid_geometry_is_rejected():
    cfg = _base()
    cfg.n[2] = 1  # active axis with one cell
    assert _init(cfg) == mhd.MHD_ERR_ARG
    cfg = _base()
    cfg.hi[1] = cfg.lo[1]
    assert _init(cfg) == mhd.MHD_ERR_ARG
    cfg = _base()
    cfg.bc[0][0] = mhd.MHD_PERIODIC
    cfg.bc[0][1] = mhd.MHD_OUTFLOW
    assert _init(cfg) == mhd.MHD_ERR_ARG
    s, _ = W.orszag_tang(8)
    cfg = mhd.make_config(s, "f64")
    cfg.n[2] = 3  # inactive axis must have one cell
    assert _init(cfg) == mhd.MHD_ERR_ARG


@pytest.mark.parametrize("n", [(0, 8, 8), (-5, 8, 8), (8, 0, 8), ((1 << 30) + 1, 8, 8),
                               (1 << 14, 1 << 14, 1 << 13)])
def test_empty_negative_and_oversized_grids_are_rejected(n):
    # empty or negative axes, an axis beyond 2^30 cells, more than 2^40 cells
    cfg = _base()
    for d in range(3):
        cfg.n[d] = n[d]
    assert _init(cfg) == mhd.MHD_ERR_ARG


def test_constrained_transport_grid_limit():
    # constrained-transport passes index cells in 32 bits: 2^31 cells or more
    # are refused (1300^3 = 2.197e9)
    s, _ = W.orszag_tang_3d_ct(8)
    cfg = mhd.make_config(s, "f32")
    for d in range(3):
        cfg.n[d] = 1300
    assert _init(cfg) == mhd.MHD_ERR_ARG


def test_null_arguments():
    lib = mhd.load_library()
    assert lib.mhd_init(None, None, None) == mhd.MHD_ERR_ARG
    assert lib.mhd_step(None, None, None, None, 1.0, 1.0, 1.0) == mhd.MHD_ERR_ARG
    assert lib.mhd_cfl_dt(None, None, None) == mhd.MHD_ERR_ARG
    assert lib.mhd_get_sums(None, None) == mhd.MHD_ERR_ARG
    assert lib.mhd_step_info(None, None) == mhd.MHD_ERR_ARG
    lib.mhd_destroy(None)


@pytest.mark.skipif(have_gpu(), reason="checks the no-device path")
def test_no_device_is_reported():
    assert _init(_base()) == mhd.MHD_ERR_NO_DEVICE
    s, _ = W.turbulence(8)
    with pytest.raises(mhd.MHDError) as e:
        mhd.Context(s, "f32")
    assert e.value.status == mhd.MHD_ERR_NO_DEVICE
