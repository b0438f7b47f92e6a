"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It drives ``liboracle.so`` (plain C,
FP64) and holds the oracle's own time loop:

* per step: ``dt, c_h = CFL(U^n)`` (maximum over cells and active axes of
  ``|v_d| + c_f,d``), ``dt`` clipped so that ``t`` does not pass ``t_end``,
  ``damp = exp(-alpha c_h dt / dh_min)`` (Dedner et al. 2002 mixed GLM,
  parabolic part applied as an exact decay once per step), then one SSP-RK2
  or SSP-RK3 step (Shu & Osher 1988).

Arrays are numpy float64, structure-of-arrays ``[9][nz][ny][nx]``; with
constrained transport (setup ``"ct": True``) ``[12][nz][ny][nx]``, the last
three the face-centred field on each cell's lower x, y and z face.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_RIEMANN = {"hll": 0, "hlld": 1}
_LIMITER = {"minmod": 0, "mc": 1, "wenoz": 2}
_BC = {"periodic": 0, "outflow": 1}


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("glm", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("glm_alpha", ctypes.c_double),
        ("time_order", ctypes.c_int32),
        ("ct", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # MHD_ORACLE_LIB names another build of the same source (for example
        # one compiled with sanitizers); otherwise the in-tree build
        path = os.environ.get("MHD_ORACLE_LIB") or _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(_Cfg)
        for name, args in {
            "orc_prim_to_cons": [cp, dp, dp],
            "orc_cons_to_prim": [cp, dp, dp],
            "orc_cfl": [cp, dp, dp],
            "orc_rhs": [cp, dp, ctypes.c_double, dp],
            "orc_step": [cp, dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double],
            "orc_sums": [cp, dp, dp],
            "orc_face_flux": [cp, ctypes.c_int, dp, dp, ctypes.c_double, dp],
            "orc_ct_emf": [cp, dp, dp],
        }.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.orc_fast_speed.argtypes = [dp, ctypes.c_double, ctypes.c_int]
        L.orc_fast_speed.restype = ctypes.c_double
        L.orc_limited_slope.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_limited_slope.restype = ctypes.c_double
        L.orc_wenoz.argtypes = [dp]
        L.orc_wenoz.restype = ctypes.c_double
        L.orc_glm_interface.argtypes = [ctypes.c_double] * 5 + [dp]
        L.orc_glm_interface.restype = None
        L.orc_hlld_fan.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_hlld_fan.restype = None
        L.orc_rotated_flux.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.orc_rotated_flux.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st == 1:
        raise OracleError(f"{what}: non-physical state (rho<=0, p<=0 or non-finite)")
    if st != 0:
        raise OracleError(f"{what}: bad argument (status {st})")


def _ct_mode(setup):
    """0 without constrained transport, 1 with the arithmetic-mean edge EMF,
    2 with the upwind edge EMF (setup "ct_emf": "mean" or "upwind")."""
    if not setup.get("ct", False):
        return 0
    return {"mean": 1, "upwind": 2}[setup.get("ct_emf", "mean")]


class Oracle:
    """FP64 CPU reference for one problem setup (a dict, see the workloads)."""

    def __init__(self, setup):
        self.setup = dict(setup)
        c = _Cfg()
        c.ndim = int(setup["ndim"])
        c.riemann = _RIEMANN[setup["riemann"]]
        c.limiter = _LIMITER[setup.get("limiter", "minmod")]
        c.glm = 1 if setup.get("glm", True) else 0
        for d in range(3):
            c.n[d] = int(setup["n"][d])
            c.lo[d] = float(setup["lo"][d])
            c.hi[d] = float(setup["hi"][d])
            for s in range(2):
                c.bc[d][s] = _BC[setup["bc"][d][s]]
        c.gamma = float(setup["gamma"])
        c.cfl = float(setup["cfl"])
        c.glm_alpha = float(setup.get("glm_alpha", 0.1))
        c.time_order = int(setup.get("time_order", 2))
        c.ct = _ct_mode(setup)
        self.cfg = c
        self.nstate = 12 if c.ct else 9
        self.shape = (self.nstate, int(setup["n"][2]), int(setup["n"][1]), int(setup["n"][0]))
        self.ndim = c.ndim
        self.dx = [(c.hi[d] - c.lo[d]) / c.n[d] for d in range(3)]
        self.dh_min = min(self.dx[d] for d in range(c.ndim))
        self.cell_volume = math.prod(self.dx[d] for d in range(c.ndim))

    # -- array maps -------------------------------------------------------
    def prim_to_cons(self, V):
        V = _f64(V).reshape(self.shape)
        U = np.empty_like(V)
        _check(lib().orc_prim_to_cons(ctypes.byref(self.cfg), _p(V), _p(U)), "prim_to_cons")
        return U

    def cons_to_prim(self, U):
        U = _f64(U).reshape(self.shape)
        V = np.empty_like(U)
        _check(lib().orc_cons_to_prim(ctypes.byref(self.cfg), _p(U), _p(V)), "cons_to_prim")
        return V

    def cfl(self, U):
        """(dt, c_h) of the state U, dt not clipped."""
        U = _f64(U).reshape(self.shape)
        out = np.zeros(2)
        _check(lib().orc_cfl(ctypes.byref(self.cfg), _p(U), _p(out)), "cfl")
        return float(out[0]), float(out[1])

    def rhs(self, U, ch):
        U = _f64(U).reshape(self.shape)
        L = np.empty_like(U)
        _check(lib().orc_rhs(ctypes.byref(self.cfg), _p(U), float(ch), _p(L)), "rhs")
        return L

    def damp(self, dt, ch):
        if not self.setup.get("glm", True) or self.cfg.ct:
            return 1.0
        return math.exp(-float(self.setup.get("glm_alpha", 0.1)) * ch * dt / self.dh_min)

    def step(self, U, dt, ch, damp=None, want_u1=False):
        U = _f64(U).reshape(self.shape)
        if damp is None:
            damp = self.damp(dt, ch)
        out = np.empty_like(U)
        u1 = np.empty_like(U) if want_u1 else None
        st = lib().orc_step(ctypes.byref(self.cfg), _p(U), _p(out),
                            _p(u1) if want_u1 else None, float(dt), float(ch), float(damp))
        _check(st, "step")
        return (out, u1) if want_u1 else out

    def sums(self, U):
        """Sums of the 9 cell-centred components times the cell volume."""
        U = _f64(U).reshape(self.shape)
        out = np.zeros(9)
        _check(lib().orc_sums(ctypes.byref(self.cfg), _p(U), _p(out)), "sums")
        return out

    def ct_emf(self, U):
        """Edge EMFs (3, nz, ny, nx) of a constrained-transport state: Ex,
        Ey, Ez on each cell's lower edges."""
        U = _f64(U).reshape(self.shape)
        E = np.zeros((3,) + self.shape[1:])
        _check(lib().orc_ct_emf(ctypes.byref(self.cfg), _p(U), _p(E)), "ct_emf")
        return E

    def div_b(self, U):
        """Divergence of the face field of each cell (constrained transport):
        sum over axes of (b_d(upper face) - b_d(lower face)) / dx_d."""
        U = _f64(U).reshape(self.shape)
        if not self.cfg.ct:
            raise OracleError("div_b needs a constrained-transport state")
        div = np.zeros(self.shape[1:])
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            b = U[9 + d]
            div += (np.roll(b, -1, axis=ax) - b) / self.dx[d]
        return div

    # -- time loop -------------------------------------------------------
    def run(self, U, nsteps=None, t_end=None, t0=0.0, record=None):
        """Advance U by nsteps steps or to t_end (whichever is given; both
        allowed, then the first reached).  Returns (U, t, history) where
        history lists (dt, c_h, damp) per step."""
        U = _f64(U).reshape(self.shape).copy()
        t = t0
        hist = []
        s = 0
        while True:
            if nsteps is not None and s >= nsteps:
                break
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            dt, ch = self.cfl(U)
            if t_end is not None and t + dt > t_end:
                dt = t_end - t
            dmp = self.damp(dt, ch)
            U = self.step(U, dt, ch, dmp)
            t += dt
            hist.append((dt, ch, dmp))
            s += 1
            if record is not None:
                record(s, U)
        return U, t, hist

    def replay(self, U, history):
        """Advance U with a recorded (dt, c_h, damp) list."""
        U = _f64(U).reshape(self.shape).copy()
        for dt, ch, dmp in history:
            U = self.step(U, dt, ch, dmp)
        return U


def set_threads(n):
    """OpenMP team size of the oracle's loops (n > 0)."""
    lib().orc_set_threads(int(n))


def threads():
    """OpenMP team size the oracle's loops use."""
    return int(lib().orc_threads())


# -- pointwise pieces used by the pin tests ---------------------------------

def fast_speed(V9, gamma, d):
    v = _f64(V9)
    return lib().orc_fast_speed(_p(v), float(gamma), int(d))


def limited_slope(limiter, a, b):
    return lib().orc_limited_slope(_LIMITER[limiter], float(a), float(b))


def wenoz(v5):
    """WENO-Z value at the right face of the middle of five cell values."""
    v = _f64(np.asarray(v5, dtype=np.float64).reshape(5))
    return lib().orc_wenoz(_p(v))


def glm_interface(bnL, bnR, psiL, psiR, ch):
    out = np.zeros(2)
    lib().orc_glm_interface(float(bnL), float(bnR), float(psiL), float(psiR), float(ch), _p(out))
    return float(out[0]), float(out[1])


def face_flux(setup_or_oracle, d, VL, VR, ch):
    o = setup_or_oracle if isinstance(setup_or_oracle, Oracle) else Oracle(setup_or_oracle)
    VL, VR = _f64(VL), _f64(VR)
    F = np.zeros(9)
    _check(lib().orc_face_flux(ctypes.byref(o.cfg), int(d), _p(VL), _p(VR), float(ch), _p(F)),
           "face_flux")
    return F


def hlld_fan(qL, qR, gamma):
    """Rotated-frame HLLD fan: dict of speeds and 8-component states."""
    qL, qR = _f64(qL), _f64(qR)
    out = np.zeros(69)
    lib().orc_hlld_fan(_p(qL), _p(qR), float(gamma), _p(out))
    names = ["UL", "UsL", "UssL", "UssR", "UsR", "UR", "FL", "FR"]
    res = {"s": out[:5].copy()}
    for i, nm in enumerate(names):
        res[nm] = out[5 + 8 * i: 13 + 8 * i].copy()
    return res


def rotated_flux(riemann, qL, qR, gamma):
    qL, qR = _f64(qL), _f64(qR)
    F = np.zeros(8)
    lib().orc_rotated_flux(_RIEMANN[riemann], _p(qL), _p(qR), float(gamma), _p(F))
    return F
