"""Pins of the whole oracle step against invariants and exact solutions.

* uniform states are fixed points, bit for bit (zero flux differences and
  (a + a)/2 = a);
* periodic grids conserve rho, m, E, B exactly up to rounding (telescoping);
* translation on a periodic axis commutes with the step, bit for bit; the
  three axes are interchangeable (cyclic relabelling);
* mirror symmetry x -> 1-x and the 180-degree rotation symmetry of the
  Orszag-Tang vortex are kept;
* GLM damping of a uniform psi is the product of the per-step factors;
* Brio-Wu: the boundary fluxes are known in closed form while the waves are
  inside the box, so sum(m_x) = (p_T,L - p_T,R) t and sum(m_y) = -2 Bx By,L t;
* Sod (B = 0): converges to the exact Euler solution;
* circularly polarised Alfven wave: exact travelling solution, second-order
  convergence;
* HLLD keeps an isolated stationary contact exactly steady, HLL does not;
* CFL step of a uniform state has the closed form C dx / (|v| + c_f).
"""
import math
import os

import numpy as np
import pytest

from oracle import coracle as C
from paper_2510_24175_amd import workloads as W
from tests import exact_euler


def _run(setup, V, nsteps=None, t_end=None):
    o = C.Oracle(setup)
    U = o.prim_to_cons(V)
    U, t, h = o.run(U, nsteps=nsteps, t_end=t_end)
    return o, U, t, h


@pytest.mark.parametrize("riemann", ["hll", "hlld"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_uniform_state_is_bitwise_fixed_point(riemann, ndim):
    n = {1: (16,), 2: (8, 6), 3: (6, 5, 4)}[ndim]
    s, V = W.uniform(n, ndim=ndim, riemann=riemann)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    U, _, _ = o.run(U0, nsteps=100)
    np.testing.assert_array_equal(U, U0)


@pytest.mark.parametrize("riemann", ["hll", "hlld"])
def test_periodic_conservation(riemann):
    s, V = W.turbulence(12, riemann=riemann)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    U, _, _ = o.run(U0, nsteps=20)
    s0, s1 = o.sums(U0), o.sums(U)
    scale = np.array([np.abs(U0[q]).sum() for q in range(9)]) * o.cell_volume
    rel = np.abs(s1 - s0)[:8] / scale[:8]
    assert rel.max() <= 1e-13, rel


def test_translation_commutes_bitwise():
    s, V = W.turbulence(10)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    dt, ch = o.cfl(U0)
    U1 = o.step(U0, dt, ch)
    for axis, shift in [(3, 3), (2, -4), (1, 7)]:
        Us = np.roll(U0, shift, axis=axis)
        np.testing.assert_array_equal(o.step(Us, dt, ch), np.roll(U1, shift, axis=axis))


@pytest.mark.parametrize("riemann", ["hll", "hlld"])
def test_axes_are_interchangeable(riemann):
    """A 1D problem laid along x, y or z (uniform across) evolves identically
    under the cyclic relabelling x -> y -> z."""
    s1, V1 = W.brio_wu(48)
    s1["riemann"] = riemann
    s1["bc"] = W.PERIODIC3
    base = None
    for d in range(3):
        n = [1, 1, 1]
        n[d] = 48
        n = [max(v, 1) for v in n]
        n_full = [4, 4, 4]
        n_full[d] = 48
        s = W.make_setup("perm", 3, n_full, gamma=2.0, cfl=0.4, riemann=riemann)
        # relabel: component along x of the 1D problem goes to axis d
        V = np.empty((9, n_full[2], n_full[1], n_full[0]))
        prof = V1[:, 0, 0, :]  # (9, 48)
        shape = [1, 1, 1]
        shape[2 - d] = 48
        for q in range(9):
            if q in (1, 2, 3) or q in (5, 6, 7):
                base_q = 1 if q < 4 else 5
                src = base_q + ((q - base_q) - d) % 3
            else:
                src = q
            V[q] = prof[src].reshape(shape)
        o = C.Oracle(s)
        U = o.prim_to_cons(V)
        U, _, _ = o.run(U, nsteps=30)
        # bring back to the x frame and take one line
        line = np.empty((9, 48))
        for q in range(9):
            if q in (1, 2, 3) or q in (5, 6, 7):
                base_q = 1 if q < 4 else 5
                dst = base_q + ((q - base_q) + d) % 3
            else:
                dst = q
            arr = np.moveaxis(U[dst], 2 - d, 2)
            line[q] = arr[0, 0, :]
        if base is None:
            base = line
        else:
            np.testing.assert_array_equal(line, base)


def test_mirror_symmetry():
    s, V = W.turbulence(12)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    M = U0[:, :, :, ::-1].copy()
    M[1] *= -1  # m_x
    M[5] *= -1  # B_x
    hist = o.run(U0, nsteps=10)[2]
    A = o.replay(U0, hist)
    B = o.replay(M, hist)
    B = B[:, :, :, ::-1].copy()
    B[1] *= -1
    B[5] *= -1
    scale = np.abs(A).max(axis=(1, 2, 3), keepdims=True) + 1e-300
    assert (np.abs(A - B) / scale)[:8].max() <= 1e-13


def test_orszag_tang_rotation_symmetry():
    s, V = W.orszag_tang(48)
    o, U, _, _ = _run(s, V, nsteps=40)
    R = U[:, :, ::-1, ::-1].copy()
    for q in (1, 2, 5, 6):  # vector components flip under the 180-degree rotation
        R[q] *= -1
    scale = np.abs(U).max(axis=(1, 2, 3), keepdims=True) + 1e-300
    assert (np.abs(U - R) / scale)[:8].max() <= 1e-12


def test_psi_decay_closed_form():
    s, V = W.uniform((8, 8, 8), ndim=3, state=(1.0, 0.1, 0.2, -0.1, 1.0, 0.3, 0.2, 0.1, 0.05))
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    U, _, hist = o.run(U0, nsteps=25)
    factor = 1.0
    for dt, ch, _ in hist:
        factor *= math.exp(-0.1 * ch * dt / o.dh_min)
    np.testing.assert_allclose(U[8], 0.05 * factor, rtol=1e-15, atol=0)
    np.testing.assert_array_equal(U[:8], U0[:8])


def test_brio_wu_boundary_flux_invariants():
    s, V = W.brio_wu(400)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    for t_end in (0.05, 0.1):
        U, t, _ = o.run(U0, t_end=t_end)
        assert t == pytest.approx(t_end, rel=1e-15)
        s0, s1 = o.sums(U0), o.sums(U)
        ptL = 1.0 + 0.5 * (0.75 ** 2 + 1.0)
        ptR = 0.1 + 0.5 * (0.75 ** 2 + 1.0)
        assert s1[0] == pytest.approx(s0[0], rel=1e-13)
        assert s1[4] == pytest.approx(s0[4], rel=1e-13)
        assert abs(s1[6]) <= 1e-14
        assert s1[1] == pytest.approx((ptL - ptR) * t, rel=1e-12)
        assert s1[2] == pytest.approx(-2.0 * 0.75 * 1.0 * t, rel=1e-12)


def _golden(name):
    """key -> (value, tolerance) from a fixture under tests/golden/."""
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = (float(line[1]), float(line[2]))
    return out


def test_exact_riemann_solver_matches_tabulated_sod_star_state():
    # the exact solver the Sod test samples, against the textbook table
    g = _golden("sod_star_state.txt")
    L, R, gamma = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4
    ps, us, res = exact_euler.star_state(L, R, gamma)
    assert abs(res) < 1e-12
    assert abs(ps - g["p_star"][0]) <= g["p_star"][1]
    assert abs(us - g["u_star"][0]) <= g["u_star"][1]
    # star densities: left of the contact behind a rarefaction, right behind a shock
    rho_l = L[0] * (ps / L[2]) ** (1.0 / gamma)
    mu = (gamma - 1.0) / (gamma + 1.0)
    rho_r = R[0] * (ps / R[2] + mu) / (mu * ps / R[2] + 1.0)
    assert abs(rho_l - g["rho_star_left"][0]) <= g["rho_star_left"][1]
    assert abs(rho_r - g["rho_star_right"][0]) <= g["rho_star_right"][1]
    x = np.array([-0.05, 0.05])  # just left / right of the contact at x/t = u*
    rho, u, p = exact_euler.sample(L, R, gamma, us + x * 0.1)
    assert abs(rho[0] - rho_l) <= 1e-9 and abs(rho[1] - rho_r) <= 1e-9
    assert np.all(np.abs(p - ps) <= 1e-9) and np.all(np.abs(u - us) <= 1e-9)


@pytest.mark.parametrize("riemann", ["hll", "hlld"])
def test_sod_converges_to_exact_solution(riemann):
    ps, us, res = exact_euler.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert abs(res) < 1e-12
    errs = {}
    for n in (100, 200, 400, 800):
        s, V = W.sod(n, riemann=riemann)
        o, U, t, _ = _run(s, V, t_end=0.2)
        x = W.cell_centres(s)[0]
        rho_ex, _, _ = exact_euler.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (x - 0.5) / t)
        errs[n] = np.mean(np.abs(U[0, 0, 0] - rho_ex))
    assert errs[400] <= 1e-2
    order = math.log2(errs[100] / errs[800]) / 3.0
    assert order >= 0.6, errs


def _cpa_error(n, ndim, k):
    s, V = W.cpa_wave(n, ndim=ndim, k=k)
    o, U, t, _ = _run(s, V, t_end=s["period"])
    Vf = o.cons_to_prim(U)
    comps = [1, 2, 3, 5, 6, 7]
    return np.mean(np.abs(Vf[comps] - V[comps]))


def test_alfven_wave_second_order_1d():
    # minmod clips smooth extrema, so the asymptotic order is reached slowly
    e = [_cpa_error((n,), 1, (1, 0, 0)) for n in (64, 128, 256)]
    order = math.log2(e[1] / e[2])
    assert order >= 1.8, e


def test_alfven_wave_second_order_2d_oblique():
    e = [_cpa_error((n, n), 2, (1, 1, 0)) for n in (32, 64, 128)]
    order = math.log2(e[1] / e[2])
    assert order >= 1.8, e


def test_hlld_keeps_stationary_contact():
    s, V = W.stationary_contact(64, riemann="hlld")
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    U, _, _ = o.run(U0, nsteps=100)
    np.testing.assert_allclose(U, U0, rtol=0, atol=1e-14)
    s, V = W.stationary_contact(64, riemann="hll")
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    U, _, _ = o.run(U0, nsteps=100)
    assert np.abs(U[0] - U0[0]).max() > 1e-2


def test_cfl_closed_form_uniform():
    state = (1.3, 0.2, -0.3, 0.1, 0.9, 0.7, -0.4, 0.25, 0.0)
    s, V = W.uniform((8, 4, 2), ndim=3, state=state)
    s["hi"] = (1.0, 2.0, 0.5)
    o = C.Oracle(s)
    dt, ch = o.cfl(o.prim_to_cons(V))
    rho, p, g = state[0], state[4], 5.0 / 3.0
    a2 = g * p / rho
    B = np.array(state[5:8])
    lam = []
    for d in range(3):
        b2, bd2 = (B @ B) / rho, B[d] ** 2 / rho
        cf = math.sqrt(0.5 * (a2 + b2 + math.sqrt((a2 + b2) ** 2 - 4 * a2 * bd2)))
        lam.append(abs(state[1 + d]) + cf)
    dx = [1.0 / 8, 2.0 / 4, 0.5 / 2]
    assert ch == pytest.approx(max(lam), rel=1e-14)
    assert dt == pytest.approx(0.3 / max(l / h for l, h in zip(lam, dx)), rel=1e-14)


@pytest.mark.parametrize("riemann", ["hll", "hlld"])
def test_field_aligned_degenerate_uniform(riemann):
    # a^2 = b^2 = b_x^2 = 1 exactly (rho 1, p 1/2, gamma 2, B along x, dyadic
    # velocities): the x fast speed is 1 from a zero discriminant and every
    # HLLD x face takes the degenerate star branch (D = 0); the CFL maxima
    # are (|v_d| + c_f,d) with c_f = (1, sqrt 2, sqrt 2), and the state is a
    # fixed point of the step
    state = (1.0, 0.5, -0.25, 0.125, 0.5, 1.0, 0.0, 0.0, 0.0)
    s, V = W.uniform((8, 6, 4), ndim=3, state=state, riemann=riemann, gamma=2.0)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    dt, ch = o.cfl(U0)
    lam = [1.5, 0.25 + math.sqrt(2.0), 0.125 + math.sqrt(2.0)]
    assert ch == pytest.approx(max(lam), rel=1e-15)
    assert dt == pytest.approx(0.3 / max(l * n for l, n in zip(lam, (8, 6, 4))), rel=1e-15)
    U1 = o.step(U0, dt, ch)
    assert np.array_equal(U1, U0)


def test_nonphysical_state_is_an_error():
    s, V = W.uniform((6, 6, 6), ndim=3)
    o = C.Oracle(s)
    U = o.prim_to_cons(V)
    U[4, 2, 3, 1] = 0.1  # E below kinetic + magnetic energy: p < 0
    with pytest.raises(C.OracleError):
        o.cfl(U)
    with pytest.raises(C.OracleError):
        o.step(U, 1e-3, 1.0)


def test_subblock_reproduces_full_grid_cell():
    """One step at a cell depends on cells within 4 along each axis (two
    PLM stages), so an 11^3 periodic window around the cell, stepped with any
    boundary, gives the same value at its centre, bit for bit.  This is how
    the full-size parity test samples the oracle."""
    s, V = W.turbulence(16)
    o = C.Oracle(s)
    U0 = o.prim_to_cons(V)
    dt, ch = o.cfl(U0)
    full = o.step(U0, dt, ch)
    r = 5
    sb = W.make_setup("sub", 3, (2 * r + 1,) * 3, gamma=s["gamma"], cfl=s["cfl"],
                      riemann=s["riemann"], bc=(("outflow", "outflow"),) * 3,
                      hi=tuple((2 * r + 1) / 16 for _ in range(3)))
    ob = C.Oracle(sb)
    for (k, j, i) in [(0, 0, 0), (7, 3, 15), (15, 15, 8)]:
        idx = np.ix_(range(9), [(k + a) % 16 for a in range(-r, r + 1)],
                     [(j + a) % 16 for a in range(-r, r + 1)],
                     [(i + a) % 16 for a in range(-r, r + 1)])
        out = ob.step(U0[idx], dt, ch, o.damp(dt, ch))
        np.testing.assert_array_equal(out[:, r, r, r], full[:, k, j, i])


def _rhs_by_hand(o, setup, U, ch, cells):
    """L at a few cells assembled here from the separately pinned pieces:
    ghost values by the boundary rule, limited slopes, face states and the
    oracle's face flux, differenced along each active axis."""
    V = o.cons_to_prim(U)
    n = setup["n"]
    out = {}
    for cell in cells:  # (i, j, k)
        L = np.zeros(9)
        for d in range(setup["ndim"]):
            dx = (setup["hi"][d] - setup["lo"][d]) / n[d]

            def at(off):
                c = list(cell)
                m = c[d] + off
                if setup["bc"][d][0 if m < 0 else 1] == "periodic":
                    m %= n[d]
                else:
                    m = min(max(m, 0), n[d] - 1)
                c[d] = m
                return V[:, c[2], c[1], c[0]]

            W5 = [at(o_) for o_ in (-2, -1, 0, 1, 2)]
            slope = lambda a, b, c: np.array([C.limited_slope(setup["limiter"], b[q] - a[q],
                                                              c[q] - b[q]) for q in range(9)])
            sl = [None] + [slope(W5[m - 1], W5[m], W5[m + 1]) for m in (1, 2, 3)]
            Fm = C.face_flux(o, d, W5[1] + 0.5 * sl[1], W5[2] - 0.5 * sl[2], ch)
            Fp = C.face_flux(o, d, W5[2] + 0.5 * sl[2], W5[3] - 0.5 * sl[3], ch)
            L -= (Fp - Fm) / dx
        out[cell] = L
    return out


def test_rhs_assembly_at_outflow_boundaries():
    s, V = W.brio_wu(12)
    V[1, 0, 0] = np.linspace(-0.3, 0.4, 12)  # make every boundary slope matter
    V[8, 0, 0] = np.linspace(0.02, -0.01, 12)
    o = C.Oracle(s)
    U = o.prim_to_cons(V)
    L = o.rhs(U, 1.7)
    cells = [(i, 0, 0) for i in (0, 1, 2, 9, 10, 11)]
    for c, ref in _rhs_by_hand(o, s, U, 1.7, cells).items():
        np.testing.assert_allclose(L[:, 0, 0, c[0]], ref, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_rhs_assembly_3d(bc):
    s, V = W.turbulence((7, 6, 5))
    s["bc"] = ((bc, bc),) * 3
    s["limiter"] = "mc"
    V[8] = 0.05 * V[1]  # non-zero psi
    o = C.Oracle(s)
    U = o.prim_to_cons(V)
    L = o.rhs(U, 2.1)
    cells = [(0, 0, 0), (6, 5, 4), (3, 1, 2), (1, 4, 0)]
    for c, ref in _rhs_by_hand(o, s, U, 2.1, cells).items():
        np.testing.assert_allclose(L[:, c[2], c[1], c[0]], ref, rtol=1e-13, atol=1e-12)
