"""Seeded synthetic inputs: problem setups and primitive initial fields.

This module holds none of the scheme's arithmetic.  It only draws random
numbers and samples closed-form initial conditions at cell centres
``x_i = lo + (i + 1/2) dx``; each side of a comparison (the HIP library
and the CPU oracle) converts the returned primitive fields
``V = (rho, vx, vy, vz, p, Bx, By, Bz, psi)`` to conserved variables with
its own equation of state.

Arrays are float64, shape ``(9, nz, ny, nx)`` (x fastest).  A *setup* is a
plain dict naming the grid, the solver options and the run length.

Workloads (the paper benchmarks the 3D Orszag-Tang vortex and the
circularly polarised Alfven wave, section "Results for gPLUTO"; the setups
of those runs are not printed, so these are synthetic stand-ins):

* ``brio_wu``      1D Riemann problem, 400 cells, gamma=2, Bx=0.75.
* ``turbulence``   3D periodic decaying turbulence, seeded Gaussian mode
                   sums with k^-2 power in 1 <= |k| <= 4, divergence-free B.
* ``orszag_tang``  2D periodic vortex with seeded +-5% amplitudes.
* ``orszag_tang_3d`` 3D periodic vortex: the 2D fields with a z-modulated
                   velocity (the paper's first benchmark problem).
* ``cpa_wave``     circularly polarised Alfven wave (exact nonlinear
                   travelling solution), 1D/2D/3D, any direction;
                   ``cpa_wave_3d`` along the cube diagonal (the paper's
                   second benchmark problem).
* ``sod``, ``uniform``, ``stationary_contact``, ``switch_on_tube``:
                   closed-form test states.
"""
import math

import numpy as np

PERIODIC3 = (("periodic", "periodic"),) * 3
OUTFLOW_X = (("outflow", "outflow"), ("periodic", "periodic"), ("periodic", "periodic"))


def make_setup(name, ndim, n, *, gamma, cfl, riemann="hlld", limiter="minmod", bc=PERIODIC3,
               glm=True, glm_alpha=0.1, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), nsteps=None,
               t_end=None, time_order=2):
    """A problem setup.  limiter: "minmod" or "mc" (PLM) or "wenoz" (the
    fifth-order WENO-Z reconstruction); time_order 2 (SSP-RK2) or 3
    (SSP-RK3)."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    return {
        "name": name, "ndim": int(ndim), "n": n, "lo": tuple(lo), "hi": tuple(hi),
        "gamma": float(gamma), "cfl": float(cfl), "riemann": riemann, "limiter": limiter,
        "bc": tuple(tuple(b) for b in bc), "glm": bool(glm), "glm_alpha": float(glm_alpha),
        "nsteps": nsteps, "t_end": t_end, "time_order": int(time_order),
    }


def cell_centres(setup):
    """1D coordinate arrays (x, y, z) of the cell centres."""
    out = []
    for d in range(3):
        n = setup["n"][d]
        lo, hi = setup["lo"][d], setup["hi"][d]
        out.append(lo + (np.arange(n) + 0.5) * (hi - lo) / n)
    return out


def _empty(setup):
    nx, ny, nz = setup["n"]
    return np.zeros((9, nz, ny, nx))


# ---------------------------------------------------------------- 1D -------

def brio_wu(n=400):
    """Brio & Wu (1988)-type shock tube: gamma=2, Bx=0.75, left (rho,p,By) =
    (1,1,1), right (0.125,0.1,-1), v=0, Bz=0; outflow; to t=0.1 with
    minmod + HLL, RK2, CFL 0.4."""
    s = make_setup("brio_wu", 1, (n,), gamma=2.0, cfl=0.4, riemann="hll", bc=OUTFLOW_X,
                   t_end=0.1)
    x = cell_centres(s)[0]
    V = _empty(s)
    left = x < 0.5
    V[0, 0, 0] = np.where(left, 1.0, 0.125)
    V[4, 0, 0] = np.where(left, 1.0, 0.1)
    V[5] = 0.75
    V[6, 0, 0] = np.where(left, 1.0, -1.0)
    return s, V


def sod(n, riemann="hll", gamma=1.4, t_end=0.2):
    """Sod (1978) shock tube with B = 0: (rho,p) = (1,1) | (0.125,0.1)."""
    s = make_setup("sod", 1, (n,), gamma=gamma, cfl=0.4, riemann=riemann, bc=OUTFLOW_X,
                   t_end=t_end)
    x = cell_centres(s)[0]
    V = _empty(s)
    left = x < 0.5
    V[0, 0, 0] = np.where(left, 1.0, 0.125)
    V[4, 0, 0] = np.where(left, 1.0, 0.1)
    return s, V


def stationary_contact(n=64, riemann="hlld"):
    """Isolated contact: density jump, v=0, uniform p and B with Bn != 0."""
    s = make_setup("contact", 1, (n,), gamma=5.0 / 3.0, cfl=0.4, riemann=riemann,
                   bc=OUTFLOW_X, nsteps=100)
    x = cell_centres(s)[0]
    V = _empty(s)
    V[0, 0, 0] = np.where(x < 0.5, 1.0, 0.3)
    V[4] = 1.0
    V[5] = 1.0
    V[6] = 0.5
    V[7] = 0.3
    return s, V


def switch_on_tube(n=400, riemann="hlld", t_end=0.08):
    """1D tube with a strong normal field and no tangential field on the
    left: gamma = 5/3, B_x = 3, left (rho, p, B_y) = (3, 3, 0), right
    (1, 1, 1), v = 0, B_z = 0; outflow, CFL 0.4.  On the left the Alfven
    speed exceeds the sound speed and the tangential field is zero, so the
    fast and Alfven speeds coincide there: the degenerate case of the HLLD
    star states (keep v_t and B_t) at every interface of that region until
    the waves from the jump switch the tangential field on."""
    s = make_setup("switch_on", 1, (n,), gamma=5.0 / 3.0, cfl=0.4, riemann=riemann, bc=OUTFLOW_X,
                   t_end=t_end)
    x = cell_centres(s)[0]
    V = _empty(s)
    left = x < 0.5
    V[0, 0, 0] = np.where(left, 3.0, 1.0)
    V[4, 0, 0] = np.where(left, 3.0, 1.0)
    V[5] = 3.0
    V[6, 0, 0] = np.where(left, 0.0, 1.0)
    return s, V


# ------------------------------------------------------------ uniform ------

def uniform(n, ndim=3, state=(1.3, 0.2, -0.3, 0.1, 0.9, 0.7, -0.4, 0.25, 0.0), riemann="hlld",
            cfl=0.3, gamma=5.0 / 3.0):
    n = tuple(n) + (1,) * (3 - len(n))
    s = make_setup("uniform", ndim, n, gamma=gamma, cfl=cfl, riemann=riemann)
    V = _empty(s)
    for q in range(9):
        V[q] = state[q]
    return s, V


# ------------------------------------------------------- Alfven wave -------

def cpa_wave(n, ndim=1, k=(1, 0, 0), amplitude=1e-3, rho=1.0, p=1.0, b0=1.0, riemann="hlld",
             cfl=0.4, gamma=5.0 / 3.0):
    """Circularly polarised Alfven wave travelling along +k.

    B = b0 khat + A (sin phi e1 + cos phi e2),  v = -(B - b0 khat)/sqrt(rho),
    phi = 2 pi k.x; |B| and the total pressure are uniform, so this is an
    exact travelling solution at speed b0/sqrt(rho) for any amplitude.  One
    period is 1/|k| / (b0/sqrt(rho)) on the unit box."""
    n = tuple(n) + (1,) * (3 - len(n))
    s = make_setup("cpa", ndim, n, gamma=gamma, cfl=cfl, riemann=riemann)
    k = np.asarray(k, dtype=float)
    kn = np.linalg.norm(k)
    kh = k / kn
    # e1 perpendicular to k in the plane of k and z-hat (or y-hat for k || z)
    ref = np.array([0.0, 0.0, 1.0]) if abs(kh[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(ref, kh)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    x, y, z = cell_centres(s)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    phi = 2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z)
    V = _empty(s)
    V[0] = rho
    V[4] = p
    for a in range(3):
        db = amplitude * (np.sin(phi) * e1[a] + np.cos(phi) * e2[a])
        V[5 + a] = b0 * kh[a] + db
        V[1 + a] = -db / math.sqrt(rho)
    s["period"] = 1.0 / kn / (b0 / math.sqrt(rho))
    return s, V


def cpa_wave_3d(n, amplitude=0.1, riemann="hlld", cfl=0.3, limiter="wenoz", time_order=3):
    """3D circularly polarised Alfven wave on the periodic unit cube with
    k = (1, 1, 1) (wavelength 1/sqrt 3 along the diagonal), in the usual
    parameters of the test (Toth 2000; Gardiner & Stone 2008): rho = 1,
    p = 0.1, B_parallel = 1, perpendicular amplitude 0.1, gamma = 5/3.  The
    scheme defaults to the paper's benchmark one (WENO-Z, SSP-RK3)."""
    if isinstance(n, int):
        n = (n, n, n)
    s, V = cpa_wave(n, ndim=3, k=(1, 1, 1), amplitude=amplitude, rho=1.0, p=0.1, b0=1.0,
                    riemann=riemann, cfl=cfl)
    s["name"] = "cpa3d"
    s["limiter"], s["time_order"] = limiter, time_order
    return s, V


# -------------------------------------------- largest grids (on device) ----

def smooth_modes_device(n, device, riemann="hlld", cfl=0.3, limiter="minmod", time_order=2,
                        ct_emf=None, ripple=0.0):
    """Smooth periodic fields on an n^3 (or n = (nx, ny, nz)) grid on the unit
    box, built with torch on `device` (for grids whose FP64 primitives do not
    fit comfortably in host memory): a few low Fourier modes with a different
    wave vector in every component, so that a permuted or shifted axis shows
    in any cell, and a divergence-free field (each B component independent of
    its own coordinate).  With ct_emf ("mean" or "upwind") the setup is for
    constrained transport (GLM off) and the face fields, components 9..11,
    equal the cell field (each is constant along its own axis, so the
    discrete divergence is exactly zero).  ripple > 0 (GLM only) adds
    ripple * sin(2 pi (x + 2y + 3z) + q) to component q, so that no component
    is constant along any axis (limiter arguments then never tie at rounding
    noise).  Returns (setup, V) with V a float64 (9 or 12, nz, ny, nx) tensor.
    Deterministic; no random numbers."""
    import torch
    nx, ny, nz = (n, n, n) if isinstance(n, int) else tuple(n)
    s = make_setup("smooth_modes", 3, (nx, ny, nz), gamma=5.0 / 3.0, cfl=cfl, riemann=riemann,
                   limiter=limiter, time_order=time_order)
    if ct_emf is not None:
        s["ct"], s["glm"], s["ct_emf"] = True, False, ct_emf

    def centres(m):
        return (torch.arange(m, dtype=torch.float64, device=device) + 0.5) / m

    x, y, z = centres(nx).view(1, 1, nx), centres(ny).view(1, ny, 1), centres(nz).view(nz, 1, 1)
    tp = 2.0 * math.pi
    V = torch.empty((9 if ct_emf is None else 12, nz, ny, nx), dtype=torch.float64, device=device)
    V[0] = 1.0 + 0.25 * torch.sin(tp * (x + 2.0 * y + 3.0 * z) + 0.3)
    V[1] = 0.4 * torch.sin(tp * (y + z))
    V[2] = 0.4 * torch.sin(tp * (z + 2.0 * x) + 0.7)
    V[3] = 0.4 * torch.sin(tp * (x - y) + 1.1)
    V[4] = 1.0 + 0.2 * torch.cos(tp * (3.0 * x - y + z))
    V[5] = 0.3 * torch.cos(tp * (y - 2.0 * z))
    V[6] = 0.3 * torch.cos(tp * (z + x) + 0.5)
    V[7] = 0.3 * torch.cos(tp * (2.0 * x - y) + 0.9)
    V[8] = 0.0
    if ripple:
        if ct_emf is not None:
            raise ValueError("ripple breaks the divergence-free face field")
        for q in range(9):
            V[q] += ripple * torch.sin(tp * (x + 2.0 * y + 3.0 * z) + float(q))
    if ct_emf is not None:
        V[9:12] = V[5:8]
    return s, V


# -------------------------------------------------------- turbulence -------

def half_space_modes(kmax=4):
    """Integer wavevectors with 1 <= |k| <= kmax in the half space
    (kx>0) or (kx=0, ky>0) or (kx=ky=0, kz>0), in lexicographic order."""
    out = []
    r = range(-kmax, kmax + 1)
    for kx in r:
        for ky in r:
            for kz in r:
                k2 = kx * kx + ky * ky + kz * kz
                if not (1 <= k2 <= kmax * kmax):
                    continue
                if kx > 0 or (kx == 0 and ky > 0) or (kx == 0 and ky == 0 and kz > 0):
                    out.append((kx, ky, kz))
    return out


def _mode_coeffs(seed, power_exp, kmax=4):
    """Complex 3-vector coefficient c_k = a_k - i b_k per half-space mode,
    a_k, b_k ~ N(0, |k|^power_exp) componentwise, so that
    f(x) = sum_k a_k cos(2 pi k.x) + b_k sin(2 pi k.x) = Re sum c_k e^{2 pi i k.x}."""
    rng = np.random.default_rng(seed)
    modes = half_space_modes(kmax)
    coeffs = []
    for k in modes:
        std = math.sqrt(float(k[0] ** 2 + k[1] ** 2 + k[2] ** 2) ** power_exp)
        a = rng.normal(0.0, std, 3)
        b = rng.normal(0.0, std, 3)
        coeffs.append(a - 1j * b)
    return modes, coeffs


def _sample_mode_sum(setup, modes, coeffs, kmax=4):
    """Evaluate Re sum_k c_k e^{2 pi i k.x} (c_k complex 3-vectors) at the
    cell centres, separably: per axis a (2kmax+1) x n table of e^{2 pi i k x}
    and two real matrix products.  Returns (3, nz, ny, nx)."""
    xs = cell_centres(setup)
    nx, ny, nz = setup["n"]
    K = 2 * kmax + 1
    ex = [np.exp(2j * math.pi * (kk - kmax) * xs[0]) for kk in range(K)]
    ey = [np.exp(2j * math.pi * (kk - kmax) * xs[1]) for kk in range(K)]
    ez = [np.exp(2j * math.pi * (kk - kmax) * xs[2]) for kk in range(K)]
    Ex, Ey, Ez = np.array(ex), np.array(ey), np.array(ez)  # (K, n)
    out = np.empty((3, nz, ny, nx))
    for a in range(3):
        C = np.zeros((K, K, K), dtype=complex)  # [kz, ky, kx]
        for k, c in zip(modes, coeffs):
            C[k[2] + kmax, k[1] + kmax, k[0] + kmax] += c[a]
        # G[kz, y, x] = sum_{ky,kx} C[kz,ky,kx] Ey[ky,y] Ex[kx,x]
        G = np.einsum("zab,ay,bx->zyx", C, Ey, Ex, optimize=True).reshape(K, ny * nx)
        # f[z, yx] = Re sum_kz Ez[kz, z] G[kz, yx], as one real product
        A = np.concatenate([Ez.real.T, -Ez.imag.T], axis=1)           # (nz, 2K)
        B = np.concatenate([G.real, G.imag], axis=0)                  # (2K, ny*nx)
        np.matmul(A, B, out=out[a].reshape(nz, ny * nx))
    return out


def turbulence(n, seed_v=1, seed_a=2, vrms=0.5, brms=0.5, riemann="hlld", cfl=0.3, nsteps=100,
               kmax=4):
    """3D periodic decaying MHD turbulence on [0,1]^3.

    rho = 1, p = 1, gamma = 5/3, psi = 0.  v is a Gaussian mode sum over the
    half-space integer wavevectors 1 <= |k| <= kmax with per-mode variance
    |k|^-2; B = curl A, taken analytically from a mode sum A with variance
    |k|^-4 (so B has |k|^-2 power and is exactly solenoidal in the
    continuum).  Both are scaled to the requested rms over the cells."""
    if isinstance(n, int):
        n = (n, n, n)
    s = make_setup("turbulence", 3, n, gamma=5.0 / 3.0, cfl=cfl, riemann=riemann, nsteps=nsteps)
    modes, cv = _mode_coeffs(seed_v, -1.0, kmax)
    v = _sample_mode_sum(s, modes, cv, kmax)
    modes, ca = _mode_coeffs(seed_a, -2.0, kmax)
    cb = [2j * math.pi * np.cross(np.array(k, dtype=float), c) for k, c in zip(modes, ca)]
    b = _sample_mode_sum(s, modes, cb, kmax)
    v *= vrms / math.sqrt(np.mean(np.sum(v * v, axis=0)))
    b *= brms / math.sqrt(np.mean(np.sum(b * b, axis=0)))
    V = np.empty((9,) + v.shape[1:])
    V[0] = 1.0
    V[1:4] = v
    V[4] = 1.0
    V[5:8] = b
    V[8] = 0.0
    return s, V


def smooth_direction(n, seed, kmax=4):
    """Smooth random perturbation (3 fields) from the same mode-sum
    generator, each component scaled to unit rms; used as a direction for
    finite-difference checks."""
    if isinstance(n, int):
        n = (n, n, n)
    s = make_setup("direction", 3, n, gamma=5.0 / 3.0, cfl=0.3)
    modes, c = _mode_coeffs(seed, -1.0, kmax)
    f = _sample_mode_sum(s, modes, c, kmax)
    for a in range(3):
        f[a] /= math.sqrt(np.mean(f[a] * f[a]))
    return f


# ------------------------------------------------------- Orszag-Tang -------

def orszag_tang(n=1024, seed=3, riemann="hlld", cfl=0.4, t_end=0.5):
    """2D periodic Orszag & Tang (1979)-type vortex on [0,1]^2:
    rho = 25/(36 pi), p = 5/(12 pi), gamma = 5/3,
    v = (-a1 sin 2pi y, a2 sin 2pi x), B = B0 (-a3 sin 2pi y, a4 sin 4pi x),
    B0 = 1/sqrt(4 pi), a_i = 1 + 0.05 u_i with u_i ~ U(-1, 1) from the seed.
    Courant number 0.4 (the setup names none)."""
    if isinstance(n, int):
        n = (n, n)
    s = make_setup("orszag_tang", 2, n, gamma=5.0 / 3.0, cfl=cfl, riemann=riemann, t_end=t_end)
    rng = np.random.default_rng(seed)
    a = 1.0 + 0.05 * rng.uniform(-1.0, 1.0, 4)
    x, y, _ = cell_centres(s)
    Y, X = np.meshgrid(y, x, indexing="ij")
    b0 = 1.0 / math.sqrt(4 * math.pi)
    V = _empty(s)
    V[0] = 25.0 / (36.0 * math.pi)
    V[1, 0] = -a[0] * np.sin(2 * math.pi * Y)
    V[2, 0] = a[1] * np.sin(2 * math.pi * X)
    V[4] = 5.0 / (12.0 * math.pi)
    V[5, 0] = -b0 * a[2] * np.sin(2 * math.pi * Y)
    V[6, 0] = b0 * a[3] * np.sin(4 * math.pi * X)
    s["amplitudes"] = a.tolist()
    return s, V


def orszag_tang_3d(n, eps=0.2, riemann="hlld", cfl=0.3, limiter="wenoz", time_order=3, t_end=None):
    """3D periodic Orszag-Tang-type vortex on [0,1]^3: the 2D vortex
    (rho = 25/(36 pi), p = 5/(12 pi), gamma = 5/3, B = B0 (-sin 2pi y,
    sin 4pi x, 0), B0 = 1/sqrt(4 pi)) with the velocity modulated along z,
    v = ((1 + eps sin 2pi z)(-sin 2pi y), (1 + eps sin 2pi z) sin 2pi x,
    eps sin 2pi z), eps = 0.2, the way Helzel, Rossmanith & Taetz (2011)
    extend the vortex to three dimensions.  B is solenoidal and the fields
    are symmetric under a half turn about the z axis through the box
    centre.  The scheme defaults to the paper's benchmark one (WENO-Z,
    SSP-RK3)."""
    if isinstance(n, int):
        n = (n, n, n)
    s = make_setup("orszag_tang_3d", 3, n, gamma=5.0 / 3.0, cfl=cfl, riemann=riemann,
                   limiter=limiter, time_order=time_order, t_end=t_end)
    x, y, z = cell_centres(s)
    sx, sy = np.sin(2 * math.pi * x), np.sin(2 * math.pi * y)
    s4x = np.sin(4 * math.pi * x)
    mz = 1.0 + eps * np.sin(2 * math.pi * z)
    b0 = 1.0 / math.sqrt(4 * math.pi)
    V = _empty(s)
    V[0] = 25.0 / (36.0 * math.pi)
    V[1] = -mz[:, None, None] * sy[None, :, None]
    V[2] = mz[:, None, None] * sx[None, None, :]
    V[3] = (eps * np.sin(2 * math.pi * z))[:, None, None]
    V[4] = 5.0 / (12.0 * math.pi)
    V[5] = -b0 * sy[None, :, None]
    V[6] = b0 * s4x[None, None, :]
    s["eps"] = float(eps)
    return s, V


# ------------------------------------------- constrained transport -------
#
# With constrained transport the state carries the face-centred field on each
# cell's lower x, y and z face as three more components (12 in all), and the
# cell-centred B is the mean of the two faces of a cell along each axis.  The
# initial face fields below have zero discrete divergence: either each face
# component is independent of its own coordinate, or the field is the
# discrete curl of an edge-centred vector potential.

def _face_coords(setup):
    """Cell-centre and lower-face coordinate arrays per axis."""
    out = []
    for d in range(3):
        n = setup["n"][d]
        lo, hi = setup["lo"][d], setup["hi"][d]
        h = (hi - lo) / n
        out.append((lo + (np.arange(n) + 0.5) * h, lo + np.arange(n) * h, h))
    return out


def _with_faces(V, faces):
    W = np.zeros((12,) + V.shape[1:])
    W[:9] = V
    W[9:] = faces
    return W


def orszag_tang_3d_ct(n, eps=0.2, riemann="hlld", cfl=0.3, limiter="wenoz", time_order=3,
                      t_end=None, emf="mean"):
    """The 3D Orszag-Tang vortex of ``orszag_tang_3d`` for constrained
    transport (GLM off): face fields bx = -B0 sin 2pi y, by = B0 sin 4pi x,
    bz = 0 sampled on the faces (each independent of its own coordinate, so
    the discrete divergence is exactly zero).  emf: "mean" (arithmetic mean
    of the face fluxes) or "upwind" edge EMFs."""
    s, V = orszag_tang_3d(n, eps=eps, riemann=riemann, cfl=cfl, limiter=limiter,
                          time_order=time_order, t_end=t_end)
    s["name"], s["ct"], s["glm"], s["ct_emf"] = "orszag_tang_3d_ct", True, False, emf
    (xc, _, _), (yc, _, _), _ = _face_coords(s)
    b0 = 1.0 / math.sqrt(4 * math.pi)
    nx, ny, nz = s["n"]
    faces = np.zeros((3, nz, ny, nx))
    faces[0] = (-b0 * np.sin(2 * math.pi * yc))[None, :, None]
    faces[1] = (b0 * np.sin(4 * math.pi * xc))[None, None, :]
    return s, _with_faces(V, faces)


def cpa_wave_3d_ct(n, amplitude=0.1, riemann="hlld", cfl=0.3, limiter="wenoz", time_order=3,
                   emf="mean"):
    """The diagonal circularly polarised Alfven wave of ``cpa_wave_3d`` for
    constrained transport: the face field is b0 khat plus the discrete curl
    of the edge-centred potential A = a/(2 pi |k|) (sin phi e1 + cos phi e2),
    whose continuous curl is the wave's perturbation a (sin phi e1 +
    cos phi e2).  emf as for ``orszag_tang_3d_ct``."""
    s, V = cpa_wave_3d(n, amplitude=amplitude, riemann=riemann, cfl=cfl, limiter=limiter,
                       time_order=time_order)
    s["name"], s["ct"], s["glm"], s["ct_emf"] = "cpa3d_ct", True, False, emf
    k = np.array([1.0, 1.0, 1.0])
    kn = np.linalg.norm(k)
    kh = k / kn
    ref = np.array([0.0, 0.0, 1.0]) if abs(kh[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(ref, kh)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    (xc, xf, dx), (yc, yf, dy), (zc, zf, dz) = _face_coords(s)
    c = amplitude / (2 * math.pi * kn)

    def pot(comp, X, Y, Z):
        Z3, Y3, X3 = np.meshgrid(Z, Y, X, indexing="ij")
        phi = 2 * math.pi * (k[0] * X3 + k[1] * Y3 + k[2] * Z3)
        return c * (np.sin(phi) * e1[comp] + np.cos(phi) * e2[comp])

    Ax = pot(0, xc, yf, zf)  # x edges: (x_i, y_{j-1/2}, z_{k-1/2})
    Ay = pot(1, xf, yc, zf)  # y edges: (x_{i-1/2}, y_j, z_{k-1/2})
    Az = pot(2, xf, yf, zc)  # z edges: (x_{i-1/2}, y_{j-1/2}, z_k)
    up = lambda a, ax: np.roll(a, -1, axis=ax)  # value at the next edge along an axis
    faces = np.empty((3,) + Ax.shape)
    faces[0] = kh[0] + (up(Az, 1) - Az) / dy - (up(Ay, 0) - Ay) / dz
    faces[1] = kh[1] + (up(Ax, 0) - Ax) / dz - (up(Az, 2) - Az) / dx
    faces[2] = kh[2] + (up(Ay, 2) - Ay) / dx - (up(Ax, 1) - Ax) / dy
    return s, _with_faces(V, faces)
