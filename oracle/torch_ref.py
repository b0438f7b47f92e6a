"""Vectorised FP64 PyTorch-CPU version of the oracle step, for reference
gradients (test infrastructure only).

Same scheme and formulas as ``mhd_oracle.c`` (PLM + GLM + HLL/HLLD +
SSP-RK2 + psi damping, dt and c_h given), written with whole-array torch
operations so that ``torch.autograd`` differentiates it.  Every branch of
the scheme is a ``torch.where`` whose gradient follows the selected branch;
at exact ties the choices are: minmod takes the left difference when
|a| = |b| != 0; where an argument is exactly zero (uniform fields,
symmetric samples) the derivative is the one a central difference sees
(see limited_slope); the MC limiter prefers 2*minmod over the central
difference; the minima and maxima of the outer wave speeds (Davis's for
HLL; min/max of the normal velocities and the larger fast speed for HLLD)
take the left state;
sign(B_n = 0) = +1.
Denominators of branches that are not taken are replaced by 1 so that they
cannot poison gradients.

Arrays: (9, nz, ny, nx) float64 tensors on the CPU.
"""

import numpy as np
import torch

EPS64 = 2.220446049250313e-16


def _cat_idx(n, periodic):
    """Source index of padded coordinates -2 .. n+1 along one axis."""
    m = np.arange(-2, n + 2)
    if periodic:
        return torch.from_numpy(np.mod(m, n))
    return torch.from_numpy(np.clip(m, 0, n - 1))


def cons_to_prim(U, gamma):
    rho = U[0]
    v = U[1:4] / rho
    kin = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho
    mag = 0.5 * (U[5] * U[5] + U[6] * U[6] + U[7] * U[7])
    p = (gamma - 1.0) * (U[4] - kin - mag)
    return torch.cat([rho[None], v, p[None], U[5:9]], 0)


def prim_to_cons(V, gamma):
    rho = V[0]
    E = V[4] / (gamma - 1.0) + 0.5 * rho * (V[1] * V[1] + V[2] * V[2] + V[3] * V[3]) \
        + 0.5 * (V[5] * V[5] + V[6] * V[6] + V[7] * V[7])
    return torch.cat([rho[None], rho * V[1:4], E[None], V[5:9]], 0)


def limited_slope(a, b, limiter):
    """minmod(a, b) or MC = minmod(2a, 2b, (a+b)/2); value 0 when a*b <= 0.

    Where an argument is exactly zero the limiter has a kink; the expressions
    chosen there keep the value 0 but give the derivative a central
    difference sees along smooth directions: (1/2, 1/2) at a = b = 0, and
    c toward a zero argument when the other is not zero (c = 1/2 for minmod,
    1 for MC, i.e. half of the branch slope 1 or 2)."""
    pos = a * b > 0
    mm = torch.where(a.abs() <= b.abs(), a, b)
    c = 0.5
    if limiter == "mc":
        two = 2.0 * mm
        cen = 0.5 * (a + b)
        mm = torch.where(two.abs() <= cen.abs(), two, cen)
        c = 1.0
    za, zb = a == 0, b == 0
    zero = torch.where(za & zb, 0.5 * (a + b),
           torch.where(za, c * a, torch.where(zb, c * b, torch.zeros_like(a))))
    return torch.where(pos, mm, zero)


def fast_speed(rho, p, bsq, bn2, gamma):
    a2 = gamma * p / rho
    b2 = bsq / rho
    n2 = bn2 / rho
    disc = (a2 - b2) * (a2 - b2) + 4.0 * a2 * (b2 - n2)
    disc = torch.where(disc > 0, disc, torch.zeros_like(disc))
    return torch.sqrt(0.5 * (a2 + b2 + torch.sqrt(disc)))


def _phys(q, gamma):
    rho, u, v1, v2, p, bn, b1, b2 = q
    bsq = bn * bn + b1 * b1 + b2 * b2
    pt = p + 0.5 * bsq
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v1 * v1 + v2 * v2) + 0.5 * bsq
    vb = u * bn + v1 * b1 + v2 * b2
    f = [rho * u, rho * u * u + pt - bn * bn, rho * u * v1 - bn * b1, rho * u * v2 - bn * b2,
         (E + pt) * u - bn * vb, torch.zeros_like(u), u * b1 - v1 * bn, u * b2 - v2 * bn]
    c = [rho, rho * u, rho * v1, rho * v2, E, bn, b1, b2]
    return f, c, E, pt, vb, bsq


def hll(qL, qR, gamma):
    fL, cL_, _, _, _, bsqL = _phys(qL, gamma)
    fR, cR_, _, _, _, bsqR = _phys(qR, gamma)
    cL = fast_speed(qL[0], qL[4], bsqL, qL[5] * qL[5], gamma)
    cR = fast_speed(qR[0], qR[4], bsqR, qR[5] * qR[5], gamma)
    xl, xr = qL[1] - cL, qR[1] - cR
    sL = torch.where(xl <= xr, xl, xr)
    yl, yr = qL[1] + cL, qR[1] + cR
    sR = torch.where(yl >= yr, yl, yr)
    zero = torch.zeros_like(sL)
    sLc = torch.where(sL <= 0, sL, zero)
    sRc = torch.where(sR >= 0, sR, zero)
    return [(sRc * fL[k] - sLc * fR[k] + sLc * sRc * (cR_[k] - cL_[k])) / (sRc - sLc) for k in range(8)]


def _star(q, E, pt, vb, S, sM, pts):
    rho, u, v1, v2, p, bn, b1, b2 = q
    su = S - u
    sd = S - sM
    m = rho * su
    rs = m / sd
    mm = m * sd
    bn2 = bn * bn
    D = mm - bn2
    deg = D.abs() <= 16.0 * EPS64 * (mm.abs() + bn2)
    Ds = torch.where(deg, torch.ones_like(D), D)
    cv = bn * (sM - u) / Ds
    cb = (m * su - bn2) / Ds
    vs1 = torch.where(deg, v1, v1 - b1 * cv)
    vs2 = torch.where(deg, v2, v2 - b2 * cv)
    bs1 = torch.where(deg, b1, b1 * cb)
    bs2 = torch.where(deg, b2, b2 * cb)
    vbs = sM * bn + vs1 * bs1 + vs2 * bs2
    Es = (su * E - pt * u + pts * sM + bn * (vb - vbs)) / sd
    return rs, vs1, vs2, bs1, bs2, Es, vbs


def hlld(qL, qR, gamma):
    fL, UL, EL, ptL, vbL, bsqL = _phys(qL, gamma)
    fR, UR, ER, ptR, vbR, bsqR = _phys(qR, gamma)
    bn = qL[5]
    cL = fast_speed(qL[0], qL[4], bsqL, bn * bn, gamma)
    cR = fast_speed(qR[0], qR[4], bsqR, bn * bn, gamma)
    uL, uR = qL[1], qR[1]
    # outer speeds min(u_L, u_R) - max(c_L, c_R), max(u_L, u_R) + max(c_L, c_R)
    cm = torch.where(cL >= cR, cL, cR)
    sL = torch.where(uL <= uR, uL, uR) - cm
    sR = torch.where(uL >= uR, uL, uR) + cm
    mL = (sL - uL) * qL[0]
    mR = (sR - uR) * qR[0]
    sM = (mR * uR - mL * uL - ptR + ptL) / (mR - mL)
    pts = (mR * ptL - mL * ptR + mL * mR * (uR - uL)) / (mR - mL)
    rsL, v1L, v2L, b1L, b2L, EsL, vbsL = _star(qL, EL, ptL, vbL, sL, sM, pts)
    rsR, v1R, v2R, b1R, b2R, EsR, vbsR = _star(qR, ER, ptR, vbR, sR, sM, pts)
    sqL, sqR = torch.sqrt(rsL), torch.sqrt(rsR)
    sgn = torch.where(bn >= 0, torch.ones_like(bn), -torch.ones_like(bn))
    abn = sgn * bn
    ssL = sM - abn / sqL
    ssR = sM + abn / sqR
    den = sqL + sqR
    v1s = (sqL * v1L + sqR * v1R + (b1R - b1L) * sgn) / den
    v2s = (sqL * v2L + sqR * v2R + (b2R - b2L) * sgn) / den
    b1s = (sqL * b1R + sqR * b1L + sqL * sqR * (v1R - v1L) * sgn) / den
    b2s = (sqL * b2R + sqR * b2L + sqL * sqR * (v2R - v2L) * sgn) / den
    vbss = sM * bn + v1s * b1s + v2s * b2s
    EssL = EsL - sqL * (vbsL - vbss) * sgn
    EssR = EsR + sqR * (vbsR - vbss) * sgn
    usL = [rsL, rsL * sM, rsL * v1L, rsL * v2L, EsL, bn, b1L, b2L]
    usR = [rsR, rsR * sM, rsR * v1R, rsR * v2R, EsR, bn, b1R, b2R]
    ussL = [rsL, rsL * sM, rsL * v1s, rsL * v2s, EssL, bn, b1s, b2s]
    ussR = [rsR, rsR * sM, rsR * v1s, rsR * v2s, EssR, bn, b1s, b2s]
    rL = sL >= 0
    rsLreg = (sL < 0) & (ssL >= 0)
    rssL = (ssL < 0) & (sM >= 0)
    rssR = (sM < 0) & (ssR >= 0)
    rsRreg = (ssR < 0) & (sR > 0)
    out = []
    for k in range(8):
        fsL = fL[k] + sL * (usL[k] - UL[k])
        fsR = fR[k] + sR * (usR[k] - UR[k])
        fssL = fsL + ssL * (ussL[k] - usL[k])
        fssR = fsR + ssR * (ussR[k] - usR[k])
        F = torch.where(rL, fL[k],
            torch.where(rsLreg, fsL,
            torch.where(rssL, fssL,
            torch.where(rssR, fssR,
            torch.where(rsRreg, fsR, fR[k])))))
        out.append(F)
    return out


def face_flux(VL, VR, d, setup, ch):
    """Interface flux (9 comps, unrotated) from primitive face states."""
    gamma = setup["gamma"]
    ax = [d, (d + 1) % 3, (d + 2) % 3]
    bnL, bnR = VL[5 + d], VR[5 + d]
    if setup.get("glm", True):
        bns = 0.5 * (bnL + bnR) - (VR[8] - VL[8]) / (2.0 * ch)
        psis = 0.5 * (VL[8] + VR[8]) - 0.5 * ch * (bnR - bnL)
    else:
        bns = 0.5 * (bnL + bnR)
        psis = torch.zeros_like(bnL)
    qL = [VL[0], VL[1 + ax[0]], VL[1 + ax[1]], VL[1 + ax[2]], VL[4], bns, VL[5 + ax[1]], VL[5 + ax[2]]]
    qR = [VR[0], VR[1 + ax[0]], VR[1 + ax[1]], VR[1 + ax[2]], VR[4], bns, VR[5 + ax[1]], VR[5 + ax[2]]]
    f = hlld(qL, qR, gamma) if setup["riemann"] == "hlld" else hll(qL, qR, gamma)
    F = [None] * 9
    F[0] = f[0]
    F[4] = f[4]
    F[1 + ax[0]], F[1 + ax[1]], F[1 + ax[2]] = f[1], f[2], f[3]
    F[5 + ax[1]], F[5 + ax[2]] = f[6], f[7]
    if setup.get("glm", True):
        F[5 + d] = psis
        F[8] = ch * ch * bns
    else:
        F[5 + d] = torch.zeros_like(bns)
        F[8] = torch.zeros_like(bns)
    return torch.stack(F, 0)


def rhs(U, setup, ch):
    """L(U) = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d."""
    V = cons_to_prim(U, setup["gamma"])
    L = torch.zeros_like(U)
    for d in range(setup["ndim"]):
        n = setup["n"][d]
        dx = (setup["hi"][d] - setup["lo"][d]) / n
        axis = 3 - d  # tensor axis of spatial axis d
        idx = _cat_idx(n, setup["bc"][d][0] == "periodic")
        W = torch.index_select(V, axis, idx)  # padded cells -2 .. n+1
        def sl(a, b):
            return W.narrow(axis, a, b - a)
        # slopes of padded cells 1 .. n+2 (cells -1 .. n)
        dm = sl(1, n + 3) - sl(0, n + 2)
        dp = sl(2, n + 4) - sl(1, n + 3)
        S = limited_slope(dm, dp, setup.get("limiter", "minmod"))
        C = sl(1, n + 3)
        face_L = (C + 0.5 * S).narrow(axis, 0, n + 1)      # cells -1 .. n-1
        face_R = (C - 0.5 * S).narrow(axis, 1, n + 1)      # cells  0 .. n
        F = face_flux(face_L, face_R, d, setup, ch)           # faces -1/2 .. n-1/2
        L = L - (F.narrow(axis, 1, n) - F.narrow(axis, 0, n)) / dx
    return L


def step(U, setup, dt, ch, damp):
    U1 = U + dt * rhs(U, setup, ch)
    W = 0.5 * (U + U1 + dt * rhs(U1, setup, ch))
    scale = torch.ones(9, 1, 1, 1, dtype=U.dtype)
    scale[8] = damp
    return W * scale


def rollout(U, setup, history, checkpoint=True):
    """Replay a (dt, c_h, damp) list; per-step activation checkpointing keeps
    the memory of long runs to one state per step."""
    from torch.utils.checkpoint import checkpoint as ckpt
    for dt, ch, dmp in history:
        if checkpoint and U.requires_grad:
            U = ckpt(step, U, setup, dt, ch, dmp, use_reentrant=False)
        else:
            U = step(U, setup, dt, ch, dmp)
    return U


def kinetic_energy(U, cell_volume):
    return 0.5 * ((U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]).sum() * cell_volume
