// Adjoint (vector-Jacobian product) of one SSP-RK2 step with dt, c_h and
// the GLM decay factor held fixed.
//
// Forward step:  U1 = Un + dt L(Un),  W = (Un + U1 + dt L(U1))/2,
//                U_next = D W with D scaling psi by damp.
// Given lam' = dJ/dU_next:   mu  = D lam'
//                            lam1 = mu/2 + (dt/2) J_L(U1)^T mu
//                            lamn = mu/2 + lam1 + dt J_L(Un)^T lam1
// J_L(U)^T v is built in two passes:
//   * adj_face_kernel<D> (one thread per face along axis D): recompute the
//     4-cell stencil, PLM face states and the face flux, then take the
//     flux cotangent g = (v_b - v_a)/dx_D (L_a = -(F_{a+1/2} - ..)/dx) back
//     through the Riemann solver, the GLM interface solve and the limited
//     slopes to the primitive cotangents of the 4 stencil cells, written as
//     4 x 9 contributions per face;
//   * adj_cell_kernel (one thread per cell): gather, in a fixed order, the
//     contributions of every (face, stencil position) that maps to the cell
//     (periodic wrap or outflow clamp), apply the transpose of the
//     conserved -> primitive Jacobian in FP64, and form lam1 or lamn.
// Local VJP arithmetic is in the state type T; gathering and the lambda
// combinations are FP64.  Kinks take the branch the forward took; where a
// limiter argument is exactly zero the derivative is the one a central
// difference sees (1/2 toward each zero argument for minmod, 1 for MC).
#pragma once

#include "mhd_physics.hpp"
#include "mhd_stage.hpp"

namespace mhd {

// cotangents of the rotated primaries and of the derived quantities
template <typename T> struct RBar {
    T rho = 0, u = 0, v1 = 0, v2 = 0, p = 0, bn = 0, b1 = 0, b2 = 0;
};
template <typename T> struct DBar {
    T irho = 0, bsq = 0, E = 0, pt = 0, vb = 0;
};

// reverse of rstate_finish: derived (irho, bsq, E, pt, vb) -> primaries
template <typename T>
__device__ __forceinline__ void finish_rev(const RState<T> &s, const Phys<T> &ph, const DBar<T> &d,
                                           RBar<T> &b)
{
    b.p += d.E * ph.inv_gm1 + d.pt;
    const T ke = s.u * s.u + s.v1 * s.v1 + s.v2 * s.v2;
    b.rho += T(0.5) * ke * d.E - s.irho * s.irho * d.irho;
    const T keb = T(0.5) * s.rho * d.E;
    b.u += T(2) * s.u * keb + s.bn * d.vb;
    b.v1 += T(2) * s.v1 * keb + s.b1 * d.vb;
    b.v2 += T(2) * s.v2 * keb + s.b2 * d.vb;
    const T bsqb = d.bsq + T(0.5) * d.E + T(0.5) * d.pt;
    b.bn += T(2) * s.bn * bsqb + s.u * d.vb;
    b.b1 += T(2) * s.b1 * bsqb + s.v1 * d.vb;
    b.b2 += T(2) * s.b2 * bsqb + s.v2 * d.vb;
}

// reverse of rstate_flux (physical flux f and conserved vector c)
template <typename T>
__device__ __forceinline__ void flux_rev(const RState<T> &s, const T *fb, const T *cb, RBar<T> &b,
                                         DBar<T> &d)
{
    const T mu = s.rho * s.u;
    const T mub = fb[0] + fb[1] * s.u + fb[2] * s.v1 + fb[3] * s.v2 + cb[1];
    b.u += fb[1] * mu + fb[4] * (s.E + s.pt) + fb[6] * s.b1 + fb[7] * s.b2 + mub * s.rho;
    d.pt += fb[1] + fb[4] * s.u;
    b.bn += -T(2) * s.bn * fb[1] - s.b1 * fb[2] - s.b2 * fb[3] - s.vb * fb[4] - s.v1 * fb[6] -
            s.v2 * fb[7] + cb[5];
    b.b1 += -s.bn * fb[2] + s.u * fb[6] + cb[6];
    b.b2 += -s.bn * fb[3] + s.u * fb[7] + cb[7];
    b.v1 += mu * fb[2] - s.bn * fb[6] + s.rho * cb[2];
    b.v2 += mu * fb[3] - s.bn * fb[7] + s.rho * cb[3];
    d.E += fb[4] * s.u + cb[4];
    d.vb += -s.bn * fb[4];
    b.rho += cb[0] + s.v1 * cb[2] + s.v2 * cb[3] + mub * s.u;
}

// reverse of rstate_fast: c = sqrt((a2 + b2 + sqrt(disc))/2)
template <typename T>
__device__ __forceinline__ void fast_rev(const RState<T> &s, const Phys<T> &ph, T c, T cbar, RBar<T> &b,
                                         DBar<T> &d)
{
    const T a2 = ph.gamma * s.p * s.irho, b2 = s.bsq * s.irho, bn2 = s.bn * s.bn;
    const T n2 = bn2 * s.irho;
    const T dab = a2 - b2;
    const T disc0 = dab * dab + T(4) * a2 * (b2 - n2);
    const bool dpos = disc0 > T(0);
    const T sd = Num<T>::sqrt(dpos ? disc0 : T(0));
    const T c2b = cbar * T(0.5) * Num<T>::rcp(c);
    T a2b = T(0.5) * c2b, b2b = T(0.5) * c2b;
    const T sdb = T(0.5) * c2b;
    const T discb = (dpos && sd > T(0)) ? sdb * T(0.5) * Num<T>::rcp(sd) : T(0);
    const T dabb = T(2) * dab * discb;
    a2b += dabb + T(4) * (b2 - n2) * discb;
    b2b += -dabb + T(4) * a2 * discb;
    const T n2b = -T(4) * a2 * discb;
    b.p += ph.gamma * s.irho * a2b;
    d.irho += ph.gamma * s.p * a2b + s.bsq * b2b + bn2 * n2b;
    d.bsq += s.irho * b2b;
    b.bn += T(2) * s.bn * s.irho * n2b;
}

template <typename T>
__device__ __forceinline__ void hll_vjp(const RState<T> &L, const RState<T> &R, const Phys<T> &ph,
                                        const T *Fb, RBar<T> &Lb, RBar<T> &Rb, DBar<T> &Ld,
                                        DBar<T> &Rd, T &bnb)
{
    T FL[8], UL[8], FR[8], UR[8];
    rstate_flux(L, FL, UL);
    rstate_flux(R, FR, UR);
    const T cL = rstate_fast(L, ph), cR = rstate_fast(R, ph);
    const T xL = L.u - cL, xR = R.u - cR, yL = L.u + cL, yR = R.u + cR;
    const bool selx = xL <= xR, sely = yL >= yR;
    const T xm = selx ? xL : xR, ym = sely ? yL : yR;
    const bool lneg = xm <= T(0), rpos = ym >= T(0);
    const T sL = lneg ? xm : T(0), sR = rpos ? ym : T(0);
    const T id = Num<T>::rcp(sR - sL);
    T FLb[8], FRb[8], ULb[8], URb[8];
    T sLb = 0, sRb = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const T dU = UR[k] - UL[k];
        const T F = (sR * FL[k] - sL * FR[k] + sL * sR * dU) * id;
        FLb[k] = sR * id * Fb[k];
        FRb[k] = -sL * id * Fb[k];
        URb[k] = sL * sR * id * Fb[k];
        ULb[k] = -URb[k];
        sRb += Fb[k] * (FL[k] + sL * dU - F) * id;
        sLb += Fb[k] * (-FR[k] + sR * dU + F) * id;
    }
    const T xmb = lneg ? sLb : T(0), ymb = rpos ? sRb : T(0);
    T cLb = 0, cRb = 0;
    if (selx) { Lb.u += xmb; cLb -= xmb; } else { Rb.u += xmb; cRb -= xmb; }
    if (sely) { Lb.u += ymb; cLb += ymb; } else { Rb.u += ymb; cRb += ymb; }
    flux_rev(L, FLb, ULb, Lb, Ld);
    flux_rev(R, FRb, URb, Rb, Rd);
    fast_rev(L, ph, cL, cLb, Lb, Ld);
    fast_rev(R, ph, cR, cRb, Rb, Rd);
    (void)bnb;
}

// single-star state with the intermediates its reverse needs
template <typename T> struct StarT {
    T su, sd, isd, m, rho, mm, D, iD, cv, cb, v1, v2, b1, b2, vb, Enum, E, isq, sq;
    bool deg;
};
template <typename T> struct StarB {
    T rho = 0, v1 = 0, v2 = 0, b1 = 0, b2 = 0, E = 0, vb = 0, sq = 0, isq = 0;
};

template <typename T>
__device__ __forceinline__ void star_fwd(const RState<T> &s, T S, T sM, T pts, StarT<T> &o)
{
    o.su = S - s.u;
    o.sd = S - sM;
    o.isd = Num<T>::rcp(o.sd);
    o.m = s.rho * o.su;
    o.rho = o.m * o.isd;
    o.mm = o.m * o.sd;
    const T bn2 = s.bn * s.bn;
    o.D = o.mm - bn2;
    o.deg = Num<T>::abs(o.D) <= T(16) * Num<T>::eps * (Num<T>::abs(o.mm) + bn2);
    o.iD = Num<T>::rcp(o.D);
    o.cv = s.bn * (sM - s.u) * o.iD;
    o.cb = (o.m * o.su - bn2) * o.iD;
    o.v1 = o.deg ? s.v1 : s.v1 - s.b1 * o.cv;
    o.v2 = o.deg ? s.v2 : s.v2 - s.b2 * o.cv;
    o.b1 = o.deg ? s.b1 : s.b1 * o.cb;
    o.b2 = o.deg ? s.b2 : s.b2 * o.cb;
    o.vb = sM * s.bn + o.v1 * o.b1 + o.v2 * o.b2;
    o.Enum = o.su * s.E - s.pt * s.u + pts * sM + s.bn * (s.vb - o.vb);
    o.E = o.Enum * o.isd;
    o.isq = Num<T>::rsqrt(o.rho);
    o.sq = o.rho * o.isq;
}

template <typename T>
__device__ __forceinline__ void star_rev(const RState<T> &s, T sM, T pts, const StarT<T> &o, StarB<T> ob,
                                         RBar<T> &sb, DBar<T> &sd_, T &Sb, T &sMb, T &ptsb, T &bnb)
{
    ob.rho += ob.sq * o.isq;
    ob.isq += ob.sq * o.rho;
    ob.rho += ob.isq * T(-0.5) * o.isq * o.isq * o.isq;
    const T Enumb = ob.E * o.isd;
    T isdb = ob.E * o.Enum;
    T sub = Enumb * s.E;
    sd_.E += Enumb * o.su;
    sd_.pt -= Enumb * s.u;
    sb.u -= Enumb * s.pt;
    ptsb += Enumb * sM;
    sMb += Enumb * pts;
    bnb += Enumb * (s.vb - o.vb);
    sd_.vb += Enumb * s.bn;
    ob.vb -= Enumb * s.bn;
    sMb += ob.vb * s.bn;
    bnb += ob.vb * sM;
    ob.v1 += ob.vb * o.b1;
    ob.b1 += ob.vb * o.v1;
    ob.v2 += ob.vb * o.b2;
    ob.b2 += ob.vb * o.v2;
    T mb = 0, sdb = 0;
    sb.v1 += ob.v1;
    sb.v2 += ob.v2;
    if (o.deg) {
        sb.b1 += ob.b1;
        sb.b2 += ob.b2;
    } else {
        sb.b1 += -ob.v1 * o.cv + ob.b1 * o.cb;
        sb.b2 += -ob.v2 * o.cv + ob.b2 * o.cb;
        const T cvb = -(ob.v1 * s.b1 + ob.v2 * s.b2);
        const T cbb = ob.b1 * s.b1 + ob.b2 * s.b2;
        const T smu = sM - s.u;
        bnb += cvb * smu * o.iD;
        sMb += cvb * s.bn * o.iD;
        sb.u -= cvb * s.bn * o.iD;
        T iDb = cvb * s.bn * smu;
        const T bn2 = s.bn * s.bn;
        mb += cbb * o.su * o.iD;
        sub += cbb * o.m * o.iD;
        bnb -= T(2) * s.bn * cbb * o.iD;
        iDb += cbb * (o.m * o.su - bn2);
        const T Db = -o.iD * o.iD * iDb;
        bnb -= T(2) * s.bn * Db;
        mb += Db * o.sd;
        sdb += Db * o.m;
    }
    mb += ob.rho * o.isd;
    isdb += ob.rho * o.m;
    sdb += -o.isd * o.isd * isdb;
    sb.rho += mb * o.su;
    sub += mb * s.rho;
    Sb += sub + sdb;
    sb.u -= sub;
    sMb -= sdb;
}

template <typename T>
__device__ __forceinline__ void hlld_vjp(const RState<T> &L, const RState<T> &R, const Phys<T> &ph,
                                         const T *Fb, RBar<T> &Lb, RBar<T> &Rb, DBar<T> &Ld,
                                         DBar<T> &Rd, T &bnb)
{
    // ---- forward (same arithmetic as hlld_flux) ----
    const T cL = rstate_fast(L, ph), cR = rstate_fast(R, ph);
    const T xL = L.u - cL, xR = R.u - cR, yL = L.u + cL, yR = R.u + cR;
    const bool selx = xL <= xR, sely = yL >= yR;
    const T sL = selx ? xL : xR, sR = sely ? yL : yR;
    const T mL = (sL - L.u) * L.rho, mR = (sR - R.u) * R.rho;
    const T idm = Num<T>::rcp(mR - mL);
    const T nsM = mR * R.u - mL * L.u - R.pt + L.pt;
    const T sM = nsM * idm;
    const T du = R.u - L.u;
    const T npt = mR * L.pt - mL * R.pt + mL * mR * du;
    const T pts = npt * idm;
    const T bn = L.bn;
    StarT<T> sl, sr;
    star_fwd(L, sL, sM, pts, sl);
    star_fwd(R, sR, sM, pts, sr);
    const T sgn = bn >= T(0) ? T(1) : T(-1);
    const T abn = Num<T>::abs(bn);
    const T ssL = sM - abn * sl.isq;
    const T ssR = sM + abn * sr.isq;
    const T iden = Num<T>::rcp(sl.sq + sr.sq);
    const T M1 = sl.sq * sl.v1 + sr.sq * sr.v1 + (sr.b1 - sl.b1) * sgn;
    const T M2 = sl.sq * sl.v2 + sr.sq * sr.v2 + (sr.b2 - sl.b2) * sgn;
    const T v1 = M1 * iden, v2 = M2 * iden;
    const T sqq = sl.sq * sr.sq;
    const T N1 = sl.sq * sr.b1 + sr.sq * sl.b1 + sqq * (sr.v1 - sl.v1) * sgn;
    const T N2 = sl.sq * sr.b2 + sr.sq * sl.b2 + sqq * (sr.v2 - sl.v2) * sgn;
    const T b1 = N1 * iden, b2 = N2 * iden;
    const T vbss = sM * bn + v1 * b1 + v2 * b2;
    const bool left = sM >= T(0);
    const RState<T> &S = left ? L : R;
    const StarT<T> &st = left ? sl : sr;
    const T s_out = left ? sL : sR;
    const T s_in = left ? ssL : ssR;
    const bool outer = left ? (sL >= T(0)) : (sR <= T(0));
    const bool dbl = left ? (ssL < T(0)) : (ssR >= T(0));
    const T a1 = outer ? T(0) : s_out;
    const T a2 = (outer || !dbl) ? T(0) : s_in;
    const T sig = left ? T(-1) : T(1);
    const T Ess = st.E + sig * st.sq * (st.vb - vbss) * sgn;
    T f[8], u[8];
    rstate_flux(S, f, u);
    const T us[8] = {st.rho, st.rho * sM, st.rho * st.v1, st.rho * st.v2, st.E, bn, st.b1, st.b2};
    const T uss[8] = {st.rho, st.rho * sM, st.rho * v1, st.rho * v2, Ess, bn, b1, b2};

    // ---- reverse ----
    T ub[8];
    T a1b = 0, a2b = 0;
    StarB<T> stb;
    T sMb = 0, v1b = 0, v2b = 0, b1b = 0, b2b = 0, Essb = 0, vbssb = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ub[k] = -a1 * Fb[k];
        a1b += Fb[k] * (us[k] - u[k]);
        a2b += Fb[k] * (uss[k] - us[k]);
    }
    // uss = (rho*, rho* sM, rho* v1**, rho* v2**, E**, bn, b1**, b2**), weight a2
    {
        T w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k] = a2 * Fb[k];
        stb.rho += w[0] + w[1] * sM + w[2] * v1 + w[3] * v2;
        sMb += w[1] * st.rho;
        v1b += w[2] * st.rho;
        v2b += w[3] * st.rho;
        Essb += w[4];
        bnb += w[5];
        b1b += w[6];
        b2b += w[7];
    }
    // us, weight a1 - a2
    {
        T w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k] = (a1 - a2) * Fb[k];
        stb.rho += w[0] + w[1] * sM + w[2] * st.v1 + w[3] * st.v2;
        sMb += w[1] * st.rho;
        stb.v1 += w[2] * st.rho;
        stb.v2 += w[3] * st.rho;
        stb.E += w[4];
        bnb += w[5];
        stb.b1 += w[6];
        stb.b2 += w[7];
    }
    const T s_out_b = outer ? T(0) : a1b;
    const T s_in_b = (outer || !dbl) ? T(0) : a2b;
    // E** = E*_a + sig sq_a (vb*_a - vbss) sgn
    stb.E += Essb;
    stb.sq += sig * (st.vb - vbss) * sgn * Essb;
    stb.vb += sig * st.sq * sgn * Essb;
    vbssb -= sig * st.sq * sgn * Essb;
    // vbss = sM bn + v1 b1 + v2 b2
    sMb += bn * vbssb;
    bnb += sM * vbssb;
    v1b += b1 * vbssb;
    b1b += v1 * vbssb;
    v2b += b2 * vbssb;
    b2b += v2 * vbssb;
    // double-star tangential components
    const T N1b = b1b * iden, N2b = b2b * iden, M1b = v1b * iden, M2b = v2b * iden;
    const T idenb = b1b * N1 + b2b * N2 + v1b * M1 + v2b * M2;
    StarB<T> slb, srb;
    slb.sq += N1b * sr.b1 + N2b * sr.b2 + M1b * sl.v1 + M2b * sl.v2;
    srb.sq += N1b * sl.b1 + N2b * sl.b2 + M1b * sr.v1 + M2b * sr.v2;
    srb.b1 += N1b * sl.sq + M1b * sgn;
    srb.b2 += N2b * sl.sq + M2b * sgn;
    slb.b1 += N1b * sr.sq - M1b * sgn;
    slb.b2 += N2b * sr.sq - M2b * sgn;
    const T sqqb = (N1b * (sr.v1 - sl.v1) + N2b * (sr.v2 - sl.v2)) * sgn;
    srb.v1 += N1b * sqq * sgn + M1b * sr.sq;
    slb.v1 += -N1b * sqq * sgn + M1b * sl.sq;
    srb.v2 += N2b * sqq * sgn + M2b * sr.sq;
    slb.v2 += -N2b * sqq * sgn + M2b * sl.sq;
    slb.sq += sqqb * sr.sq;
    srb.sq += sqqb * sl.sq;
    const T sqsb = -iden * iden * idenb;
    slb.sq += sqsb;
    srb.sq += sqsb;
    // inner speeds s*L = sM - |bn| isq_L, s*R = sM + |bn| isq_R
    T abnb = 0;
    if (left) {
        sMb += s_in_b;
        abnb -= s_in_b * sl.isq;
        slb.isq -= s_in_b * abn;
    } else {
        sMb += s_in_b;
        abnb += s_in_b * sr.isq;
        srb.isq += s_in_b * abn;
    }
    bnb += sgn * abnb;
    // the side's own star cotangents
    StarB<T> &sideb = left ? slb : srb;
    sideb.rho += stb.rho;
    sideb.v1 += stb.v1;
    sideb.v2 += stb.v2;
    sideb.b1 += stb.b1;
    sideb.b2 += stb.b2;
    sideb.E += stb.E;
    sideb.vb += stb.vb;
    sideb.sq += stb.sq;
    sideb.isq += stb.isq;
    T sLb = left ? s_out_b : T(0);
    T sRb = left ? T(0) : s_out_b;
    T ptsb = 0;
    star_rev(L, sM, pts, sl, slb, Lb, Ld, sLb, sMb, ptsb, bnb);
    star_rev(R, sM, pts, sr, srb, Rb, Rd, sRb, sMb, ptsb, bnb);
    // pts = npt idm, sM = nsM idm
    const T nptb = ptsb * idm;
    T idmb = ptsb * npt + sMb * nsM;
    const T nsMb = sMb * idm;
    T mRb = nptb * (L.pt + mL * du) + nsMb * R.u;
    T mLb = nptb * (-R.pt + mR * du) - nsMb * L.u;
    Ld.pt += nptb * mR + nsMb;
    Rd.pt += -nptb * mL - nsMb;
    const T dub = nptb * mL * mR;
    Rb.u += dub + nsMb * mR;
    Lb.u += -dub - nsMb * mL;
    const T denb = -idm * idm * idmb;
    mRb += denb;
    mLb -= denb;
    sLb += mLb * L.rho;
    Lb.u -= mLb * L.rho;
    Lb.rho += mLb * (sL - L.u);
    sRb += mRb * R.rho;
    Rb.u -= mRb * R.rho;
    Rb.rho += mRb * (sR - R.u);
    T cLb = 0, cRb = 0;
    if (selx) { Lb.u += sLb; cLb -= sLb; } else { Rb.u += sLb; cRb -= sLb; }
    if (sely) { Lb.u += sRb; cLb += sRb; } else { Rb.u += sRb; cRb += sRb; }
    // flux and conserved vector of the side state (F = f + a1 (us - u) + ...)
    if (left)
        flux_rev(L, Fb, ub, Lb, Ld);
    else
        flux_rev(R, Fb, ub, Rb, Rd);
    fast_rev(L, ph, cL, cLb, Lb, Ld);
    fast_rev(R, ph, cR, cRb, Rb, Rd);
}

// VJP of face_flux along a compile-time axis D: given gb = dJ/dF (9 comps,
// unrotated), return dJ/dVL and dJ/dVR (primitive face states).
template <typename T, int SOLVER, int D>
__device__ __forceinline__ void face_flux_vjp(const T *VL, const T *VR, const Phys<T> &ph, const T *gb,
                                              T *VLb, T *VRb)
{
    constexpr int d1 = D == 2 ? 0 : D + 1;
    constexpr int d2 = D == 0 ? 2 : D - 1;
    const T bnL = VL[BX + D], bnR = VR[BX + D];
    T bns;
    if (ph.glm)
        bns = T(0.5) * (bnL + bnR) - (VR[PSI] - VL[PSI]) * ph.half_ich;
    else
        bns = T(0.5) * (bnL + bnR);
    RState<T> L, R;
    L.rho = VL[RHO]; L.u = VL[VX + D]; L.v1 = VL[VX + d1]; L.v2 = VL[VX + d2]; L.p = VL[PRS];
    L.bn = bns; L.b1 = VL[BX + d1]; L.b2 = VL[BX + d2];
    R.rho = VR[RHO]; R.u = VR[VX + D]; R.v1 = VR[VX + d1]; R.v2 = VR[VX + d2]; R.p = VR[PRS];
    R.bn = bns; R.b1 = VR[BX + d1]; R.b2 = VR[BX + d2];
    rstate_finish(L, ph);
    rstate_finish(R, ph);
    const T fb[8] = {gb[RHO], gb[MX + D], gb[MX + d1], gb[MX + d2], gb[ENG], T(0), gb[BX + d1], gb[BX + d2]};
    const T psisb = ph.glm ? gb[BX + D] : T(0);
    T bnsb = ph.glm ? ph.ch2 * gb[PSI] : T(0);
    RBar<T> Lb, Rb;
    DBar<T> Ld, Rd;
    if (SOLVER == SOLVER_HLLD)
        hlld_vjp(L, R, ph, fb, Lb, Rb, Ld, Rd, bnsb);
    else
        hll_vjp(L, R, ph, fb, Lb, Rb, Ld, Rd, bnsb);
    finish_rev(L, ph, Ld, Lb);
    finish_rev(R, ph, Rd, Rb);
    bnsb += Lb.bn + Rb.bn;
    VLb[RHO] = Lb.rho; VLb[VX + D] = Lb.u; VLb[VX + d1] = Lb.v1; VLb[VX + d2] = Lb.v2;
    VLb[PRS] = Lb.p; VLb[BX + d1] = Lb.b1; VLb[BX + d2] = Lb.b2;
    VRb[RHO] = Rb.rho; VRb[VX + D] = Rb.u; VRb[VX + d1] = Rb.v1; VRb[VX + d2] = Rb.v2;
    VRb[PRS] = Rb.p; VRb[BX + d1] = Rb.b1; VRb[BX + d2] = Rb.b2;
    if (ph.glm) {
        VLb[BX + D] = T(0.5) * bnsb + T(0.5) * ph.ch * psisb;
        VRb[BX + D] = T(0.5) * bnsb - T(0.5) * ph.ch * psisb;
        VLb[PSI] = bnsb * ph.half_ich + T(0.5) * psisb;
        VRb[PSI] = -bnsb * ph.half_ich + T(0.5) * psisb;
    } else {
        VLb[BX + D] = VRb[BX + D] = T(0.5) * bnsb;
        VLb[PSI] = VRb[PSI] = T(0);
    }
}

// limited slope with its derivative coefficients (dp, dq) w.r.t. the
// backward and forward differences a and b
template <typename T>
__device__ __forceinline__ T slope_d(T a, T b, int limiter, T &dp, T &dq)
{
    const T aa = Num<T>::abs(a), ab = Num<T>::abs(b);
    const bool pos = a * b > T(0);
    const bool left = aa <= ab;
    T m = left ? a : b;
    T cp = left ? T(1) : T(0), cq = left ? T(0) : T(1);
    T c0 = T(0.5);
    if (limiter == LIM_MC) {
        const T two = T(2) * m, cen = T(0.5) * (a + b);
        const bool tw = Num<T>::abs(two) <= Num<T>::abs(cen);
        m = tw ? two : cen;
        cp = tw ? T(2) * cp : T(0.5);
        cq = tw ? T(2) * cq : T(0.5);
        c0 = T(1);
    }
    const bool za = a == T(0), zb = b == T(0);
    dp = pos ? cp : ((za && zb) ? T(0.5) : (za ? c0 : T(0)));
    dq = pos ? cq : ((za && zb) ? T(0.5) : (zb ? c0 : T(0)));
    return pos ? m : T(0);
}

template <typename T> struct AdjArgs {
    const T *U;           // state the stage VJP linearises about (Un or U1)
    const double *lam;    // cotangent v of L (lam' for the stage-2 VJP, lam1 for stage 1)
    double psi_scale;     // damp for the stage-2 VJP (v = D lam'), 1 otherwise
    T *C;                 // contributions [36][nfaces] of this axis
    int *flag;
    int n[3];
    long long nxy, ncell;
    int per[3];
    int nf;               // faces along the axis: n (periodic) or n + 1 (outflow)
    long long nfaces;
    double idx;           // 1/dx along the axis
    Phys<T> ph;
};

template <typename T, int SOLVER, int D>
__global__ void __launch_bounds__(256) adj_face_kernel(const AdjArgs<T> a)
{
    const long long fid = (long long)blockIdx.x * 256 + threadIdx.x;
    if (fid >= a.nfaces) return;
    int e[3] = {a.n[0], a.n[1], a.n[2]};
    e[D] = a.nf;
    int c3[3];
    c3[0] = (int)(fid % e[0]);
    c3[1] = (int)((fid / e[0]) % e[1]);
    c3[2] = (int)(fid / ((long long)e[0] * e[1]));
    const int f = c3[D];
    const int n = a.n[D];
    const bool outflow = !a.per[D];
    auto cell = [&](int pos) -> long long {
        int c[3] = {c3[0], c3[1], c3[2]};
        c[D] = remap_index(pos, n, a.per[D]);
        return ((long long)c[2] * a.n[1] + c[1]) * a.n[0] + c[0];
    };
    T W[4][NQ];
    bool ok = true;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        T u[NQ];
        load_cell(a.U, a.ncell, cell(f - 2 + m), u);
        ok &= cons_to_prim(u, a.ph, W[m]);
    }
    if (!ok) atomicOr(a.flag, 1);
    T VL[NQ], VR[NQ], dp1[NQ], dq1[NQ], dp2[NQ], dq2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T s1 = slope_d(W[1][q] - W[0][q], W[2][q] - W[1][q], a.ph.limiter, dp1[q], dq1[q]);
        const T s2 = slope_d(W[2][q] - W[1][q], W[3][q] - W[2][q], a.ph.limiter, dp2[q], dq2[q]);
        VL[q] = W[1][q] + T(0.5) * s1;
        VR[q] = W[2][q] - T(0.5) * s2;
    }
    // flux cotangent: F enters L_b (+1/dx) and L_a (-1/dx), a = f-1, b = f;
    // an outflow boundary face has no interior cell on its outer side
    const bool has_a = !(outflow && f == 0), has_b = !(outflow && f == n);
    const long long ca = cell(f - 1), cb = cell(f);
    T gb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double sc = q == PSI ? a.psi_scale : 1.0;
        const double va = has_a ? a.lam[q * a.ncell + ca] : 0.0;
        const double vb = has_b ? a.lam[q * a.ncell + cb] : 0.0;
        gb[q] = (T)((vb - va) * sc * a.idx);
    }
    T VLb[NQ], VRb[NQ];
    face_flux_vjp<T, SOLVER, D>(VL, VR, a.ph, gb, VLb, VRb);
    // PLM reverse: VL = W1 + s1/2, VR = W2 - s2/2, s1 = lim(W1-W0, W2-W1),
    // s2 = lim(W2-W1, W3-W2)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T s1b = T(0.5) * VLb[q], s2b = T(-0.5) * VRb[q];
        const T p1 = s1b * dp1[q], q1 = s1b * dq1[q], p2 = s2b * dp2[q], q2 = s2b * dq2[q];
        const long long base = (long long)q * a.nfaces + fid;
        a.C[base] = -p1;                                        // cell f-2
        a.C[base + 9 * a.nfaces] = VLb[q] + p1 - q1 - p2;       // cell f-1
        a.C[base + 18 * a.nfaces] = VRb[q] + q1 + p2 - q2;      // cell f
        a.C[base + 27 * a.nfaces] = q2;                         // cell f+1
    }
}

template <typename T> struct AdjCellArgs {
    const T *U;             // state of the linearisation
    const T *C[3];          // contributions per axis
    long long nfaces[3];
    int nf[3];
    int n[3];
    int per[3];
    long long ncell;
    double gm1;
    const double *lamp;     // lam' = dJ/dU_next
    const double *lam1;     // stage-1 pass only
    double *out;            // lam1 (stage-2 pass) or lamn (stage-1 pass)
    double damp, dt;
};

template <typename T, int NDIM, int PASS>
__global__ void __launch_bounds__(256) adj_cell_kernel(const AdjCellArgs<T> a)
{
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= a.ncell) return;
    const int ci[3] = {(int)(c % a.n[0]), (int)((c / a.n[0]) % a.n[1]),
                       (int)(c / ((long long)a.n[0] * a.n[1]))};
    double vb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) vb[q] = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        const int n = a.n[d], x = ci[d];
        auto add = [&](int f, int m) {
            int e[3] = {ci[0], ci[1], ci[2]};
            int ne[3] = {a.n[0], a.n[1], a.n[2]};
            e[d] = f;
            ne[d] = a.nf[d];
            const long long fid = ((long long)e[2] * ne[1] + e[1]) * ne[0] + e[0];
            const T *Cd = a.C[d];
#pragma unroll
            for (int q = 0; q < NQ; ++q) vb[q] += (double)Cd[((long long)m * NQ + q) * a.nfaces[d] + fid];
        };
        // faces whose stencil position f-2+m is this cell
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int f = x + 2 - m;
            if (a.per[d]) {
                f = f >= n ? f - n : (f < 0 ? f + n : f);
                add(f, m);
            } else if (f >= 0 && f <= n) {
                add(f, m);
            }
        }
        if (!a.per[d]) {
            // ghost positions clamped onto the boundary cells
            if (x == 0) {
                add(0, 0);
                add(0, 1);
                add(1, 0);
            }
            if (x == n - 1) {
                add(n, 2);
                add(n, 3);
                add(n - 1, 3);
            }
        }
    }
    // transpose of the conserved -> primitive Jacobian (FP64)
    double u[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) u[q] = (double)a.U[q * a.ncell + c];
    const double ir = 1.0 / u[RHO];
    const double v[3] = {u[MX] * ir, u[MY] * ir, u[MZ] * ir};
    const double vsq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double r[NQ];
    r[RHO] = vb[RHO] - (v[0] * vb[VX] + v[1] * vb[VY] + v[2] * vb[VZ]) * ir + a.gm1 * 0.5 * vsq * vb[PRS];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[MX + k] = vb[VX + k] * ir - a.gm1 * v[k] * vb[PRS];
        r[BX + k] = vb[BX + k] - a.gm1 * u[BX + k] * vb[PRS];
    }
    r[ENG] = a.gm1 * vb[PRS];
    r[PSI] = vb[PSI];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double mu = a.lamp[q * a.ncell + c] * (q == PSI ? a.damp : 1.0);
        double o;
        if (PASS == 2)
            o = 0.5 * mu + 0.5 * a.dt * r[q];
        else
            o = 0.5 * mu + a.lam1[q * a.ncell + c] + a.dt * r[q];
        a.out[q * a.ncell + c] = o;
    }
}

} // namespace mhd
