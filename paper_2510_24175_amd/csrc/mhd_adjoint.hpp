// Adjoint (vector-Jacobian product) of one SSP-RK2 step with dt, c_h and
// the GLM decay factor held fixed.
//
// Forward step:  U1 = Un + dt L(Un),  W = (Un + U1 + dt L(U1))/2,
//                U_next = D W with D scaling psi by damp.
// Given lam' = dJ/dU_next:   mu  = D lam'
//                            lam1 = mu/2 + (dt/2) J_L(U1)^T mu
//                            lamn = mu/2 + lam1 + dt J_L(Un)^T lam1
// Each line is one fused pass over the grid (adj_stage_kernel below): the
// face VJPs (recomputed stencil, PLM, GLM interface solve and Riemann
// solver, reversed) are taken per tile in LDS, the limited-slope reverse and
// the gather to cells follow in the same workgroup, and the primitive ->
// conserved transpose and the lambda combination close the pass.
// Local VJP arithmetic is in the state type T; the transpose to conserved
// cotangents and the lambda combinations are FP64.  Kinks take the branch
// the forward took; where a limiter argument is exactly zero the derivative
// is the one a central difference sees (1/2 toward each zero argument for
// minmod, 1 for MC).
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

// reverse of rstate_prepare: cotangents of (irho, bsq, pt) -> primaries
template <typename T>
__device__ __forceinline__ void prepare_rev(const RState<T> &s, const DBar<T> &d, RBar<T> &b)
{
    b.p += d.pt;
    b.rho -= s.irho * s.irho * d.irho;
    const T bsqb = d.bsq + T(0.5) * d.pt;
    b.bn += T(2) * s.bn * bsqb;
    b.b1 += T(2) * s.b1 * bsqb;
    b.b2 += T(2) * s.b2 * bsqb;
}

// reverse of rstate_energy: cotangents of (E, v.B) -> primaries
template <typename T>
__device__ __forceinline__ void energy_rev(const RState<T> &s, const Phys<T> &ph, T Eb, T vbb, RBar<T> &b)
{
    b.p += Eb * ph.inv_gm1;
    b.rho += T(0.5) * (s.u * s.u + s.v1 * s.v1 + s.v2 * s.v2) * Eb;
    const T rE = s.rho * Eb;
    b.u += s.u * rE + s.bn * vbb;
    b.v1 += s.v1 * rE + s.b1 * vbb;
    b.v2 += s.v2 * rE + s.b2 * vbb;
    b.bn += s.bn * Eb + s.u * vbb;
    b.b1 += s.b1 * Eb + s.v1 * vbb;
    b.b2 += s.b2 * Eb + s.v2 * vbb;
}

// reverse of rstate_flux (physical flux f and conserved vector c); the
// cotangents of E, v.B and pt go to d
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

// fast speed of a prepared state (same arithmetic as fast_speed), with the
// root of the discriminant that its reverse reuses
template <typename T>
__device__ __forceinline__ T fast_fwd(const RState<T> &s, const Phys<T> &ph, T &sd)
{
    const T a2 = ph.gamma * s.p * s.irho;
    const T b2 = s.bsq * s.irho;
    const T bn2 = (s.bn * s.bn) * s.irho;
    const T dab = a2 - b2;
    T disc = dab * dab + T(4) * a2 * (b2 - bn2);
    disc = Num<T>::max(disc, T(0));
    sd = Num<T>::sqrt(disc);
    return Num<T>::sqrt(T(0.5) * (a2 + b2 + sd));
}

// reverse of fast_fwd: c = sqrt((a2 + b2 + sd)/2), sd = sqrt(max(disc, 0))
template <typename T>
__device__ __forceinline__ void fast_rev(const RState<T> &s, const Phys<T> &ph, T c, T sd, T cbar,
                                         RBar<T> &b, DBar<T> &d)
{
    const T a2 = ph.gamma * s.p * s.irho, b2 = s.bsq * s.irho, bn2 = s.bn * s.bn;
    const T n2 = bn2 * s.irho;
    const T dab = a2 - b2;
    const T c2b = cbar * T(0.5) * Num<T>::rcp(c);
    T a2b = T(0.5) * c2b, b2b = T(0.5) * c2b;
    const T discb = sd > T(0) ? T(0.25) * c2b * Num<T>::rcp(sd) : T(0);
    const T dabb = T(2) * dab * discb;
    a2b += dabb + T(4) * (b2 - n2) * discb;
    b2b += -dabb + T(4) * a2 * discb;
    const T n2b = -T(4) * a2 * discb;
    b.p += ph.gamma * s.irho * a2b;
    d.irho += ph.gamma * s.p * a2b + s.bsq * b2b + bn2 * n2b;
    d.bsq += s.irho * b2b;
    b.bn += T(2) * s.bn * s.irho * n2b;
}

// HLL VJP on prepared states; their energies are formed here (as hll_flux
// does) and reversed here, so Ld and Rd return irho, bsq and pt cotangents
template <typename T>
__device__ __forceinline__ void hll_vjp(const RState<T> &L, const RState<T> &R, const Phys<T> &ph,
                                        const T *Fb, RBar<T> &Lb, RBar<T> &Rb, DBar<T> &Ld,
                                        DBar<T> &Rd, T &bnb)
{
    RState<T> Le = L, Re = R;
    rstate_energy(Le, ph);
    rstate_energy(Re, ph);
    T FL[8], UL[8], FR[8], UR[8];
    rstate_flux(Le, FL, UL);
    rstate_flux(Re, FR, UR);
    T sdL, sdR;
    const T cL = fast_fwd(L, ph, sdL), cR = fast_fwd(R, ph, sdR);
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
    flux_rev(Le, FLb, ULb, Lb, Ld);
    flux_rev(Re, FRb, URb, Rb, Rd);
    energy_rev(Le, ph, Ld.E, Ld.vb, Lb);
    energy_rev(Re, ph, Rd.E, Rd.vb, Rb);
    fast_rev(L, ph, cL, sdL, cLb, Lb, Ld);
    fast_rev(R, ph, cR, sdR, cRb, Rb, Rd);
    (void)bnb;
}

// single-star state without its energy (formed for the picked side only),
// with the intermediates its reverse needs
template <typename T> struct StarT {
    T su, sd, isd, m, rho, mm, D, iD, cv, cb, v1, v2, b1, b2, isq, sq;
    bool deg;
};
// cotangents of a single-star state's outputs and of S - u and 1/(S - S_M)
template <typename T> struct StarB {
    T rho = 0, v1 = 0, v2 = 0, b1 = 0, b2 = 0, sq = 0, isq = 0, su = 0, isd = 0;
};

template <typename T>
__device__ __forceinline__ void star_fwd(const RState<T> &s, T S, T sM, StarT<T> &o)
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
    o.isq = Num<T>::rsqrt(o.rho);
    o.sq = o.rho * o.isq;
}

template <typename T>
__device__ __forceinline__ void star_rev(const RState<T> &s, T sM, const StarT<T> &o, const StarB<T> &ob,
                                         RBar<T> &sb, T &Sb, T &sMb, T &bnb)
{
    // sq = rho isq, isq = rho^(-1/2)
    const T isqb = ob.isq + ob.sq * o.rho;
    const T rhob = ob.rho + ob.sq * o.isq - T(0.5) * o.isq * o.isq * o.isq * isqb;
    T mb = 0, sdb = 0, sub = ob.su, isdb = ob.isd;
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
    mb += rhob * o.isd;
    isdb += rhob * o.m;
    sdb += -o.isd * o.isd * isdb;
    sb.rho += mb * o.su;
    sub += mb * s.rho;
    Sb += sub + sdb;
    sb.u -= sub;
    sMb -= sdb;
}

// field-wise selects (a select of references would put both structs in
// private memory)
template <typename T>
__device__ __forceinline__ RState<T> pick_state(bool c, const RState<T> &a, const RState<T> &b)
{
    RState<T> o;
    o.rho = c ? a.rho : b.rho; o.u = c ? a.u : b.u; o.v1 = c ? a.v1 : b.v1; o.v2 = c ? a.v2 : b.v2;
    o.p = c ? a.p : b.p; o.bn = c ? a.bn : b.bn; o.b1 = c ? a.b1 : b.b1; o.b2 = c ? a.b2 : b.b2;
    o.irho = c ? a.irho : b.irho; o.bsq = c ? a.bsq : b.bsq; o.E = c ? a.E : b.E;
    o.pt = c ? a.pt : b.pt; o.vb = c ? a.vb : b.vb;
    return o;
}
// HLLD VJP on prepared states (Miyoshi & Kusano 2005, same arithmetic and
// decisions as hlld_flux): the forward is recomputed, then reversed
// statement by statement.  The side the flux is taken from (left of the
// contact when S_M >= 0) alone carries energies; its cotangents are added to
// the left or right accumulators with 0/1 weights.
template <typename T>
__device__ __forceinline__ void hlld_vjp(const RState<T> &L, const RState<T> &R, const Phys<T> &ph,
                                         const T *Fb, RBar<T> &Lb, RBar<T> &Rb, DBar<T> &Ld,
                                         DBar<T> &Rd, T &bnb)
{
    // ---- forward ----
    T sdL, sdR;
    const T cL = fast_fwd(L, ph, sdL), cR = fast_fwd(R, ph, sdR);
    // outer speeds as hlld_flux; ties pick the left state
    const bool uminl = L.u <= R.u, umaxl = L.u >= R.u, cmaxl = cL >= cR;
    const T cm = cmaxl ? cL : cR;
    const T sL = (uminl ? L.u : R.u) - cm, sR = (umaxl ? L.u : R.u) + cm;
    const T mL = (sL - L.u) * L.rho, mR = (sR - R.u) * R.rho;
    const T idm = Num<T>::rcp(mR - mL);
    const T nsM = mR * R.u - mL * L.u - R.pt + L.pt;
    const T sM = nsM * idm;
    const T du = R.u - L.u;
    const T npt = mR * L.pt - mL * R.pt + mL * mR * du;
    const T pts = npt * idm;
    const T bn = L.bn;
    StarT<T> sl, sr;
    star_fwd(L, sL, sM, sl);
    star_fwd(R, sR, sM, sr);
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
    const T wl = left ? T(1) : T(0), wr = T(1) - wl;
    RState<T> S = pick_state(left, L, R);
    rstate_energy(S, ph);
    StarT<T> st;
    st.su = left ? sl.su : sr.su; st.sd = left ? sl.sd : sr.sd; st.isd = left ? sl.isd : sr.isd;
    st.m = left ? sl.m : sr.m; st.rho = left ? sl.rho : sr.rho; st.mm = left ? sl.mm : sr.mm;
    st.D = left ? sl.D : sr.D; st.iD = left ? sl.iD : sr.iD; st.cv = left ? sl.cv : sr.cv;
    st.cb = left ? sl.cb : sr.cb; st.v1 = left ? sl.v1 : sr.v1; st.v2 = left ? sl.v2 : sr.v2;
    st.b1 = left ? sl.b1 : sr.b1; st.b2 = left ? sl.b2 : sr.b2;
    st.isq = left ? sl.isq : sr.isq; st.sq = left ? sl.sq : sr.sq; st.deg = left ? sl.deg : sr.deg;
    // single-star energy of the picked side
    const T vbs = sM * bn + st.v1 * st.b1 + st.v2 * st.b2;
    const T Enum = st.su * S.E - S.pt * S.u + pts * sM + bn * (S.vb - vbs);
    const T Es = Enum * st.isd;
    const T s_out = left ? sL : sR;
    const T s_in = left ? ssL : ssR;
    const bool outer = left ? (sL >= T(0)) : (sR <= T(0));
    const bool dbl = left ? (ssL < T(0)) : (ssR >= T(0));
    const T a1 = outer ? T(0) : s_out;
    const T a2 = (outer || !dbl) ? T(0) : s_in;
    const T sig = left ? T(-1) : T(1);
    const T Ess = Es + sig * st.sq * (vbs - vbss) * sgn;
    T f[8], u[8];
    rstate_flux(S, f, u);
    const T us[8] = {st.rho, st.rho * sM, st.rho * st.v1, st.rho * st.v2, Es, bn, st.b1, st.b2};
    const T uss[8] = {st.rho, st.rho * sM, st.rho * v1, st.rho * v2, Ess, bn, b1, b2};

    // ---- reverse ----
    // F = f + a1 (us - u) + a2 (uss - us)
    T ub[8];
    T a1b = 0, a2b = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ub[k] = -a1 * Fb[k];
        a1b += Fb[k] * (us[k] - u[k]);
        a2b += Fb[k] * (uss[k] - us[k]);
    }
    StarB<T> stb;
    T sMb, v1b, v2b, b1b, b2b, Essb, Esb;
    {
        // uss with weight a2, us with weight a1 - a2
        T w[8], x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            w[k] = a2 * Fb[k];
            x[k] = (a1 - a2) * Fb[k];
        }
        stb.rho = w[0] + w[1] * sM + w[2] * v1 + w[3] * v2 + x[0] + x[1] * sM + x[2] * st.v1 + x[3] * st.v2;
        sMb = (w[1] + x[1]) * st.rho;
        v1b = w[2] * st.rho;
        v2b = w[3] * st.rho;
        Essb = w[4];
        bnb += w[5] + x[5];
        b1b = w[6];
        b2b = w[7];
        stb.v1 = x[2] * st.rho;
        stb.v2 = x[3] * st.rho;
        Esb = x[4];
        stb.b1 = x[6];
        stb.b2 = x[7];
    }
    const T s_out_b = outer ? T(0) : a1b;
    const T s_in_b = (outer || !dbl) ? T(0) : a2b;
    // E** = E* + sig sq* (v*.B* - v**.B**) sgn
    Esb += Essb;
    stb.sq = sig * (vbs - vbss) * sgn * Essb;
    T vbsb = sig * st.sq * sgn * Essb;
    const T vbssb = -vbsb;
    // vbss = sM bn + v1 b1 + v2 b2
    sMb += bn * vbssb;
    bnb += sM * vbssb;
    v1b += b1 * vbssb;
    b1b += v1 * vbssb;
    v2b += b2 * vbssb;
    b2b += v2 * vbssb;
    // picked single-star energy: Es = Enum isd, vbs = sM bn + v1* b1* + v2* b2*
    const T Enumb = Esb * st.isd;
    stb.isd = Esb * Enum;
    stb.su = Enumb * S.E;
    RBar<T> xb;
    DBar<T> xd;
    xd.E = Enumb * st.su;
    xd.pt = -Enumb * S.u;
    xb.u = -Enumb * S.pt;
    T ptsb = Enumb * sM;
    sMb += Enumb * pts;
    bnb += Enumb * (S.vb - vbs);
    xd.vb = Enumb * bn;
    vbsb -= Enumb * bn;
    sMb += vbsb * bn;
    bnb += vbsb * sM;
    stb.v1 += vbsb * st.b1;
    stb.b1 += vbsb * st.v1;
    stb.v2 += vbsb * st.b2;
    stb.b2 += vbsb * st.v2;
    // double-star tangential components
    const T N1b = b1b * iden, N2b = b2b * iden, M1b = v1b * iden, M2b = v2b * iden;
    const T idenb = b1b * N1 + b2b * N2 + v1b * M1 + v2b * M2;
    StarB<T> slb, srb;
    const T sqqb = (N1b * (sr.v1 - sl.v1) + N2b * (sr.v2 - sl.v2)) * sgn;
    const T sqsb = -iden * iden * idenb;
    slb.sq = N1b * sr.b1 + N2b * sr.b2 + M1b * sl.v1 + M2b * sl.v2 + sqqb * sr.sq + sqsb;
    srb.sq = N1b * sl.b1 + N2b * sl.b2 + M1b * sr.v1 + M2b * sr.v2 + sqqb * sl.sq + sqsb;
    srb.b1 = N1b * sl.sq + M1b * sgn;
    srb.b2 = N2b * sl.sq + M2b * sgn;
    slb.b1 = N1b * sr.sq - M1b * sgn;
    slb.b2 = N2b * sr.sq - M2b * sgn;
    srb.v1 = N1b * sqq * sgn + M1b * sr.sq;
    slb.v1 = -N1b * sqq * sgn + M1b * sl.sq;
    srb.v2 = N2b * sqq * sgn + M2b * sr.sq;
    slb.v2 = -N2b * sqq * sgn + M2b * sl.sq;
    // inner speeds s*L = sM - |bn| isq_L, s*R = sM + |bn| isq_R
    sMb += s_in_b;
    slb.isq = -wl * s_in_b * abn;
    srb.isq = wr * s_in_b * abn;
    bnb += sgn * s_in_b * (wr * sr.isq - wl * sl.isq);
    // the picked side's own star cotangents
    slb.rho = wl * stb.rho; srb.rho = wr * stb.rho;
    slb.v1 += wl * stb.v1; srb.v1 += wr * stb.v1;
    slb.v2 += wl * stb.v2; srb.v2 += wr * stb.v2;
    slb.b1 += wl * stb.b1; srb.b1 += wr * stb.b1;
    slb.b2 += wl * stb.b2; srb.b2 += wr * stb.b2;
    slb.sq += wl * stb.sq; srb.sq += wr * stb.sq;
    slb.su = wl * stb.su; srb.su = wr * stb.su;
    slb.isd = wl * stb.isd; srb.isd = wr * stb.isd;
    T sLb = wl * s_out_b;
    T sRb = wr * s_out_b;
    star_rev(L, sM, sl, slb, Lb, sLb, sMb, bnb);
    star_rev(R, sM, sr, srb, Rb, sRb, sMb, bnb);
    // pts = npt idm, sM = nsM idm
    const T nptb = ptsb * idm;
    const T idmb = ptsb * npt + sMb * nsM;
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
    if (uminl) Lb.u += sLb; else Rb.u += sLb;
    if (umaxl) Lb.u += sRb; else Rb.u += sRb;
    if (cmaxl) cLb += sRb - sLb; else cRb += sRb - sLb;
    // flux, conserved vector and energy of the picked side
    flux_rev(S, Fb, ub, xb, xd);
    energy_rev(S, ph, xd.E, xd.vb, xb);
    Lb.rho += wl * xb.rho; Rb.rho += wr * xb.rho;
    Lb.u += wl * xb.u; Rb.u += wr * xb.u;
    Lb.v1 += wl * xb.v1; Rb.v1 += wr * xb.v1;
    Lb.v2 += wl * xb.v2; Rb.v2 += wr * xb.v2;
    Lb.p += wl * xb.p; Rb.p += wr * xb.p;
    Lb.bn += wl * xb.bn; Rb.bn += wr * xb.bn;
    Lb.b1 += wl * xb.b1; Rb.b1 += wr * xb.b1;
    Lb.b2 += wl * xb.b2; Rb.b2 += wr * xb.b2;
    Ld.pt += wl * xd.pt; Rd.pt += wr * xd.pt;
    fast_rev(L, ph, cL, sdL, cLb, Lb, Ld);
    fast_rev(R, ph, cR, sdR, cRb, Rb, Rd);
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
    rstate_prepare(L);
    rstate_prepare(R);
    const T fb[8] = {gb[RHO], gb[MX + D], gb[MX + d1], gb[MX + d2], gb[ENG], T(0), gb[BX + d1], gb[BX + d2]};
    const T psisb = ph.glm ? gb[BX + D] : T(0);
    T bnsb = ph.glm ? ph.ch2 * gb[PSI] : T(0);
    RBar<T> Lb, Rb;
    DBar<T> Ld, Rd;
    if (SOLVER == SOLVER_HLLD)
        hlld_vjp(L, R, ph, fb, Lb, Rb, Ld, Rd, bnsb);
    else
        hll_vjp(L, R, ph, fb, Lb, Rb, Ld, Rd, bnsb);
    prepare_rev(L, Ld, Lb);
    prepare_rev(R, Rd, Rb);
    bnsb += Lb.bn + Rb.bn;
    VLb[RHO] = Lb.rho; VLb[VX + D] = Lb.u; VLb[VX + d1] = Lb.v1; VLb[VX + d2] = Lb.v2;
    VLb[PRS] = Lb.p; VLb[BX + d1] = Lb.b1; VLb[BX + d2] = Lb.b2;
    VRb[RHO] = Rb.rho; VRb[VX + D] = Rb.u; VRb[VX + d1] = Rb.v1; VRb[VX + d2] = Rb.v2;
    VRb[PRS] = Rb.p; VRb[BX + d1] = Rb.b1; VRb[BX + d2] = Rb.b2;
    // (without GLM, psisb = 0 and ch = half_ich = 0: the psi cotangents vanish)
    VLb[BX + D] = T(0.5) * bnsb + T(0.5) * ph.ch * psisb;
    VRb[BX + D] = T(0.5) * bnsb - T(0.5) * ph.ch * psisb;
    VLb[PSI] = bnsb * ph.half_ich + T(0.5) * psisb;
    VRb[PSI] = -bnsb * ph.half_ich + T(0.5) * psisb;
}

// limited slope with its derivative coefficients (dp, dq) w.r.t. the
// backward and forward differences a and b
template <int LIM, typename T>
__device__ __forceinline__ T slope_d(T a, T b, T &dp, T &dq)
{
    const T aa = Num<T>::abs(a), ab = Num<T>::abs(b);
    const bool pos = a * b > T(0);
    const bool left = aa <= ab;
    T m = left ? a : b;
    T cp = left ? T(1) : T(0), cq = left ? T(0) : T(1);
    T c0 = T(0.5);
    if (LIM == LIM_MC) {
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


// ---------------------------------------------------------------------------
// Fused adjoint stage.
//
// One pass over the grid forms r = J_L(U)^T v for every cell and combines it
// with mu = D lam':
//   pass 2 (about U1, v = mu):    lam1 = mu/2 + (dt/2) r
//   pass 1 (about Un, v = lam1):  lamn = mu/2 + lam1 + dt r
//
// Per axis, with face c the lower face of cell c: the flux cotangent is
// g_f = (v_f - v_{f-1})/dx, and the face VJP returns the cotangents VLb_f,
// VRb_f of the reconstructed states VL_f = W_{f-1} + s_{f-1}/2 and
// VR_f = W_f - s_f/2.  With the slope cotangent sb_c = (VLb_{c+1} - VRb_c)/2,
// (dp_c, dq_c) the derivatives of the limited slope of c with respect to its
// backward and forward differences, A_c = sb_c dp_c, B_c = sb_c dq_c and
// E_c = VLb_{c+1} + VRb_c + A_c - B_c, the primitive cotangent of cell c is
//   Wb_c = E_c - A_{c+1} + B_{c-1}.
// Positions past the grid follow the boundary rule: periodic wrap; outflow
// takes the clamped boundary state and a zero v, so faces beyond the
// boundary faces carry no cotangent, and the ghost cells fold into the
// boundary cells through four substitutions:
//   B_{-1} <- VLb_0,  E_0 <- E_0 - A_0,  A_n <- -VRb_n,  E_{n-1} <- E_{n-1} + B_{n-1}.
//
// Work decomposition (as the forward stage): a workgroup owns 64 x TY
// columns and marches along z.  The primitive plane with a 3-cell x/y halo
// sits in LDS; x- and y-faces (TX + 3 per row, TY + 3 rows per column) are
// items whose (VLb, VRb) go to LDS; each cell item (own cells plus one halo
// cell per side) reads its two face slots and overwrites them with (A, B),
// which the neighbours read after a barrier.  z-faces come from a register
// window of four planes, the z-direction A, B, E and the partial sum
// X_k = E_k + B_{k-1} slide along with it (three warm-up faces per chunk).
// Local VJP arithmetic is in T; the three axis sums, the primitive ->
// conserved transpose and the lambda combination are FP64.
// ---------------------------------------------------------------------------

template <typename T> struct AdjStageArgs {
    const T *U;          // state of the linearisation: U1 (pass 2) or Un (pass 1)
    const double *lamp;  // lam' = dJ/dU_next
    const double *lam1;  // pass 1: lam1 (the cotangent v); unused in pass 2
    double *out;         // pass 2: lam1; pass 1: lamn
    int *flag;           // non-physical flag
    int nx, ny, nz;
    long long nxy, ncell;
    int per[3];
    int kz, tiles_x, tiles_y, chunks, nblocks;
    double dt, damp;
    double idx[3];       // 1/dx per axis
    double gm1;
    Phys<T> ph;
};

// cell item of one component: returns E_c (with the outflow substitutions
// for the boundary cells), sets A_c and B_c (substituted for the ghosts)
struct CellFlags {
    bool outflow;  // the axis is outflow (uniform over the grid)
    bool ghost_lo, first, ghost_hi, last;
};
__device__ __forceinline__ CellFlags cell_flags(int c, int n, int per)
{
    CellFlags f;
    f.outflow = !per;
    f.ghost_lo = c == -1;
    f.first = c == 0;
    f.ghost_hi = c == n;
    f.last = c == n - 1;
    return f;
}

template <typename T>
__device__ __forceinline__ T cell_item_d(T vl, T vr, T dp, T dq, CellFlags fl, T &A, T &B)
{
    const T sb = T(0.5) * (vl - vr);
    A = sb * dp;
    B = sb * dq;
    T E = vl + vr + A - B;
    if (fl.outflow) {
        E = fl.first ? E - A : E;
        E = fl.last ? E + B : E;
        B = fl.ghost_lo ? vl : B;
        A = fl.ghost_hi ? -vr : A;
    }
    return E;
}

template <int LIM, typename T>
__device__ __forceinline__ T cell_item(T vl, T vr, T wm, T w0, T wp, CellFlags fl, T &A, T &B)
{
    T dp, dq;
    slope_d<LIM>(w0 - wm, wp - w0, dp, dq);
    return cell_item_d(vl, vr, dp, dq, fl, A, B);
}


// extended index -> cell index along an axis for the cotangent v (-1: zero
// outside an outflow axis); the periodic wrap is remap_index's
__device__ __forceinline__ int v_index(int m, int n, int per)
{
    if (per) return remap_index(m, n, 1);
    return (m < 0 || m >= n) ? -1 : m;
}

template <typename T, int SOLVER, int LIM, int NDIM, int PASS, int TY>
__global__ void __launch_bounds__(TX *TY) adj_stage_kernel(const AdjStageArgs<T> a)
{
    constexpr int NT = TX * TY;
    constexpr int H = 3;                         // LDS halo width
    constexpr int HY = NDIM >= 2 ? H : 0;
    constexpr int PX = TX + 2 * H;
    constexpr int PY = TY + 2 * HY;
    constexpr int PLANE = PX * PY;
    constexpr int FXW = TX + 3;                  // x faces i0-1 .. i0+TX+1 per row
    constexpr int NFX = TY * FXW;
    constexpr int FYR = NDIM >= 2 ? TY + 3 : 0;  // y face rows j0-1 .. j0+TY+1
    constexpr int NFY = FYR * TX;
    constexpr int NCHX = (NFX + TX - 1) / TX;
    constexpr int NCHUNK = NCHX + FYR;
    constexpr int NHX = 2 * H * TY;
    constexpr int NH = NHX + (NDIM >= 2 ? 2 * H * TX : 0);
    constexpr int HPT = (NH + NT - 1) / NT;
    constexpr int NCX = 2 * TY;                  // x halo cell items
    constexpr int NCXC = (NCX + TX - 1) / TX;
    constexpr int NCCH = NCXC + (NDIM >= 2 ? 2 : 0);

    __shared__ T P[NQ * PLANE];
    __shared__ T FX[2 * NQ * NFX];                     // [side][q][row][face]
    __shared__ T FY[NDIM >= 2 ? 2 * NQ * NFY : 1];     // [side][q][face row][column]

    const int t = threadIdx.x;
    const int tx = t & (TX - 1);
    const int ty = t / TX;
    const int wave = __builtin_amdgcn_readfirstlane(ty);
    const int lb = logical_block(blockIdx.x, a.nblocks);
    const int tile_x = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int tile_y = rest % a.tiles_y;
    const int chunk = rest / a.tiles_y;
    const int i0 = tile_x * TX, j0 = tile_y * TY;
    const int k0 = chunk * a.kz;
    const int k1 = min(k0 + a.kz, a.nz);
    const int i = i0 + tx, j = j0 + ty;
    const bool active = (i < a.nx) & (j < a.ny);

    const int ri = remap_index(i, a.nx, a.per[0]);
    const int rj = remap_index(j, a.ny, a.per[1]);
    const long long own = (long long)rj * a.nx + ri;
    int h_slot[HPT];
    long long h_off[HPT];
#pragma unroll
    for (int m = 0; m < HPT; ++m) {
        const int h = t + m * NT;
        h_slot[m] = 0;
        h_off[m] = 0;
        if (h < NH) {
            int lx, ly;
            if (h < NHX) {
                const int r = h / (2 * H), s = h % (2 * H);
                lx = s < H ? s : TX + s;
                ly = r + HY;
            } else {
                const int hy = h - NHX;
                const int r6 = hy / TX, c = hy % TX;
                lx = c + H;
                ly = r6 < H ? r6 : TY + r6;
            }
            h_slot[m] = ly * PX + lx;
            const int gi = remap_index(i0 + lx - H, a.nx, a.per[0]);
            const int gj = remap_index(j0 + ly - HY, a.ny, a.per[1]);
            h_off[m] = (long long)gj * a.nx + gi;
        }
    }
    const int own_slot = (ty + HY) * PX + tx + H;
    bool ok = true;

    auto zoff = [&](int k) -> long long {
        return (long long)remap_index(k, a.nz, a.per[2]) * a.nxy;
    };
    auto prim_at = [&](long long c, T *v) {
        T u[NQ];
        load_cell(a.U, a.ncell, c, u);
        ok &= cons_to_prim(u, a.ph, v);
    };
    // flux cotangent of a face between cells ca and cb (-1: outside, zero)
    auto face_g = [&](long long ca, long long cb, double idx, T *gb) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double va = 0.0, vb = 0.0;
            if (PASS == 2) {
                const double sc = q == PSI ? a.damp : 1.0;
                if (ca >= 0) va = a.lamp[q * a.ncell + ca] * sc;
                if (cb >= 0) vb = a.lamp[q * a.ncell + cb] * sc;
            } else {
                if (ca >= 0) va = a.lam1[q * a.ncell + ca];
                if (cb >= 0) vb = a.lam1[q * a.ncell + cb];
            }
            gb[q] = (T)((vb - va) * idx);
        }
    };
    // face VJP from an LDS stencil w0..w3 (stride apart)
    auto lds_face = [&](auto dir, const T *base, int stride, const T *gb, T *VLb, T *VRb) {
        constexpr int D = decltype(dir)::value;
        T VL[NQ], VR[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T *pq = base + q * PLANE;
            const T w0 = pq[0], w1 = pq[stride], w2 = pq[2 * stride], w3 = pq[3 * stride];
            VL[q] = w1 + T(0.5) * limited_slope<LIM>(w1 - w0, w2 - w1);
            VR[q] = w2 - T(0.5) * limited_slope<LIM>(w2 - w1, w3 - w2);
        }
        face_flux_vjp<T, SOLVER, D>(VL, VR, a.ph, gb, VLb, VRb);
    };
    // cell item on the LDS stencil: faces in slots vl (VLb_{c+1}) and vr
    // (VRb_c), overwritten with A_c and B_c; returns nothing but adds E_c
    auto lds_cell = [&](const T *wc, int wstride, T *vl, T *vr, int fstride, CellFlags fl, T *E) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T *w = wc + q * PLANE;
            T A, B;
            const T e = cell_item<LIM>(vl[q * fstride], vr[q * fstride], w[-wstride], w[0], w[wstride],
                                       fl, A, B);
            vl[q * fstride] = A;
            vr[q * fstride] = B;
            if (E) E[q] += e;
        }
    };

    // z partial sums carried along the march: X_kk, B_kk, VRb_{kk+1}
    T Xz[NQ], Bz[NQ], VRz[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) Xz[q] = Bz[q] = VRz[q] = T(0);
    const int kstart = NDIM == 3 ? k0 - 3 : k0;

    for (int kk = kstart; kk < k1; ++kk) {
        const bool out = kk >= k0;
        const long long zk = zoff(kk);
        if (out) {
            // (a) primitives of plane kk into LDS
            {
                T w[NQ];
                prim_at(zk + own, w);
#pragma unroll
                for (int q = 0; q < NQ; ++q) P[q * PLANE + own_slot] = w[q];
            }
#pragma unroll
            for (int m = 0; m < HPT; ++m) {
                if (t + m * NT < NH) {
                    T hv[NQ];
                    prim_at(zk + h_off[m], hv);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) P[q * PLANE + h_slot[m]] = hv[q];
                }
            }
            __syncthreads();
            // (c) x- and y-face items, 64-wide single-direction chunks
            for (int ch = wave; ch < NCHUNK; ch += TY) {
                T gb[NQ], VLb[NQ], VRb[NQ];
                if (ch < NCHX) {
                    const int it = ch * TX + tx;
                    const bool valid = it < NFX;
                    const int r = valid ? it / FXW : 0;
                    const int fi = valid ? it - r * FXW : 0;
                    const int X = i0 - 1 + fi;
                    const long long row = zk + (long long)remap_index(j0 + r, a.ny, a.per[1]) * a.nx;
                    const int xa = v_index(X - 1, a.nx, a.per[0]), xb = v_index(X, a.nx, a.per[0]);
                    face_g(xa < 0 ? -1 : row + xa, xb < 0 ? -1 : row + xb, a.idx[0], gb);
                    lds_face(std::integral_constant<int, 0>{}, &P[(r + HY) * PX + fi], 1, gb, VLb, VRb);
                    if (valid) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            FX[q * NFX + it] = VLb[q];
                            FX[(NQ + q) * NFX + it] = VRb[q];
                        }
                    }
                } else if (NDIM >= 2) {
                    const int it = (ch - NCHX) * TX + tx;
                    const int gi = it / TX, c = it - gi * TX;
                    const int Y = j0 - 1 + gi;
                    const long long col = zk + remap_index(i0 + c, a.nx, a.per[0]);
                    const int ya = v_index(Y - 1, a.ny, a.per[1]), yb = v_index(Y, a.ny, a.per[1]);
                    face_g(ya < 0 ? -1 : col + (long long)ya * a.nx,
                           yb < 0 ? -1 : col + (long long)yb * a.nx, a.idx[1], gb);
                    lds_face(std::integral_constant<int, 1>{}, &P[gi * PX + c + H], PX, gb, VLb, VRb);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        FY[q * NFY + it] = VLb[q];
                        FY[(NQ + q) * NFY + it] = VRb[q];
                    }
                }
            }
            __syncthreads();
        }
        // (b) z-face kk+2 and the z cell item of kk+1 (planes kk .. kk+3
        // re-read, they are cache resident); R starts as Wb_z of plane kk
        T R[NQ];
        if (NDIM == 3) {
            T gb[NQ], VL[NQ], VR[NQ], VLb[NQ], VRb[NQ];
            {
                T w0[NQ], w1[NQ], w2[NQ], w3[NQ];
                prim_at(zk + own, w0);
                prim_at(zoff(kk + 1) + own, w1);
                prim_at(zoff(kk + 2) + own, w2);
                prim_at(zoff(kk + 3) + own, w3);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    VL[q] = w1[q] + T(0.5) * limited_slope<LIM>(w1[q] - w0[q], w2[q] - w1[q]);
                    VR[q] = w2[q] - T(0.5) * limited_slope<LIM>(w2[q] - w1[q], w3[q] - w2[q]);
                }
            }
            const int za = v_index(kk + 1, a.nz, a.per[2]), zb = v_index(kk + 2, a.nz, a.per[2]);
            face_g(za < 0 ? -1 : za * a.nxy + own, zb < 0 ? -1 : zb * a.nxy + own, a.idx[2], gb);
            face_flux_vjp<T, SOLVER, 2>(VL, VR, a.ph, gb, VLb, VRb);
            const CellFlags fl = cell_flags(kk + 1, a.nz, a.per[2]);
            T w0[NQ], w1[NQ], w2[NQ];
            prim_at(zk + own, w0);
            prim_at(zoff(kk + 1) + own, w1);
            prim_at(zoff(kk + 2) + own, w2);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T A, B;
                const T E = cell_item<LIM>(VLb[q], VRz[q], w0[q], w1[q], w2[q], fl, A, B);
                R[q] = Xz[q] - A;
                Xz[q] = E + Bz[q];
                Bz[q] = B;
                VRz[q] = VRb[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) R[q] = T(0);
        }
        if (!out) continue;
        // (d) cell items: own cells (x and y), then the halo cells
        {
            const int fo = ty * FXW + tx + 1;  // slot of face i (own cell's lower x face)
            lds_cell(&P[own_slot], 1, &FX[fo + 1], &FX[NQ * NFX + fo], NFX, cell_flags(i, a.nx, a.per[0]),
                     R);
            if (NDIM >= 2) {
                const int go = (ty + 1) * TX + tx;  // slot of face j (own cell's lower y face)
                lds_cell(&P[own_slot], PX, &FY[go + TX], &FY[NQ * NFY + go], NFY,
                         cell_flags(j, a.ny, a.per[1]), R);
            }
        }
        // the lambda values of the own cell that the combine needs are loaded
        // here, so that their latency overlaps the halo items and the barrier
        double mu[NQ], l1[NQ];
        if (active) {
            const long long c = zk + own;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                // pass 1 reads lam' only here (streaming); pass 2 read it for the faces
                const double lp = PASS == 1 ? __builtin_nontemporal_load(&a.lamp[q * a.ncell + c])
                                            : a.lamp[q * a.ncell + c];
                mu[q] = lp * (q == PSI ? a.damp : 1.0);
                l1[q] = PASS == 1 ? a.lam1[q * a.ncell + c] : 0.0;
            }
        }
        for (int hc = TY - 1 - wave; hc < NCCH; hc += TY) {
            if (hc < NCXC) {
                const int it = hc * TX + tx;
                if (it < NCX) {
                    const int r = it >> 1, side = it & 1;
                    const int fi = side ? TX + 1 : 0;      // face slot of the cell's lower face
                    const int X = i0 - 1 + fi;
                    const int fo = r * FXW + fi;
                    lds_cell(&P[(r + HY) * PX + fi + H - 1], 1, &FX[fo + 1], &FX[NQ * NFX + fo], NFX,
                             cell_flags(X, a.nx, a.per[0]), nullptr);
                }
            } else if (NDIM >= 2) {
                const int side = hc - NCXC;
                const int gi = side ? TY + 1 : 0;          // face row of the cell's lower face
                const int Y = j0 - 1 + gi;
                const int go = gi * TX + tx;
                lds_cell(&P[(gi + HY - 1) * PX + tx + H], PX, &FY[go + TX], &FY[NQ * NFY + go], NFY,
                         cell_flags(Y, a.ny, a.per[1]), nullptr);
            }
        }
        __syncthreads();
        // (f) neighbours' A and B, the primitive -> conserved transpose at
        // the cell's primitives (in LDS) and the lambda combination, in FP64
        if (active) {
            double wb[NQ];
            {
                const int fo = ty * FXW + tx + 1;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    double r = (double)R[q] + (double)(FX[(NQ + q) * NFX + fo - 1] - FX[q * NFX + fo + 2]);
                    if (NDIM >= 2) {
                        const int go = (ty + 1) * TX + tx;
                        r += (double)(FY[(NQ + q) * NFY + go - TX] - FY[q * NFY + go + 2 * TX]);
                    }
                    wb[q] = r;
                }
            }
            const T *w = &P[own_slot];
            const double ir = 1.0 / (double)w[RHO * PLANE];
            const double v[3] = {(double)w[VX * PLANE], (double)w[VY * PLANE], (double)w[VZ * PLANE]};
            const double vsq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            double r[NQ];
            r[RHO] = wb[RHO] - (v[0] * wb[VX] + v[1] * wb[VY] + v[2] * wb[VZ]) * ir +
                     a.gm1 * 0.5 * vsq * wb[PRS];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r[MX + k] = wb[VX + k] * ir - a.gm1 * v[k] * wb[PRS];
                r[BX + k] = wb[BX + k] - a.gm1 * (double)w[(BX + k) * PLANE] * wb[PRS];
            }
            r[ENG] = a.gm1 * wb[PRS];
            r[PSI] = wb[PSI];
            const long long c = zk + own;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double o;
                if (PASS == 2)
                    o = 0.5 * mu[q] + 0.5 * a.dt * r[q];
                else
                    o = 0.5 * mu[q] + l1[q] + a.dt * r[q];
                __builtin_nontemporal_store(o, &a.out[q * a.ncell + c]);  // written once
            }
        }
    }
    if (!ok) atomicOr(a.flag, 1);
}

} // namespace mhd
