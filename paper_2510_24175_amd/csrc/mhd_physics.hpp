// Device-side pointwise physics of the ideal-MHD finite-volume step.
//
// Conventions (shared with include/mhd.h):
//   primitive  V = (rho, vx, vy, vz, p, Bx, By, Bz, psi)
//   conserved  U = (rho, mx, my, mz, E, Bx, By, Bz, psi)
//   E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2   (magnetic pressure |B|^2/2)
// A face normal to axis d is solved in the cyclic frame (n, t1, t2) =
// (d, d+1, d+2) mod 3.  Everything is templated on the arithmetic type T
// (float or double); reciprocals and square roots go through Num<T>, which
// uses the hardware approximations in FP32, and in FP64 IEEE square roots and
// Newton-refined reciprocals.
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

enum { NQ = 9 };
enum { RHO = 0, VX = 1, VY = 2, VZ = 3, PRS = 4, BX = 5, BY = 6, BZ = 7, PSI = 8 };
enum { MX = 1, MY = 2, MZ = 3, ENG = 4 };
enum { SOLVER_HLL = 0, SOLVER_HLLD = 1 };
// reconstructions: PLM with the minmod or MC limiter, or fifth-order WENO-Z
enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_WENOZ = 2 };

template <typename T> struct Num;

// Type-exact elementary operations (the unsuffixed builtins are the double
// versions and would promote float operands).
template <> struct Num<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float abs(float x) { return __builtin_fabsf(x); }
    static __device__ __forceinline__ float min(float a, float b) { return __builtin_fminf(a, b); }
    static __device__ __forceinline__ float max(float a, float b) { return __builtin_fmaxf(a, b); }
    static __device__ __forceinline__ float copysign(float a, float b) { return __builtin_copysignf(a, b); }
    // minmod(a, b) as the median of a, b and 0 (one instruction)
    static __device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
    static constexpr float eps = 1.1920928955078125e-7f;
    static constexpr float weno_eps = 1e-30f;  // normal, with a finite reciprocal
    static constexpr float big = 3.0e38f;
};

template <> struct Num<double> {
    // reciprocal: the hardware estimate (relative error up to 2^-24.4)
    // refined by two Newton-Raphson steps (e = 1 - x r, r <- r + r e); equal
    // to the IEEE quotient on every one of 2M log-uniform samples in
    // [1e-300, 1e300] (one step leaves up to 11 ulps)
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        double e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-x, r, 1.0);
        return __builtin_fma(r, e, r);
    }
    // square root: Goldschmidt's coupled iteration from the hardware
    // reciprocal-square-root estimate y ~ 1/sqrt(x) (g = x y -> sqrt(x),
    // h = y/2 -> 1/(2 sqrt(x)), r = 1/2 - g h), then two residual corrections
    // g <- g + (x - g^2) h.  Bitwise the IEEE square root on every one of 4M
    // log-uniform samples in [1e-300, 1e300]; below that the residuals lose
    // bits in subnormal products (the kernels' roots are of sums with normal
    // terms).  x + DBL_MIN keeps the estimate finite at x = 0 (result 0);
    // negative x gives NaN.  Ten instructions against about seventeen for
    // the library's scaled sequence.
    static __device__ __forceinline__ double sqrt(double x)
    {
        const double y = __builtin_amdgcn_rsq(x + 2.2250738585072014e-308);
        double g = x * y, h = 0.5 * y;
        const double r = __builtin_fma(-g, h, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
        double d = __builtin_fma(-g, g, x);
        g = __builtin_fma(d, h, g);
        d = __builtin_fma(-g, g, x);
        return __builtin_fma(d, h, g);
    }
    // reciprocal square root: two steps of the same coupled iteration,
    // 1/sqrt(x) = 2h, within 2 ulps for normal x > 0 (NaN at 0, as the
    // refined reciprocal of a zero root)
    static __device__ __forceinline__ double rsqrt(double x)
    {
        const double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        double r = __builtin_fma(-g, h, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
        r = __builtin_fma(-g, h, 0.5);
        h = __builtin_fma(h, r, h);
        return 2.0 * h;
    }
    static __device__ __forceinline__ double abs(double x) { return __builtin_fabs(x); }
    static __device__ __forceinline__ double min(double a, double b) { return __builtin_fmin(a, b); }
    static __device__ __forceinline__ double max(double a, double b) { return __builtin_fmax(a, b); }
    static __device__ __forceinline__ double copysign(double a, double b) { return __builtin_copysign(a, b); }
    // minmod(a, b) as the median of a, b and 0 (no FP64 median instruction:
    // four min/max)
    static __device__ __forceinline__ double minmod(double a, double b)
    {
        return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
    }
    static constexpr double eps = 2.220446049250313e-16;
    static constexpr double weno_eps = 1e-40;
    static constexpr double big = 1.0e300;
};

// Per-launch constants of the scheme.
template <typename T> struct Phys {
    T gamma;     // adiabatic index
    T gm1;       // gamma - 1
    T inv_gm1;   // 1 / (gamma - 1)
    T ch;        // GLM wave speed c_h
    T ch2;       // c_h^2
    T half_ich;  // 1 / (2 c_h), 0 when GLM is off
    int glm;     // GLM cleaning on
};

// Conserved -> primitive.  Returns false for rho <= 0, p <= 0 or a
// non-finite value (NaN fails every comparison; infinities fail the upper
// bounds or turn p into NaN or -inf).
template <typename T>
__device__ __forceinline__ bool cons_to_prim(const T *u, const Phys<T> &ph, T *v)
{
    const T rho = u[RHO];
    const T ir = Num<T>::rcp(rho);
    const T vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
    const T kin = T(0.5) * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
    const T mag = T(0.5) * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
    const T p = ph.gm1 * (u[ENG] - kin - mag);
    v[RHO] = rho;
    v[VX] = vx;
    v[VY] = vy;
    v[VZ] = vz;
    v[PRS] = p;
    v[BX] = u[BX];
    v[BY] = u[BY];
    v[BZ] = u[BZ];
    v[PSI] = u[PSI];
    const T big = Num<T>::big;
    return (rho > T(0)) & (rho < big) & (p > T(0)) & (p < big) & (Num<T>::abs(u[PSI]) < big);
}

// Limited slope from the backward difference a and the forward difference b:
// minmod(a, b) (zero unless a and b have the same sign, else the one of
// smaller magnitude), or MC = minmod(2a, 2b, (a+b)/2) =
// minmod(2a, minmod(2b, (a+b)/2)).  The limiter is a compile-time parameter
// of the kernels.
template <int LIM, typename T> __device__ __forceinline__ T limited_slope(T a, T b)
{
    if (LIM == LIM_MC) return Num<T>::minmod(T(2) * a, Num<T>::minmod(T(2) * b, T(0.5) * (a + b)));
    return Num<T>::minmod(a, b);
}

// WENO-Z face values of one cell (Borges, Carmona, Costa & Don 2008; p = 1,
// eps = 1e-40 in FP64, 1e-30 in FP32 where 1e-40 is subnormal and its
// reciprocal overflows) from the five cell values v0..v4 centred on it: the
// value at its right face (rgt, x_{i+1/2}) and at its left face (lft,
// x_{i-1/2}).  The three candidate quadratics are fitted to the cell sets
// S0 = {v0,v1,v2}, S1 = {v1,v2,v3}, S2 = {v2,v3,v4}; written around v2 with
// e_k their second differences and G_k half their one-sided first
// differences (G0 = (v0 - 4v1 + 3v2)/2, G1 = (v1 - v3)/2,
// G2 = (3v2 - 4v3 + v4)/2), a candidate's face values are
// v2 + e_k/12 -+ G_k/2 and its Jiang-Shu smoothness indicator is
// beta_k = 13/12 e_k^2 + G_k^2.  Both faces share beta_k and the global
// indicator tau5 = |beta0 - beta2|; their linear weights are mirror images,
// (1, 6, 3)/10 on (S0, S1, S2) for the right face and (3, 6, 1)/10 for the
// left, each scaled by 1 + tau5 / (beta_k + eps).
//
// FP64: the weights are multiplied through by (beta0+eps)(beta1+eps)(beta2+eps),
// W_k = prod_{j != k}(beta_j + eps) (beta_k + eps + tau5) (formed as the triple product
// plus tau5 times the pair product), the linear weights
// are folded into the candidate deviations and the weight sums, and both faces
// are normalised with one reciprocal of the product of the two weight sums,
// the Newton-refined one (within an ulp).  That product lies between eps^6 and
// about 4 beta_max^6, so it and its reciprocal stay normal for indicators
// between eps and 1e51 (differences of a few 1e25 between neighbouring cell
// values).  FP32: the reciprocals are the hardware
// approximation and the ratio tau5/(beta_k + eps) is capped at 1e18 so that
// the weights stay finite for jumps whose indicators exceed FLT_MAX * eps; the
// cap only binds where two candidates are both 1e18 times smoother than
// tau5, and then their face values agree far below FP32 resolution.
template <typename T>
__device__ __forceinline__ void wenoz_pair(T v0, T v1, T v2, T v3, T v4, T &rgt, T &lft)
{
    T e0, e1, e2, G0, G1, G2;
    if constexpr (sizeof(T) == 8) {
        // from the two inner differences (11 operations instead of 14)
        const T da = v2 - v1, db = v2 - v3;
        e1 = -(da + db);
        G1 = T(0.5) * (db - da);
        e0 = (v0 - v1) + da;
        e2 = (v4 - v3) + db;
        G0 = T(0.5) * e0 + da;
        G2 = T(0.5) * e2 + db;
    } else {
        e0 = (v0 + v2) - T(2) * v1, e1 = (v1 + v3) - T(2) * v2, e2 = (v2 + v4) - T(2) * v3;
        G0 = T(0.5) * v0 - T(2) * v1 + T(1.5) * v2;
        G1 = T(0.5) * (v1 - v3);
        G2 = T(1.5) * v2 - T(2) * v3 + T(0.5) * v4;
    }
    const T c = T(13.0 / 12.0);
    const T eps = Num<T>::weno_eps;
    // FP64 adds eps to G_k^2 first (one fused operation fewer per indicator);
    // FP32 keeps eps last: the reordered sum moves FP32 results on the
    // thinnest constrained-transport grids to the edge of their error bound
    const T B0 = sizeof(T) == 8 ? c * e0 * e0 + (G0 * G0 + eps) : (c * e0 * e0 + G0 * G0) + eps;
    const T B1 = sizeof(T) == 8 ? c * e1 * e1 + (G1 * G1 + eps) : (c * e1 * e1 + G1 * G1) + eps;
    const T B2 = sizeof(T) == 8 ? c * e2 * e2 + (G2 * G2 + eps) : (c * e2 * e2 + G2 * G2) + eps;
    const T tau = Num<T>::abs(B0 - B2);
    T nr, sr, nl, sl;
    if constexpr (sizeof(T) == 8) {
        // W_k = B0 B1 B2 + tau5 prod_{j != k} B_j
        const T p12 = B1 * B2, p02 = B0 * B2, p01 = B0 * B1, P = B0 * p12;
        const T w0 = tau * p12 + P, w1 = tau * p02 + P, w2 = tau * p01 + P;
        // candidate deviations from v2 at the two faces, each scaled by its
        // linear weight ((1, 6, 3)/10 right, (3, 6, 1)/10 left)
        const T g0 = T(0.05) * G0, g1 = T(0.3) * G1, g2 = T(0.05) * G2;
        const T d0r = e0 * T(0.1 / 12.0) + g0, d0l = e0 * T(0.3 / 12.0) - T(3) * g0;
        const T d1r = e1 * T(0.05) - g1, d1l = e1 * T(0.05) + g1;
        const T d2r = e2 * T(0.3 / 12.0) - T(3) * g2, d2l = e2 * T(0.1 / 12.0) + g2;
        const T s1 = T(0.6) * w1;
        nr = w0 * d0r + w1 * d1r + w2 * d2r;
        nl = w0 * d0l + w1 * d1l + w2 * d2l;
        sr = T(0.1) * w0 + (T(0.3) * w2 + s1);
        sl = T(0.3) * w0 + (T(0.1) * w2 + s1);
    } else {
        const T h0 = e0 * T(1.0 / 12.0), h1 = e1 * T(1.0 / 12.0), h2 = e2 * T(1.0 / 12.0);
        const T d0r = h0 + T(0.5) * G0, d0l = h0 - T(0.5) * G0;
        const T d1r = h1 - T(0.5) * G1, d1l = h1 + T(0.5) * G1;
        const T d2r = h2 - T(0.5) * G2, d2l = h2 + T(0.5) * G2;
        const T m0 = Num<T>::min(tau * Num<T>::rcp(B0), T(1e18));
        const T m1 = Num<T>::min(tau * Num<T>::rcp(B1), T(1e18));
        const T m2 = Num<T>::min(tau * Num<T>::rcp(B2), T(1e18));
        const T a1 = T(0.6) + T(0.6) * m1;
        const T a0r = T(0.1) + T(0.1) * m0, a2r = T(0.3) + T(0.3) * m2;
        const T a0l = T(0.3) + T(0.3) * m0, a2l = T(0.1) + T(0.1) * m2;
        nr = a0r * d0r + a1 * d1r + a2r * d2r, sr = a0r + a1 + a2r;
        nl = a0l * d0l + a1 * d1l + a2l * d2l, sl = a0l + a1 + a2l;
    }
    if constexpr (sizeof(T) == 8) {
        const T inv = Num<T>::rcp(sr * sl);
        rgt = v2 + nr * (sl * inv);
        lft = v2 + nl * (sr * inv);
    } else {
        rgt = v2 + nr * Num<T>::rcp(sr);
        lft = v2 + nl * Num<T>::rcp(sl);
    }
}

// Fast magnetosonic speed from p, |B|^2, B_n^2 and 1/rho:
// c_f^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 (b^2 - b_n^2))) / 2.
template <typename T>
__device__ __forceinline__ T fast_speed(T p, T bsq, T bnsq, T gamma, T irho)
{
    const T a2 = gamma * p * irho;
    const T b2 = bsq * irho;
    const T bn2 = bnsq * irho;
    const T dab = a2 - b2;
    T disc = dab * dab + T(4) * a2 * (b2 - bn2);
    disc = Num<T>::max(disc, T(0));
    return Num<T>::sqrt(T(0.5) * (a2 + b2 + Num<T>::sqrt(disc)));
}

// A rotated 8-component state: rho, u (normal), v1, v2, p, bn, b1, b2, with
// its derived energy, total pressure and v.B.
template <typename T> struct RState {
    T rho, u, v1, v2, p, bn, b1, b2;
    T irho, bsq, E, pt, vb;
};

// irho, |B|^2 and total pressure of a rotated state
template <typename T>
__device__ __forceinline__ void rstate_prepare(RState<T> &s)
{
    s.irho = Num<T>::rcp(s.rho);
    s.bsq = s.bn * s.bn + s.b1 * s.b1 + s.b2 * s.b2;
    s.pt = s.p + T(0.5) * s.bsq;
}

// total energy and v.B of a prepared rotated state
template <typename T>
__device__ __forceinline__ void rstate_energy(RState<T> &s, const Phys<T> &ph)
{
    s.E = s.p * ph.inv_gm1 + T(0.5) * s.rho * (s.u * s.u + s.v1 * s.v1 + s.v2 * s.v2) +
          T(0.5) * s.bsq;
    s.vb = s.u * s.bn + s.v1 * s.b1 + s.v2 * s.b2;
}

// physical normal flux (8 comps, slot 5 unused) and conserved vector
template <typename T>
__device__ __forceinline__ void rstate_flux(const RState<T> &s, T *f, T *c)
{
    const T mu = s.rho * s.u;
    f[0] = mu;
    f[1] = mu * s.u + s.pt - s.bn * s.bn;
    f[2] = mu * s.v1 - s.bn * s.b1;
    f[3] = mu * s.v2 - s.bn * s.b2;
    f[4] = (s.E + s.pt) * s.u - s.bn * s.vb;
    f[5] = T(0);
    f[6] = s.u * s.b1 - s.v1 * s.bn;
    f[7] = s.u * s.b2 - s.v2 * s.bn;
    c[0] = s.rho;
    c[1] = mu;
    c[2] = s.rho * s.v1;
    c[3] = s.rho * s.v2;
    c[4] = s.E;
    c[5] = s.bn;
    c[6] = s.b1;
    c[7] = s.b2;
}

template <typename T>
__device__ __forceinline__ T rstate_fast(const RState<T> &s, const Phys<T> &ph)
{
    return fast_speed(s.p, s.bsq, s.bn * s.bn, ph.gamma, s.irho);
}

// HLL flux, Davis bounds clamped to the origin so one formula covers the
// supersonic cases: F = (sR FL - sL FR + sL sR (UR - UL)) / (sR - sL).
// L and R need irho, bsq and pt (rstate_prepare).
template <typename T>
__device__ __forceinline__ void hll_flux(const RState<T> &L, const RState<T> &R,
                                         const Phys<T> &ph, T *F)
{
    RState<T> Le = L, Re = R;
    rstate_energy(Le, ph);
    rstate_energy(Re, ph);
    T FL[8], UL[8], FR[8], UR[8];
    rstate_flux(Le, FL, UL);
    rstate_flux(Re, FR, UR);
    const T cL = rstate_fast(L, ph), cR = rstate_fast(R, ph);
    const T sL = Num<T>::min(Num<T>::min(L.u - cL, R.u - cR), T(0));
    const T sR = Num<T>::max(Num<T>::max(L.u + cL, R.u + cR), T(0));
    const T id = Num<T>::rcp(sR - sL);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        // slot 5 (B_n) is unused: the interface solve supplies that flux
        if (k == 5) F[k] = T(0);
        else F[k] = (sR * FL[k] - sL * FR[k] + sL * sR * (UR[k] - UL[k])) * id;
    }
}

// One side of the HLLD single-star state (Miyoshi & Kusano 2005): density,
// tangential velocity and field.  Its energy is formed only for the side the
// flux is taken from (hlld_star_energy).
template <typename T> struct Star {
    T rho, v1, v2, b1, b2;
    T su, isd; // S - u and 1/(S - S_M)
    T sq, isq; // sqrt(rho*) and 1/sqrt(rho*)
};

template <typename T>
__device__ __forceinline__ void hlld_star(const RState<T> &s, T S, T sM, Star<T> &o)
{
    o.su = S - s.u;
    o.isd = Num<T>::rcp(S - sM);
    const T m = s.rho * o.su;
    o.rho = m * o.isd;
    const T mm = m * (S - sM);
    const T bn2 = s.bn * s.bn;
    const T D = mm - bn2;
    const bool degenerate = Num<T>::abs(D) <= T(16) * Num<T>::eps * (Num<T>::abs(mm) + bn2);
    const T iD = Num<T>::rcp(D);
    // a degenerate side keeps its tangential state: cv = 0, cb = 1
    const T cv = degenerate ? T(0) : s.bn * (sM - s.u) * iD;
    const T cb = degenerate ? T(1) : (m * o.su - bn2) * iD;
    o.v1 = s.v1 - s.b1 * cv;
    o.v2 = s.v2 - s.b2 * cv;
    o.b1 = s.b1 * cb;
    o.b2 = s.b2 * cb;
    o.isq = Num<T>::rsqrt(o.rho);
    o.sq = o.rho * o.isq;
}

// v*.B* and E* of one side: E* = ((S-u)E - p_T u + p_T* S_M + B_n (v.B - v*.B*)) / (S - S_M)
template <typename T>
__device__ __forceinline__ void hlld_star_energy(const RState<T> &s, const Star<T> &o, T sM, T pts,
                                                 T &vbs, T &Es)
{
    vbs = sM * s.bn + o.v1 * o.b1 + o.v2 * o.b2;
    Es = (o.su * s.E - s.pt * s.u + pts * sM + s.bn * (s.vb - vbs)) * o.isd;
}

// HLLD flux (Miyoshi & Kusano 2005), outer speeds min(u_L, u_R) - max(c_fL,
// c_fR) and max(u_L, u_R) + max(c_fL, c_fR).  L and R need
// irho, bsq and pt (rstate_prepare); E and v.B are formed for the side the
// flux is taken from.
template <typename T>
__device__ __forceinline__ void hlld_flux(const RState<T> &L, const RState<T> &R,
                                          const Phys<T> &ph, T *F)
{
    // outer speeds: the slower (faster) normal velocity minus (plus) the
    // larger fast speed (at least as wide as Davis's bounds; keeps the
    // rotational waves inside the fan where Davis's bounds let D cross zero)
    const T cL = rstate_fast(L, ph), cR = rstate_fast(R, ph);
    const T cm = Num<T>::max(cL, cR);
    const T sL = Num<T>::min(L.u, R.u) - cm;
    const T sR = Num<T>::max(L.u, R.u) + cm;
    const T mL = (sL - L.u) * L.rho, mR = (sR - R.u) * R.rho;
    const T idm = Num<T>::rcp(mR - mL);
    const T sM = (mR * R.u - mL * L.u - R.pt + L.pt) * idm;
    const T pts = (mR * L.pt - mL * R.pt + mL * mR * (R.u - L.u)) * idm;
    const T bn = L.bn;

    Star<T> sl, sr;
    hlld_star(L, sL, sM, sl);
    hlld_star(R, sR, sM, sr);

    const T sgn = bn >= T(0) ? T(1) : T(-1);
    const T abn = Num<T>::abs(bn);
    const T ssL = sM - abn * sl.isq;
    const T ssR = sM + abn * sr.isq;
    const T iden = Num<T>::rcp(sl.sq + sr.sq);
    const T v1 = (sl.sq * sl.v1 + sr.sq * sr.v1 + (sr.b1 - sl.b1) * sgn) * iden;
    const T v2 = (sl.sq * sl.v2 + sr.sq * sr.v2 + (sr.b2 - sl.b2) * sgn) * iden;
    const T sqq = sl.sq * sr.sq;
    const T b1 = (sl.sq * sr.b1 + sr.sq * sl.b1 + sqq * (sr.v1 - sl.v1) * sgn) * iden;
    const T b2 = (sl.sq * sr.b2 + sr.sq * sl.b2 + sqq * (sr.v2 - sl.v2) * sgn) * iden;
    const T vbss = sM * bn + v1 * b1 + v2 * b2;

    // side of the contact and the region within it
    const bool left = sM >= T(0);
    RState<T> S = left ? L : R;
    rstate_energy(S, ph);
    const Star<T> st = left ? sl : sr;
    const T s_out = left ? sL : sR;
    const T s_in = left ? ssL : ssR;
    // outer region: sL >= 0 (left) or sR <= 0 (right)
    const bool outer = left ? (sL >= T(0)) : (sR <= T(0));
    // double-star region: s*L < 0 (left of contact) or s*R >= 0 (right)
    const bool dbl = left ? (ssL < T(0)) : (ssR >= T(0));
    const T a1 = outer ? T(0) : s_out;
    const T a2 = (outer || !dbl) ? T(0) : s_in;
    T vbs, Es;
    hlld_star_energy(S, st, sM, pts, vbs, Es);
    const T Ess = Es + (left ? -st.sq : st.sq) * (vbs - vbss) * sgn;

    T f[8], u[8];
    rstate_flux(S, f, u);
    const T us[8] = {st.rho, st.rho * sM, st.rho * st.v1, st.rho * st.v2, Es, bn, st.b1, st.b2};
    const T uss[8] = {st.rho, st.rho * sM, st.rho * v1, st.rho * v2, Ess, bn, b1, b2};
    // rho, the normal momentum and B_n agree in the single- and double-star
    // states; slot 5 (B_n) is unused
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k == 5) F[k] = T(0);
        else if (k <= 1) F[k] = f[k] + a1 * (us[k] - u[k]);
        else F[k] = f[k] + a1 * (us[k] - u[k]) + a2 * (uss[k] - us[k]);
    }
}

// Select a[d] for d in {0,1,2} without indexing a register array (the
// selects fold away when d is a compile-time constant).
template <typename T> __device__ __forceinline__ T pick3(int d, T a0, T a1, T a2)
{
    return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

// Interface flux from two unrotated primitive face states along axis d:
// GLM (B_n, psi) interface solve, MHD solver on the 8 MHD components with
// B_n replaced by B_n*, then F(B_n) = psi*, F(psi) = c_h^2 B_n*.  With
// constrained transport (CT) the normal field is the face's own value bnf
// and F(B_n) = F(psi) = 0.
template <typename T, int SOLVER, bool CT = false>
__device__ __forceinline__ void face_flux(const T *VL, const T *VR, int d, const Phys<T> &ph, T *F,
                                          T bnf = T(0))
{
    // frame (n, t1, t2) = (d, d+1, d+2) mod 3
    const T bnL = pick3(d, VL[BX], VL[BY], VL[BZ]);
    const T bnR = pick3(d, VR[BX], VR[BY], VR[BZ]);
    T bns, psis;
    if (CT) {
        bns = bnf;
        psis = T(0);
    } else if (ph.glm) {
        bns = T(0.5) * (bnL + bnR) - (VR[PSI] - VL[PSI]) * ph.half_ich;
        psis = T(0.5) * (VL[PSI] + VR[PSI]) - T(0.5) * ph.ch * (bnR - bnL);
    } else {
        bns = T(0.5) * (bnL + bnR);
        psis = T(0);
    }
    RState<T> L, R;
    L.rho = VL[RHO];
    L.u = pick3(d, VL[VX], VL[VY], VL[VZ]);
    L.v1 = pick3(d, VL[VY], VL[VZ], VL[VX]);
    L.v2 = pick3(d, VL[VZ], VL[VX], VL[VY]);
    L.p = VL[PRS];
    L.bn = bns;
    L.b1 = pick3(d, VL[BY], VL[BZ], VL[BX]);
    L.b2 = pick3(d, VL[BZ], VL[BX], VL[BY]);
    R.rho = VR[RHO];
    R.u = pick3(d, VR[VX], VR[VY], VR[VZ]);
    R.v1 = pick3(d, VR[VY], VR[VZ], VR[VX]);
    R.v2 = pick3(d, VR[VZ], VR[VX], VR[VY]);
    R.p = VR[PRS];
    R.bn = bns;
    R.b1 = pick3(d, VR[BY], VR[BZ], VR[BX]);
    R.b2 = pick3(d, VR[BZ], VR[BX], VR[BY]);
    rstate_prepare(L);
    rstate_prepare(R);
    T f[8];
    if (SOLVER == SOLVER_HLLD)
        hlld_flux(L, R, ph, f);
    else
        hll_flux(L, R, ph, f);
    const T fbn = (!CT && ph.glm) ? psis : T(0);
    F[RHO] = f[0];
    F[ENG] = f[4];
    // unrotate: component x is (n, t2, t1) for d = (0, 1, 2), etc.
    F[MX] = pick3(d, f[1], f[3], f[2]);
    F[MY] = pick3(d, f[2], f[1], f[3]);
    F[MZ] = pick3(d, f[3], f[2], f[1]);
    F[BX] = pick3(d, fbn, f[7], f[6]);
    F[BY] = pick3(d, f[6], fbn, f[7]);
    F[BZ] = pick3(d, f[7], f[6], fbn);
    F[PSI] = (!CT && ph.glm) ? ph.ch2 * bns : T(0);
}

// Boundary index map of a ghost or interior coordinate m on an axis of n >= 2
// cells: periodic wrap or zero-gradient clamp.  The wrap folds at most twice
// (no integer division), so it is exact for m in [-2n, 3n), which holds every
// position a stencil of an interior cell reaches (m in [-3, n + 3)); other
// coordinates, used only as padding, are clamped into the axis.
__device__ __forceinline__ int remap_index(int m, int n, int periodic)
{
    if (periodic) {
        m = m < 0 ? m + n : m;
        m = m < 0 ? m + n : m;
        m = m >= n ? m - n : m;
        m = m >= n ? m - n : m;
    }
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

} // namespace mhd
