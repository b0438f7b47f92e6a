/*
 * FP64 CPU oracle for one Godunov finite-volume ideal-MHD step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load this
 * library: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (the paper, section "Porting of gPLUTO", lists the steps
 * of one Runge-Kutta stage: boundary exchange/calculation, conservative to
 * primitive map, interface reconstruction, Riemann fluxes, right-hand side,
 * plus a divergence-control algorithm; section "Results for gPLUTO" names
 * HLLD and, for strong scaling, GLM divergence cleaning).  The paper prints
 * no equations, so each step below follows the published method it names:
 *
 *   ghosts   : 3 layers per active face, periodic wrap or zero-gradient
 *              copy of the nearest interior cell (all 9 components).
 *   prim     : rho, v = m/rho, p = (gamma-1)(E - |m|^2/(2 rho) - |B|^2/2),
 *              B, psi.  Units with magnetic pressure |B|^2/2.  No floors:
 *              rho <= 0, p <= 0 or a non-finite value is an error.
 *   PLM      : piecewise-linear (van Leer 1979) reconstruction of the 9
 *              primitives, component-wise, minmod (or MC) limited slope.
 *   WENO-Z   : (the paper's benchmark reconstruction, section "Results for
 *              gPLUTO") fifth-order WENO-Z of Borges, Carmona, Costa & Don
 *              (2008), component-wise on the primitives: three third-order
 *              candidate values, Jiang-Shu smoothness indicators, global
 *              indicator tau5 = |beta0 - beta2|, weights
 *              alpha_k = d_k (1 + tau5 / (beta_k + eps)), d = (1, 6, 3)/10,
 *              eps = 1e-40.
 *   GLM      : Dedner et al. (2002) mixed GLM: the (B_n, psi) 2x2 system is
 *              solved exactly at each interface before the MHD solver.
 *   Riemann  : HLL (Harten, Lax & van Leer 1983) with Davis wave-speed
 *              bounds min/max of u -/+ c_f, or HLLD (Miyoshi & Kusano 2005)
 *              with outer speeds min(u_L, u_R) - max(c_fL, c_fR) and
 *              max(u_L, u_R) + max(c_fL, c_fR).
 *   RHS      : L = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d, d = x, y, z.
 *   RK2      : SSP-RK2 (Shu & Osher 1988): U1 = Un + dt L(Un);
 *              Un+1 = (Un + U1 + dt L(U1)) / 2, dt and c_h fixed per step.
 *   RK3      : (the paper's benchmark integrator) SSP-RK3 (Shu & Osher
 *              1988): U1 = Un + dt L(Un); U2 = 3/4 Un + 1/4 (U1 + dt L(U1));
 *              Un+1 = 1/3 Un + 2/3 (U2 + dt L(U2)).
 *   damping  : psi <- psi * damp once per step after the RK2 update, with
 *              damp = exp(-alpha c_h dt / dh_min) supplied by the caller.
 *   CFL      : dt = C / max_{cells,d} (|v_d| + c_f,d) / dx_d,
 *              c_h = max_{cells,d} (|v_d| + c_f,d).
 *   CT       : (the paper's weak-scaling runs) constrained transport (Evans &
 *              Hawley 1988) in 3D on periodic grids, GLM off: the field lives
 *              on the cell faces, the normal field of each Riemann problem is
 *              the face value, faces advance by the discrete curl of the edge
 *              EMFs with the same Runge-Kutta stages, and the cell field is
 *              the mean of each cell's two faces per axis.  Edge EMFs (ct = 1)
 *              the arithmetic mean of the four face fluxes around the edge
 *              (Balsara & Spicer 1999), or (ct = 2) the upwind EMF of the
 *              upwind constrained transport of Londrillo & Del Zanna (2004),
 *              which the paper cites: the two-dimensional HLL average of the
 *              EMFs of the four states meeting at the edge, plus an HLL
 *              dissipation term per transverse direction.
 *
 * External arrays are structure-of-arrays, shape [9][nz][ny][nx] ([12] with
 * constrained transport: the face field on each cell's lower x, y, z face
 * in slots 9..11), x fastest, interior cells only.  Internally the oracle uses its own padded
 * array-of-structures with explicit ghost cells.
 *
 * Status codes: 0 ok, 1 non-physical state (rho<=0, p<=0 or non-finite),
 * 2 bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#include <omp.h>

#define NV 9
/* primitive slots */
enum { RHO = 0, VX = 1, VY = 2, VZ = 3, PRS = 4, BX = 5, BY = 6, BZ = 7, PSI = 8 };
/* conserved slots: RHO, MX=1, MY=2, MZ=3, ENG=4, BX, BY, BZ, PSI */
enum { MX = 1, MY = 2, MZ = 3, ENG = 4 };

enum { ORC_HLL = 0, ORC_HLLD = 1 };
enum { ORC_MINMOD = 0, ORC_MC = 1, ORC_WENOZ = 2 };
enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1 };

typedef struct {
    int32_t ndim;
    int32_t riemann;
    int32_t limiter;
    int32_t glm;
    int64_t n[3];
    double lo[3];
    double hi[3];
    int32_t bc[3][2];
    double gamma;
    double cfl;
    double glm_alpha;
    int32_t time_order; /* 2: SSP-RK2, 3: SSP-RK3 */
    int32_t ct;         /* 1: constrained transport (face-centred B), 0: cell-centred B */
} orc_cfg;

/* State components: 9 cell-centred (RHO .. PSI); with constrained transport
 * three more, the face-centred field bx, by, bz on each cell's lower x, y and
 * z face (FBX, FBY, FBZ), and the cell-centred B is the average of the two
 * faces of the cell along each axis. */
enum { FBX = 9, FBY = 10, FBZ = 11 };
static int nstate(const orc_cfg *cfg) { return cfg->ct ? 12 : NV; }

/* ------------------------------------------------------------------ */
/* pointwise physics                                                    */
/* ------------------------------------------------------------------ */

static int finite9(const double *q)
{
    for (int k = 0; k < NV; ++k)
        if (!isfinite(q[k])) return 0;
    return 1;
}

/* conservative -> primitive for one cell; returns 0 if non-physical */
static int cons_to_prim(const double *u, double gamma, double *v)
{
    if (!finite9(u)) return 0;
    double rho = u[RHO];
    if (!(rho > 0.0)) return 0;
    double vx = u[MX] / rho, vy = u[MY] / rho, vz = u[MZ] / rho;
    double kin = 0.5 * (u[MX] * u[MX] + u[MY] * u[MY] + u[MZ] * u[MZ]) / rho;
    double mag = 0.5 * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
    double p = (gamma - 1.0) * (u[ENG] - kin - mag);
    if (!(p > 0.0) || !isfinite(p)) return 0;
    v[RHO] = rho;
    v[VX] = vx;
    v[VY] = vy;
    v[VZ] = vz;
    v[PRS] = p;
    v[BX] = u[BX];
    v[BY] = u[BY];
    v[BZ] = u[BZ];
    v[PSI] = u[PSI];
    return 1;
}

/* primitive -> conservative; psi is not part of the energy */
static void prim_to_cons(const double *v, double gamma, double *u)
{
    double rho = v[RHO];
    u[RHO] = rho;
    u[MX] = rho * v[VX];
    u[MY] = rho * v[VY];
    u[MZ] = rho * v[VZ];
    u[ENG] = v[PRS] / (gamma - 1.0)
           + 0.5 * rho * (v[VX] * v[VX] + v[VY] * v[VY] + v[VZ] * v[VZ])
           + 0.5 * (v[BX] * v[BX] + v[BY] * v[BY] + v[BZ] * v[BZ]);
    u[BX] = v[BX];
    u[BY] = v[BY];
    u[BZ] = v[BZ];
    u[PSI] = v[PSI];
}

/* fast magnetosonic speed from density, pressure, |B|^2 and B_n^2:
 * c_f^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 (b^2 - b_n^2))) / 2
 * with a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_n^2 = B_n^2 / rho.       */
static double fast_speed_of(double rho, double p, double bsq, double bnsq, double gamma)
{
    double a2 = gamma * p / rho;
    double b2 = bsq / rho;
    double bn2 = bnsq / rho;
    double disc = (a2 - b2) * (a2 - b2) + 4.0 * a2 * (b2 - bn2);
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (a2 + b2 + sqrt(disc)));
}

/* fast speed along axis d of a primitive state */
static double fast_speed(const double *v, double gamma, int d)
{
    double bsq = v[BX] * v[BX] + v[BY] * v[BY] + v[BZ] * v[BZ];
    return fast_speed_of(v[RHO], v[PRS], bsq, v[BX + d] * v[BX + d], gamma);
}

/* limited slope from the left difference a and the right difference b */
static double limited_slope(int limiter, double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    double s = a > 0.0 ? 1.0 : -1.0;
    double m = fmin(fabs(a), fabs(b));
    if (limiter == ORC_MC) {
        /* monotonized central: minmod(2a, 2b, (a+b)/2) */
        m = fmin(2.0 * m, 0.5 * fabs(a + b));
    }
    return s * m;
}

/* WENO-Z value at the right face of the middle cell of v[0..4] (cells
 * i-2 .. i+2); the left face value of cell i is the same function of the
 * mirrored stencil. */
static double wenoz(const double *v)
{
    const double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    const double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    const double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    const double c = 13.0 / 12.0;
    const double b0 = c * (v[0] - 2.0 * v[1] + v[2]) * (v[0] - 2.0 * v[1] + v[2]) +
                      0.25 * (v[0] - 4.0 * v[1] + 3.0 * v[2]) * (v[0] - 4.0 * v[1] + 3.0 * v[2]);
    const double b1 = c * (v[1] - 2.0 * v[2] + v[3]) * (v[1] - 2.0 * v[2] + v[3]) +
                      0.25 * (v[1] - v[3]) * (v[1] - v[3]);
    const double b2 = c * (v[2] - 2.0 * v[3] + v[4]) * (v[2] - 2.0 * v[3] + v[4]) +
                      0.25 * (3.0 * v[2] - 4.0 * v[3] + v[4]) * (3.0 * v[2] - 4.0 * v[3] + v[4]);
    const double tau = fabs(b0 - b2);
    const double eps = 1e-40;
    const double a0 = 0.1 * (1.0 + tau / (b0 + eps));
    const double a1 = 0.6 * (1.0 + tau / (b1 + eps));
    const double a2 = 0.3 * (1.0 + tau / (b2 + eps));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* The rotated frame used by the one-dimensional solvers: for a face normal
 * to axis d the ordered triple (n, t1, t2) is the cyclic permutation
 * (x,y,z), (y,z,x) or (z,x,y).                                            */
static int axis_of(int d, int r) { return (d + r) % 3; }

/* Rotated 8-component MHD vectors: index 0 rho, 1..3 (normal, t1, t2)
 * velocity or momentum, 4 p or E, 5..7 (normal, t1, t2) magnetic field.    */

/* physical normal flux of the 8 MHD components, rotated frame;
 * q is (rho, u, vt1, vt2, p, Bn, Bt1, Bt2) and E the total energy.       */
static void physical_flux(const double *q, double E, double *f)
{
    double rho = q[0], u = q[1], v1 = q[2], v2 = q[3], p = q[4];
    double bn = q[5], b1 = q[6], b2 = q[7];
    double pt = p + 0.5 * (bn * bn + b1 * b1 + b2 * b2);
    double vb = u * bn + v1 * b1 + v2 * b2;
    f[0] = rho * u;
    f[1] = rho * u * u + pt - bn * bn;
    f[2] = rho * u * v1 - bn * b1;
    f[3] = rho * u * v2 - bn * b2;
    f[4] = (E + pt) * u - bn * vb;
    f[5] = 0.0;
    f[6] = u * b1 - v1 * bn;
    f[7] = u * b2 - v2 * bn;
}

static double total_energy(const double *q, double gamma)
{
    return q[4] / (gamma - 1.0)
         + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
         + 0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
}

static void rotated_cons(const double *q, double E, double *c)
{
    c[0] = q[0];
    c[1] = q[0] * q[1];
    c[2] = q[0] * q[2];
    c[3] = q[0] * q[3];
    c[4] = E;
    c[5] = q[5];
    c[6] = q[6];
    c[7] = q[7];
}

/* fast speed in the rotated frame (normal is slot 5) */
static double fast_speed_rot(const double *q, double gamma)
{
    double bsq = q[5] * q[5] + q[6] * q[6] + q[7] * q[7];
    return fast_speed_of(q[0], q[4], bsq, q[5] * q[5], gamma);
}

/* Harten-Lax-van Leer flux with Davis speed bounds, rotated frame */
static void hll_flux(const double *qL, const double *qR, double gamma, double *F)
{
    double EL = total_energy(qL, gamma), ER = total_energy(qR, gamma);
    double FL[8], FR[8], UL[8], UR[8];
    physical_flux(qL, EL, FL);
    physical_flux(qR, ER, FR);
    rotated_cons(qL, EL, UL);
    rotated_cons(qR, ER, UR);
    double cL = fast_speed_rot(qL, gamma), cR = fast_speed_rot(qR, gamma);
    double sL = fmin(qL[1] - cL, qR[1] - cR);
    double sR = fmax(qL[1] + cL, qR[1] + cR);
    if (sL >= 0.0) {
        memcpy(F, FL, sizeof FL);
    } else if (sR <= 0.0) {
        memcpy(F, FR, sizeof FR);
    } else {
        for (int k = 0; k < 8; ++k)
            F[k] = (sR * FL[k] - sL * FR[k] + sL * sR * (UR[k] - UL[k])) / (sR - sL);
    }
}

/* All intermediate states of the HLLD fan (Miyoshi & Kusano 2005) for two
 * rotated states with equal normal field.  Exposed for the tests.
 * speeds: sL, s*L, sM, s*R, sR.  Each state/flux is 8 rotated components. */
typedef struct {
    double s[5];
    double UL[8], UsL[8], UssL[8], UssR[8], UsR[8], UR[8];
    double FL[8], FR[8];
} hlld_fan;

/* one side (speed s) of the single-star state U* */
static void hlld_star_side(const double *q, double E, double pt, double s, double sM,
                           double pts, double *Us)
{
    double rho = q[0], u = q[1], bn = q[5];
    double rhos = rho * (s - u) / (s - sM);
    double D = rho * (s - u) * (s - sM) - bn * bn;
    double scale = fabs(rho * (s - u) * (s - sM)) + bn * bn;
    double vs1, vs2, bs1, bs2;
    if (fabs(D) <= 16.0 * DBL_EPSILON * scale) {
        /* degenerate (S* -> S): keep the tangential components */
        vs1 = q[2];
        vs2 = q[3];
        bs1 = q[6];
        bs2 = q[7];
    } else {
        double cv = bn * (sM - u) / D;
        double cb = (rho * (s - u) * (s - u) - bn * bn) / D;
        vs1 = q[2] - q[6] * cv;
        vs2 = q[3] - q[7] * cv;
        bs1 = q[6] * cb;
        bs2 = q[7] * cb;
    }
    double vb = u * bn + q[2] * q[6] + q[3] * q[7];
    double vbs = sM * bn + vs1 * bs1 + vs2 * bs2;
    double Es = ((s - u) * E - pt * u + pts * sM + bn * (vb - vbs)) / (s - sM);
    Us[0] = rhos;
    Us[1] = rhos * sM;
    Us[2] = rhos * vs1;
    Us[3] = rhos * vs2;
    Us[4] = Es;
    Us[5] = bn;
    Us[6] = bs1;
    Us[7] = bs2;
}

static void hlld_build_fan(const double *qL, const double *qR, double gamma, hlld_fan *fan)
{
    double EL = total_energy(qL, gamma), ER = total_energy(qR, gamma);
    physical_flux(qL, EL, fan->FL);
    physical_flux(qR, ER, fan->FR);
    rotated_cons(qL, EL, fan->UL);
    rotated_cons(qR, ER, fan->UR);
    double bn = qL[5]; /* equal on both sides after the GLM step */
    double cL = fast_speed_rot(qL, gamma), cR = fast_speed_rot(qR, gamma);
    double uL = qL[1], uR = qR[1];
    /* outer speeds: the slower (faster) normal velocity minus (plus) the
     * larger fast speed, a bound at least as wide as Davis's that keeps the
     * rotational waves S*_a inside [S_L, S_R] (D_a > 0) in the states where
     * Davis's bound lets D_a cross zero and the star states diverge */
    double cm = fmax(cL, cR);
    double sL = fmin(uL, uR) - cm;
    double sR = fmax(uL, uR) + cm;
    double ptL = qL[4] + 0.5 * (qL[5] * qL[5] + qL[6] * qL[6] + qL[7] * qL[7]);
    double ptR = qR[4] + 0.5 * (qR[5] * qR[5] + qR[6] * qR[6] + qR[7] * qR[7]);
    double mL = (sL - uL) * qL[0], mR = (sR - uR) * qR[0];
    double sM = (mR * uR - mL * uL - ptR + ptL) / (mR - mL);
    double pts = (mR * ptL - mL * ptR + mL * mR * (uR - uL)) / (mR - mL);

    hlld_star_side(qL, EL, ptL, sL, sM, pts, fan->UsL);
    hlld_star_side(qR, ER, ptR, sR, sM, pts, fan->UsR);

    double rsL = sqrt(fan->UsL[0]), rsR = sqrt(fan->UsR[0]);
    double sgn = bn >= 0.0 ? 1.0 : -1.0;
    double ssL = sM - fabs(bn) / rsL;
    double ssR = sM + fabs(bn) / rsR;

    /* star-state velocities and fields */
    double vL1 = fan->UsL[2] / fan->UsL[0], vL2 = fan->UsL[3] / fan->UsL[0];
    double vR1 = fan->UsR[2] / fan->UsR[0], vR2 = fan->UsR[3] / fan->UsR[0];
    double bL1 = fan->UsL[6], bL2 = fan->UsL[7], bR1 = fan->UsR[6], bR2 = fan->UsR[7];
    double den = rsL + rsR;
    double vss1 = (rsL * vL1 + rsR * vR1 + (bR1 - bL1) * sgn) / den;
    double vss2 = (rsL * vL2 + rsR * vR2 + (bR2 - bL2) * sgn) / den;
    double bss1 = (rsL * bR1 + rsR * bL1 + rsL * rsR * (vR1 - vL1) * sgn) / den;
    double bss2 = (rsL * bR2 + rsR * bL2 + rsL * rsR * (vR2 - vL2) * sgn) / den;
    double vbsL = sM * bn + vL1 * bL1 + vL2 * bL2;
    double vbsR = sM * bn + vR1 * bR1 + vR2 * bR2;
    double vbss = sM * bn + vss1 * bss1 + vss2 * bss2;
    double EssL = fan->UsL[4] - rsL * (vbsL - vbss) * sgn;
    double EssR = fan->UsR[4] + rsR * (vbsR - vbss) * sgn;

    double *A[2] = { fan->UssL, fan->UssR };
    const double *S[2] = { fan->UsL, fan->UsR };
    double Ess[2] = { EssL, EssR };
    for (int side = 0; side < 2; ++side) {
        double r = S[side][0];
        A[side][0] = r;
        A[side][1] = r * sM;
        A[side][2] = r * vss1;
        A[side][3] = r * vss2;
        A[side][4] = Ess[side];
        A[side][5] = bn;
        A[side][6] = bss1;
        A[side][7] = bss2;
    }
    fan->s[0] = sL;
    fan->s[1] = ssL;
    fan->s[2] = sM;
    fan->s[3] = ssR;
    fan->s[4] = sR;
}

static void hlld_flux(const double *qL, const double *qR, double gamma, double *F)
{
    hlld_fan fan;
    hlld_build_fan(qL, qR, gamma, &fan);
    double sL = fan.s[0], ssL = fan.s[1], sM = fan.s[2], ssR = fan.s[3], sR = fan.s[4];
    if (sL >= 0.0) {
        memcpy(F, fan.FL, sizeof fan.FL);
        return;
    }
    if (sR <= 0.0) {
        memcpy(F, fan.FR, sizeof fan.FR);
        return;
    }
    for (int k = 0; k < 8; ++k) {
        double fsL = fan.FL[k] + sL * (fan.UsL[k] - fan.UL[k]);
        double fsR = fan.FR[k] + sR * (fan.UsR[k] - fan.UR[k]);
        if (ssL >= 0.0) {
            F[k] = fsL;
        } else if (sM >= 0.0) {
            F[k] = fsL + ssL * (fan.UssL[k] - fan.UsL[k]);
        } else if (ssR >= 0.0) {
            F[k] = fsR + ssR * (fan.UssR[k] - fan.UsR[k]);
        } else {
            F[k] = fsR;
        }
    }
}

/* Exact solution of the GLM (B_n, psi) subsystem at an interface
 * (Dedner et al. 2002):  out[0] = B_n*, out[1] = psi*.                    */
static void glm_interface(double bnL, double bnR, double psiL, double psiR, double ch,
                          double *out)
{
    out[0] = 0.5 * (bnL + bnR) - (psiR - psiL) / (2.0 * ch);
    out[1] = 0.5 * (psiL + psiR) - 0.5 * ch * (bnR - bnL);
}

/* Full interface flux from two unrotated primitive face states (9 comps):
 * GLM interface solve, then the MHD solver on the 8 MHD components with
 * B_n replaced by B_n*, then F(B_n) = psi*, F(psi) = c_h^2 B_n*.          */
static void face_flux_bn(const orc_cfg *cfg, int d, const double *VL, const double *VR,
                         double ch, const double *bn_face, double *F)
{
    double bnL = VL[BX + d], bnR = VR[BX + d];
    double bns, psis;
    if (bn_face) {
        /* constrained transport: the normal field is the face's own value */
        bns = *bn_face;
        psis = 0.0;
    } else if (cfg->glm) {
        double g[2];
        glm_interface(bnL, bnR, VL[PSI], VR[PSI], ch, g);
        bns = g[0];
        psis = g[1];
    } else {
        bns = 0.5 * (bnL + bnR);
        psis = 0.0;
    }
    double qL[8], qR[8];
    const double *V2[2] = { VL, VR };
    double *Q2[2] = { qL, qR };
    for (int s = 0; s < 2; ++s) {
        const double *V = V2[s];
        double *q = Q2[s];
        q[0] = V[RHO];
        q[1] = V[VX + axis_of(d, 0)];
        q[2] = V[VX + axis_of(d, 1)];
        q[3] = V[VX + axis_of(d, 2)];
        q[4] = V[PRS];
        q[5] = bns;
        q[6] = V[BX + axis_of(d, 1)];
        q[7] = V[BX + axis_of(d, 2)];
    }
    double f[8];
    if (cfg->riemann == ORC_HLLD)
        hlld_flux(qL, qR, cfg->gamma, f);
    else
        hll_flux(qL, qR, cfg->gamma, f);
    F[RHO] = f[0];
    F[MX + axis_of(d, 0)] = f[1];
    F[MX + axis_of(d, 1)] = f[2];
    F[MX + axis_of(d, 2)] = f[3];
    F[ENG] = f[4];
    F[BX + axis_of(d, 1)] = f[6];
    F[BX + axis_of(d, 2)] = f[7];
    if (cfg->glm && !bn_face) {
        F[BX + d] = psis;
        F[PSI] = ch * ch * bns;
    } else {
        F[BX + d] = 0.0;
        F[PSI] = 0.0;
    }
}

static void face_flux(const orc_cfg *cfg, int d, const double *VL, const double *VR,
                      double ch, double *F)
{
    face_flux_bn(cfg, d, VL, VR, ch, NULL, F);
}

/* ------------------------------------------------------------------ */
/* grid with ghosts                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n[3];   /* interior cells */
    int64_t g[3];   /* ghost width: 3 on active axes, 0 otherwise */
    int64_t N[3];   /* padded extents */
    int64_t cells;  /* padded cell count */
} grid;

static void grid_make(const orc_cfg *cfg, grid *G)
{
    for (int d = 0; d < 3; ++d) {
        G->n[d] = cfg->n[d];
        G->g[d] = d < cfg->ndim ? 3 : 0;
        G->N[d] = G->n[d] + 2 * G->g[d];
    }
    G->cells = G->N[0] * G->N[1] * G->N[2];
}

/* padded index of interior coordinates (may be negative inside the ghosts) */
static int64_t pidx(const grid *G, int64_t i, int64_t j, int64_t k)
{
    return ((k + G->g[2]) * G->N[1] + (j + G->g[1])) * G->N[0] + (i + G->g[0]);
}

/* Fill the ghost layers of a padded primitive array W (AoS, 9 per cell).
 * Axes in the order x, y, z; every padded cell of the other axes is
 * covered, so corner ghosts are filled too (the stencil never reads them). */
static void fill_ghosts(const orc_cfg *cfg, const grid *G, double *W)
{
    for (int d = 0; d < cfg->ndim; ++d) {
        int64_t n = G->n[d];
        int64_t lo1 = -G->g[(d + 1) % 3], hi1 = G->n[(d + 1) % 3] + G->g[(d + 1) % 3];
        int64_t lo2 = -G->g[(d + 2) % 3], hi2 = G->n[(d + 2) % 3] + G->g[(d + 2) % 3];
        for (int64_t b = lo2; b < hi2; ++b) {
            for (int64_t a = lo1; a < hi1; ++a) {
                for (int side = 0; side < 2; ++side) {
                    for (int layer = 1; layer <= G->g[d]; ++layer) {
                        int64_t dst = side == 0 ? -layer : n - 1 + layer;
                        int64_t src;
                        if (cfg->bc[d][side] == ORC_PERIODIC)
                            src = ((dst % n) + n) % n;
                        else
                            src = side == 0 ? 0 : n - 1;
                        int64_t c[3], s[3];
                        c[d] = dst;
                        s[d] = src;
                        c[(d + 1) % 3] = s[(d + 1) % 3] = a;
                        c[(d + 2) % 3] = s[(d + 2) % 3] = b;
                        memcpy(&W[NV * pidx(G, c[0], c[1], c[2])],
                               &W[NV * pidx(G, s[0], s[1], s[2])], NV * sizeof(double));
                    }
                }
            }
        }
    }
}

/* Primitive padded array from an SoA conserved array; returns 0 if any
 * interior cell is non-physical. */
static int load_prims(const orc_cfg *cfg, const grid *G, const double *U, double *W)
{
    int64_t nx = G->n[0], ny = G->n[1], nz = G->n[2], nc = nx * ny * nz;
    int ok = 1;
#pragma omp parallel for reduction(&& : ok) schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        for (int64_t j = 0; j < ny; ++j) {
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = (k * ny + j) * nx + i;
                double u[NV];
                for (int q = 0; q < NV; ++q) u[q] = U[q * nc + c];
                if (!cons_to_prim(u, cfg->gamma, &W[NV * pidx(G, i, j, k)])) ok = 0;
            }
        }
    }
    if (ok) fill_ghosts(cfg, G, W);
    return ok;
}

/* L(U) for all interior cells, SoA [9][nz][ny][nx].  W holds primitives
 * with ghosts.  Each active direction is handled in turn: the flux through
 * every interface of a line is computed once and differenced.            */
/* With constrained transport (U non-NULL) the normal field of each face is
 * the face value held in U, and the two transverse field fluxes of every
 * cell's lower face along each axis go to Fl[6][nc]: (x face: F(By), F(Bz)),
 * (y face: F(Bx), F(Bz)), (z face: F(Bx), F(By)). */
static void rhs_from_prims(const orc_cfg *cfg, const grid *G, const double *W, double ch,
                           double *L, const double *U, double *Fl)
{
    int64_t nx = G->n[0], ny = G->n[1], nz = G->n[2], nc = nx * ny * nz;
    memset(L, 0, sizeof(double) * NV * nc);
    for (int d = 0; d < cfg->ndim; ++d) {
        double dx = (cfg->hi[d] - cfg->lo[d]) / (double)cfg->n[d];
        int64_t stride = d == 0 ? NV : (d == 1 ? NV * G->N[0] : NV * G->N[0] * G->N[1]);
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 0; k < nz; ++k) {
            for (int64_t j = 0; j < ny; ++j) {
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t c = (k * ny + j) * nx + i;
                    const double *Wc = &W[NV * pidx(G, i, j, k)];
                    double Fm[NV], Fp[NV];
                    /* faces c-1/2 and c+1/2 along d; face state on the left of
                     * face f+1/2 comes from cell f, on the right from f+1 */
                    for (int face = 0; face < 2; ++face) {
                        const double *A = Wc + (face == 0 ? -stride : 0); /* left cell */
                        const double *B = A + stride;                     /* right cell */
                        double VL[NV], VR[NV];
                        for (int q = 0; q < NV; ++q) {
                            if (cfg->limiter == ORC_WENOZ) {
                                double sa[5], sb[5];
                                for (int m = 0; m < 5; ++m) {
                                    sa[m] = A[q + (m - 2) * stride];  /* cells A-2 .. A+2 */
                                    sb[m] = B[q + (2 - m) * stride];  /* cells B+2 .. B-2 */
                                }
                                VL[q] = wenoz(sa);
                                VR[q] = wenoz(sb);
                            } else {
                                double sa = limited_slope(cfg->limiter, A[q] - A[q - stride],
                                                          B[q] - A[q]);
                                double sb = limited_slope(cfg->limiter, B[q] - A[q],
                                                          B[q + stride] - B[q]);
                                VL[q] = A[q] + 0.5 * sa;
                                VR[q] = B[q] - 0.5 * sb;
                            }
                        }
                        if (U) {
                            /* the lower face is this cell's, the upper one the
                             * next cell's along d (periodic) */
                            int64_t ii = i, jj = j, kk = k;
                            if (face == 1) {
                                if (d == 0) ii = (i + 1) % nx;
                                if (d == 1) jj = (j + 1) % ny;
                                if (d == 2) kk = (k + 1) % nz;
                            }
                            const double bn = U[(FBX + d) * nc + (kk * ny + jj) * nx + ii];
                            face_flux_bn(cfg, d, VL, VR, ch, &bn, face == 0 ? Fm : Fp);
                        } else {
                            face_flux(cfg, d, VL, VR, ch, face == 0 ? Fm : Fp);
                        }
                    }
                    if (Fl) {
                        /* the two transverse components in increasing order */
                        Fl[(2 * d) * nc + c] = Fm[d == 0 ? BY : BX];
                        Fl[(2 * d + 1) * nc + c] = Fm[d == 2 ? BY : BZ];
                    }
                    for (int q = 0; q < NV; ++q) L[q * nc + c] -= (Fp[q] - Fm[q]) / dx;
                }
            }
        }
    }
}

/* Constrained transport (Evans & Hawley 1988).  E = -v x B, so that
 * F_x(By) = -Ez, F_y(Bx) = Ez, F_y(Bz) = -Ex, F_z(By) = Ex, F_z(Bx) = -Ey,
 * F_x(Bz) = Ey.  E[3][nc] holds the EMFs on each cell's lower edges: Ex at
 * (j-1/2, k-1/2), Ey at (i-1/2, k-1/2), Ez at (i-1/2, j-1/2). */
#define CI(i, j, k) ((((k) + nz) % nz * ny + ((j) + ny) % ny) * nx + ((i) + nx) % nx)

/* Edge EMFs as the arithmetic mean of the four face fluxes around each edge
 * (Balsara & Spicer 1999). */
static void ct_emf_mean(const orc_cfg *cfg, const double *Fl, double *E)
{
    int64_t nx = cfg->n[0], ny = cfg->n[1], nz = cfg->n[2], nc = nx * ny * nz;
    const double *FxBy = Fl, *FxBz = Fl + nc, *FyBx = Fl + 2 * nc, *FyBz = Fl + 3 * nc;
    const double *FzBx = Fl + 4 * nc, *FzBy = Fl + 5 * nc;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = CI(i, j, k);
                E[c] = 0.25 * (-FyBz[CI(i, j, k - 1)] - FyBz[c] + FzBy[CI(i, j - 1, k)] + FzBy[c]);
                E[nc + c] = 0.25 * (FxBz[CI(i, j, k - 1)] + FxBz[c] - FzBx[CI(i - 1, j, k)] - FzBx[c]);
                E[2 * nc + c] = 0.25 * (-FxBy[CI(i, j - 1, k)] - FxBy[c] + FyBx[CI(i - 1, j, k)] + FyBx[c]);
            }
}

/* Upwind edge EMFs (Londrillo & Del Zanna 2004, upwind constrained
 * transport with HLL averaging).  For the EMF along axis e at an edge, with
 * (e, p, q) cyclic, four cells meet at the edge: the lower or upper one along
 * p (a = 0, 1) and along q (b = 0, 1).  Each gives a state at the edge:
 *   v^ab  = cell velocity + (1/2 - a) s_p(v) + (1/2 - b) s_q(v),
 *   B_q^a = the q-face field on side a, + (1/2 - a) s_p(B_q) along p,
 *   B_p^b = the p-face field on side b, + (1/2 - b) s_q(B_p) along q,
 *   E^ab  = -(v_p^ab B_q^a - v_q^ab B_p^b),
 * with s the minmod-limited slopes of cell (or face) values along an axis.
 * With HLL speed bounds a_p+ = max(0, v_p + c_f,p), a_p- = max(0, c_f,p - v_p)
 * over the four cells (and the same along q),
 *   E = sum_ab w_p^a w_q^b E^ab + a_p+ a_p- (B_q^1 - B_q^0) / (a_p+ + a_p-)
 *                                - a_q+ a_q- (B_p^1 - B_p^0) / (a_q+ + a_q-),
 * w_p^0 = a_p+ / (a_p+ + a_p-), w_p^1 = a_p- / (a_p+ + a_p-): along p the
 * HLL flux of B_q (F_p(B_q) = -E_e), along q that of B_p (F_q(B_p) = E_e).
 * Where the fields vary along p alone it is the one-dimensional HLL flux of
 * B_q at the p face.  W: primitives with ghosts (cell-centred B the face
 * means); U: the state with the face field. */
static void ct_emf_upwind(const orc_cfg *cfg, const grid *G, const double *W, const double *U,
                          double *E)
{
    int64_t nx = cfg->n[0], ny = cfg->n[1], nz = cfg->n[2], nc = nx * ny * nz;
    const double gamma = cfg->gamma;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t c = CI(i, j, k);
                for (int e = 0; e < 3; ++e) {
                    const int p = (e + 1) % 3, q = (e + 2) % 3;
                    int64_t dp[3] = {0, 0, 0}, dq[3] = {0, 0, 0};
                    dp[p] = 1;
                    dq[q] = 1;
                    double vp[2][2], vq[2][2];
                    double app = 0.0, apm = 0.0, aqp = 0.0, aqm = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b) {
                            /* cell (a, b) around the edge */
                            int64_t x = i + (a - 1) * dp[0] + (b - 1) * dq[0];
                            int64_t y = j + (a - 1) * dp[1] + (b - 1) * dq[1];
                            int64_t z = k + (a - 1) * dp[2] + (b - 1) * dq[2];
                            const double *V0 = &W[NV * pidx(G, x, y, z)];
                            const double *Vpm = &W[NV * pidx(G, x - dp[0], y - dp[1], z - dp[2])];
                            const double *Vpp = &W[NV * pidx(G, x + dp[0], y + dp[1], z + dp[2])];
                            const double *Vqm = &W[NV * pidx(G, x - dq[0], y - dq[1], z - dq[2])];
                            const double *Vqp = &W[NV * pidx(G, x + dq[0], y + dq[1], z + dq[2])];
                            const int up = VX + p, uq = VX + q;
                            double spp = limited_slope(ORC_MINMOD, V0[up] - Vpm[up], Vpp[up] - V0[up]);
                            double sqp = limited_slope(ORC_MINMOD, V0[up] - Vqm[up], Vqp[up] - V0[up]);
                            double spq = limited_slope(ORC_MINMOD, V0[uq] - Vpm[uq], Vpp[uq] - V0[uq]);
                            double sqq = limited_slope(ORC_MINMOD, V0[uq] - Vqm[uq], Vqp[uq] - V0[uq]);
                            vp[a][b] = V0[up] + (0.5 - a) * spp + (0.5 - b) * sqp;
                            vq[a][b] = V0[uq] + (0.5 - a) * spq + (0.5 - b) * sqq;
                            double cp = fast_speed(V0, gamma, p), cq = fast_speed(V0, gamma, q);
                            app = fmax(app, V0[up] + cp);
                            apm = fmax(apm, cp - V0[up]);
                            aqp = fmax(aqp, V0[uq] + cq);
                            aqm = fmax(aqm, cq - V0[uq]);
                        }
                    double Bq[2], Bp[2];
                    for (int a = 0; a < 2; ++a) {
                        /* q face of the cell on side a along p (at the edge's q) */
                        int64_t x = i + (a - 1) * dp[0], y = j + (a - 1) * dp[1], z = k + (a - 1) * dp[2];
                        const double *F = &U[(FBX + q) * nc];
                        double f0 = F[CI(x, y, z)];
                        double s = limited_slope(ORC_MINMOD, f0 - F[CI(x - dp[0], y - dp[1], z - dp[2])],
                                                 F[CI(x + dp[0], y + dp[1], z + dp[2])] - f0);
                        Bq[a] = f0 + (0.5 - a) * s;
                    }
                    for (int b = 0; b < 2; ++b) {
                        int64_t x = i + (b - 1) * dq[0], y = j + (b - 1) * dq[1], z = k + (b - 1) * dq[2];
                        const double *F = &U[(FBX + p) * nc];
                        double f0 = F[CI(x, y, z)];
                        double s = limited_slope(ORC_MINMOD, f0 - F[CI(x - dq[0], y - dq[1], z - dq[2])],
                                                 F[CI(x + dq[0], y + dq[1], z + dq[2])] - f0);
                        Bp[b] = f0 + (0.5 - b) * s;
                    }
                    double sp = app + apm, sq = aqp + aqm;
                    double wp[2] = {app / sp, apm / sp}, wq[2] = {aqp / sq, aqm / sq};
                    double Em = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            Em += wp[a] * wq[b] * (-(vp[a][b] * Bq[a] - vq[a][b] * Bp[b]));
                    Em += app * apm / sp * (Bq[1] - Bq[0]) - aqp * aqm / sq * (Bp[1] - Bp[0]);
                    E[e * nc + c] = Em;
                }
            }
}

/* Face rates dB/dt = -curl E of every cell's lower faces, to L[FBX..FBZ]. */
static void ct_face_rates(const orc_cfg *cfg, const double *E, double *L)
{
    int64_t nx = cfg->n[0], ny = cfg->n[1], nz = cfg->n[2], nc = nx * ny * nz;
    double dx = (cfg->hi[0] - cfg->lo[0]) / (double)nx;
    double dy = (cfg->hi[1] - cfg->lo[1]) / (double)ny;
    double dz = (cfg->hi[2] - cfg->lo[2]) / (double)nz;
    const double *Ex = E, *Ey = E + nc, *Ez = E + 2 * nc;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = CI(i, j, k);
                L[FBX * nc + c] = -((Ez[CI(i, j + 1, k)] - Ez[c]) / dy - (Ey[CI(i, j, k + 1)] - Ey[c]) / dz);
                L[FBY * nc + c] = -((Ex[CI(i, j, k + 1)] - Ex[c]) / dz - (Ez[CI(i + 1, j, k)] - Ez[c]) / dx);
                L[FBZ * nc + c] = -((Ey[CI(i + 1, j, k)] - Ey[c]) / dx - (Ex[CI(i, j + 1, k)] - Ex[c]) / dy);
            }
}

/* cell-centred B of every cell from its two faces along each axis */
static void ct_cell_field(const orc_cfg *cfg, double *U)
{
    int64_t nx = cfg->n[0], ny = cfg->n[1], nz = cfg->n[2], nc = nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = CI(i, j, k);
                U[BX * nc + c] = 0.5 * (U[FBX * nc + c] + U[FBX * nc + CI(i + 1, j, k)]);
                U[BY * nc + c] = 0.5 * (U[FBY * nc + c] + U[FBY * nc + CI(i, j + 1, k)]);
                U[BZ * nc + c] = 0.5 * (U[FBZ * nc + c] + U[FBZ * nc + CI(i, j, k + 1)]);
            }
#undef CI
}

/* Edge EMFs E[3][nc] of the state (constrained transport), from the face
 * fluxes Fl (ct = 1) or the primitives W with ghosts (ct = 2). */
static void ct_emf(const orc_cfg *cfg, const grid *G, const double *W, const double *U,
                   const double *Fl, double *E)
{
    if (cfg->ct == 2)
        ct_emf_upwind(cfg, G, W, U, E);
    else
        ct_emf_mean(cfg, Fl, E);
}

static int rhs(const orc_cfg *cfg, const double *U, double ch, double *L)
{
    grid G;
    grid_make(cfg, &G);
    int64_t nc = cfg->n[0] * cfg->n[1] * cfg->n[2];
    double *W = (double *)malloc(sizeof(double) * NV * G.cells);
    double *Fl = cfg->ct ? (double *)malloc(sizeof(double) * 6 * nc) : NULL;
    double *E = cfg->ct ? (double *)malloc(sizeof(double) * 3 * nc) : NULL;
    if (!W || (cfg->ct && (!Fl || !E))) {
        free(W);
        free(Fl);
        free(E);
        return 2;
    }
    int ok = load_prims(cfg, &G, U, W);
    if (ok) rhs_from_prims(cfg, &G, W, ch, L, cfg->ct ? U : NULL, Fl);
    if (ok && cfg->ct) {
        ct_emf(cfg, &G, W, U, Fl, E);
        ct_face_rates(cfg, E, L);
    }
    free(W);
    free(Fl);
    free(E);
    return ok ? 0 : 1;
}

/* ------------------------------------------------------------------ */
/* exported entry points (ctypes)                                       */
/* ------------------------------------------------------------------ */

static int cfg_ok(const orc_cfg *cfg)
{
    if (!cfg || cfg->ndim < 1 || cfg->ndim > 3) return 0;
    for (int d = 0; d < 3; ++d) {
        if (cfg->n[d] < 1) return 0;
        if (d >= cfg->ndim && cfg->n[d] != 1) return 0;
        if (d < cfg->ndim && !(cfg->hi[d] > cfg->lo[d])) return 0;
    }
    if (cfg->limiter < ORC_MINMOD || cfg->limiter > ORC_WENOZ) return 0;
    if (cfg->time_order != 2 && cfg->time_order != 3) return 0;
    if (cfg->ct < 0 || cfg->ct > 2) return 0;
    if (cfg->ct) {
        /* three-dimensional, periodic, no GLM */
        if (cfg->ndim != 3 || cfg->glm) return 0;
        for (int d = 0; d < 3; ++d)
            if (cfg->bc[d][0] != ORC_PERIODIC || cfg->bc[d][1] != ORC_PERIODIC) return 0;
    }
    return cfg->gamma > 1.0;
}

static int64_t ncells(const orc_cfg *cfg) { return cfg->n[0] * cfg->n[1] * cfg->n[2]; }

/* With constrained transport V and U carry the face field in slots
 * FBX..FBZ; the cell-centred B of U (and the B entering E) is the average of
 * the faces, whatever V holds in BX..BZ. */
int orc_prim_to_cons(const orc_cfg *cfg, const double *V, double *U)
{
    if (!cfg_ok(cfg)) return 2;
    int64_t nc = ncells(cfg);
    if (cfg->ct) {
        for (int q = FBX; q <= FBZ; ++q) memcpy(&U[q * nc], &V[q * nc], sizeof(double) * nc);
        ct_cell_field(cfg, U);
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[NV], u[NV];
        for (int q = 0; q < NV; ++q) v[q] = V[q * nc + c];
        if (cfg->ct)
            for (int q = BX; q <= BZ; ++q) v[q] = U[q * nc + c];
        prim_to_cons(v, cfg->gamma, u);
        for (int q = 0; q < NV; ++q) U[q * nc + c] = u[q];
    }
    return 0;
}

int orc_cons_to_prim(const orc_cfg *cfg, const double *U, double *V)
{
    if (!cfg_ok(cfg)) return 2;
    int64_t nc = ncells(cfg);
    int ok = 1;
#pragma omp parallel for reduction(&& : ok) schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[NV], u[NV];
        for (int q = 0; q < NV; ++q) u[q] = U[q * nc + c];
        if (!cons_to_prim(u, cfg->gamma, v)) {
            ok = 0;
            continue;
        }
        for (int q = 0; q < NV; ++q) V[q * nc + c] = v[q];
    }
    if (cfg->ct)
        for (int q = FBX; q <= FBZ; ++q) memcpy(&V[q * nc], &U[q * nc], sizeof(double) * nc);
    return ok ? 0 : 1;
}

/* out[0] = dt = C / max (|v_d| + c_f,d)/dx_d (not clipped), out[1] = c_h */
int orc_cfl(const orc_cfg *cfg, const double *U, double *out)
{
    if (!cfg_ok(cfg)) return 2;
    int64_t nc = ncells(cfg);
    double smax = 0.0, cmax = 0.0;
    int ok = 1;
    /* maxima do not depend on the order of the cells */
#pragma omp parallel for reduction(max : smax, cmax) reduction(&& : ok) schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double v[NV], u[NV];
        for (int q = 0; q < NV; ++q) u[q] = U[q * nc + c];
        if (!cons_to_prim(u, cfg->gamma, v)) {
            ok = 0;
            continue;
        }
        for (int d = 0; d < cfg->ndim; ++d) {
            double dx = (cfg->hi[d] - cfg->lo[d]) / (double)cfg->n[d];
            double lam = fabs(v[VX + d]) + fast_speed(v, cfg->gamma, d);
            if (lam / dx > smax) smax = lam / dx;
            if (lam > cmax) cmax = lam;
        }
    }
    if (!ok) return 1;
    out[0] = cfg->cfl / smax;
    out[1] = cmax;
    return 0;
}

int orc_rhs(const orc_cfg *cfg, const double *U, double ch, double *L)
{
    if (!cfg_ok(cfg)) return 2;
    return rhs(cfg, U, ch, L);
}

/* One SSP-RK2 or SSP-RK3 step with GLM damping.  U1_out (the first stage
 * state) may be NULL.  With constrained transport the face field takes the
 * same stage combinations and every stage's cell-centred B is then re-formed
 * from the faces. */
int orc_step(const orc_cfg *cfg, const double *Un, double *Unext, double *U1_out, double dt,
             double ch, double damp)
{
    if (!cfg_ok(cfg) || Un == Unext) return 2;
    int64_t nc = ncells(cfg), nt = nstate(cfg) * nc;
    double *L = (double *)malloc(sizeof(double) * nt);
    double *U1 = (double *)malloc(sizeof(double) * nt);
    if (!L || !U1) {
        free(L);
        free(U1);
        return 2;
    }
    int st = rhs(cfg, Un, ch, L);
    if (st == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < nt; ++a) U1[a] = Un[a] + dt * L[a];
        if (cfg->ct) ct_cell_field(cfg, U1);
        st = rhs(cfg, U1, ch, L);
    }
    if (st == 0 && cfg->time_order == 3) {
        if (U1_out) memcpy(U1_out, U1, sizeof(double) * nt);
        /* U2 = 3/4 Un + 1/4 (U1 + dt L(U1)), stored over U1 */
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < nt; ++a) U1[a] = 0.75 * Un[a] + 0.25 * (U1[a] + dt * L[a]);
        if (cfg->ct) ct_cell_field(cfg, U1);
        st = rhs(cfg, U1, ch, L);
        if (st == 0) {
#pragma omp parallel for schedule(static)
            for (int64_t a = 0; a < nt; ++a)
                Unext[a] = Un[a] / 3.0 + 2.0 / 3.0 * (U1[a] + dt * L[a]);
            if (cfg->ct) ct_cell_field(cfg, Unext);
            for (int64_t c = 0; c < nc; ++c) Unext[PSI * nc + c] *= damp;
        }
    } else if (st == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < nt; ++a) Unext[a] = 0.5 * (Un[a] + U1[a] + dt * L[a]);
        if (cfg->ct) ct_cell_field(cfg, Unext);
        for (int64_t c = 0; c < nc; ++c) Unext[PSI * nc + c] *= damp;
        if (U1_out) memcpy(U1_out, U1, sizeof(double) * nt);
    }
    free(L);
    free(U1);
    return st;
}

/* pairwise sum of x[0..n) */
static double pairwise(const double *x, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t a = 0; a < n; ++a) s += x[a];
        return s;
    }
    int64_t h = n / 2;
    return pairwise(x, h) + pairwise(x + h, n - h);
}

/* out[q] = sum over cells of U_q * cell volume (active axes only) */
int orc_sums(const orc_cfg *cfg, const double *U, double *out)
{
    if (!cfg_ok(cfg)) return 2;
    int64_t nc = ncells(cfg);
    double vol = 1.0;
    for (int d = 0; d < cfg->ndim; ++d) vol *= (cfg->hi[d] - cfg->lo[d]) / (double)cfg->n[d];
    for (int q = 0; q < NV; ++q) out[q] = pairwise(U + q * nc, nc) * vol;
    return 0;
}

/* ---- pointwise pieces, exported for the pin tests ---------------- */

double orc_fast_speed(const double *V, double gamma, int d) { return fast_speed(V, gamma, d); }

double orc_limited_slope(int limiter, double a, double b) { return limited_slope(limiter, a, b); }

double orc_wenoz(const double *v) { return wenoz(v); }

void orc_glm_interface(double bnL, double bnR, double psiL, double psiR, double ch, double *out)
{
    glm_interface(bnL, bnR, psiL, psiR, ch, out);
}

/* interface flux from unrotated primitive face states (9 components) */
int orc_face_flux(const orc_cfg *cfg, int d, const double *VL, const double *VR, double ch,
                  double *F)
{
    if (!cfg || d < 0 || d > 2) return 2;
    face_flux(cfg, d, VL, VR, ch, F);
    return 0;
}

/* HLLD fan of two rotated primitive states q = (rho,u,vt1,vt2,p,Bn,Bt1,Bt2)
 * with equal Bn.  out layout: s[5], UL, UsL, UssL, UssR, UsR, UR, FL, FR
 * (8 each) = 69 doubles. */
void orc_hlld_fan(const double *qL, const double *qR, double gamma, double *out)
{
    hlld_fan fan;
    hlld_build_fan(qL, qR, gamma, &fan);
    memcpy(out, fan.s, 5 * sizeof(double));
    const double *parts[8] = { fan.UL, fan.UsL, fan.UssL, fan.UssR, fan.UsR, fan.UR, fan.FL, fan.FR };
    for (int p = 0; p < 8; ++p) memcpy(out + 5 + 8 * p, parts[p], 8 * sizeof(double));
}

/* rotated-frame solver fluxes (8 components) for the pin tests */
void orc_rotated_flux(int riemann, const double *qL, const double *qR, double gamma, double *F)
{
    if (riemann == ORC_HLLD)
        hlld_flux(qL, qR, gamma, F);
    else
        hll_flux(qL, qR, gamma, F);
}

/* edge EMFs E[3][nc] of a constrained-transport state (for the pin tests):
 * Ex, Ey, Ez on each cell's lower edges; c_h is unused without GLM */
int orc_ct_emf(const orc_cfg *cfg, const double *U, double *E)
{
    if (!cfg_ok(cfg) || !cfg->ct) return 2;
    grid G;
    grid_make(cfg, &G);
    int64_t nc = ncells(cfg);
    double *W = (double *)malloc(sizeof(double) * NV * G.cells);
    double *Fl = (double *)malloc(sizeof(double) * 6 * nc);
    double *L = (double *)malloc(sizeof(double) * NV * nc);
    if (!W || !Fl || !L) {
        free(W);
        free(Fl);
        free(L);
        return 2;
    }
    int ok = load_prims(cfg, &G, U, W);
    if (ok) {
        rhs_from_prims(cfg, &G, W, 1.0, L, U, Fl);
        ct_emf(cfg, &G, W, U, Fl, E);
    }
    free(W);
    free(Fl);
    free(L);
    return ok ? 0 : 1;
}

/* host threads of the parallel loops (for the timed CPU baseline): set and
 * query the OpenMP team size */
void orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int orc_threads(void) { return omp_get_max_threads(); }
