// Fused Runge-Kutta stage kernel: ghost fill (index remap), conservative ->
// primitive, reconstruction (PLM or WENO-Z), GLM + Riemann fluxes on every
// face, flux divergence and the stage combine, in one pass over the grid.
//
// Work decomposition (gfx950, wave64):
//   * a workgroup owns a tile of TX = 64 (x) by TY (y) columns and marches
//     along z over a chunk of planes [k0, k1);
//   * one wave per tile row, one lane per column; the primitive state of
//     the current plane, with an x/y halo of the stencil's half width (2
//     cells PLM, 3 WENO-Z), sits in LDS;
//   * z-faces come from a per-lane register window slid along the march
//     (PLM: V(k), V(k+1) and the limited slope of V(k); WENO-Z: V(k-1) ..
//     V(k+2) and the upper face value of cell k), so every z-face flux is
//     computed once per chunk plus one warm-up face;
//   * x- and y-faces of the plane are a flat work list of
//     TY(TX+1) + (TY+1)TX items spread over the workgroup; their fluxes
//     go through LDS to the cells on both sides, so each face is solved
//     once per tile.  WENO-Z first reconstructs every cell the faces need
//     once per direction (both of its face values) into LDS;
//   * ghost cells are never stored: out-of-range coordinates are mapped to
//     interior cells by the boundary rule when addresses are formed.
// Stage kinds (KIND): 1 writes U1 = Un + dt L(Un); 2 the SSP-RK2 result
// (Un + U1 + dt L(U1)) / 2; 3 the SSP-RK3 stage 3/4 Un + 1/4 (U1 + dt L(U1));
// 4 the SSP-RK3 result 1/3 Un + 2/3 (U2 + dt L(U2)).  The last stage of
// either integrator damps psi and reduces on its output the CFL maxima and
// the FP64 conservation sums into per-block partials (with helper waves,
// the helpers take these reductions off the column owners).
#pragma once

#include <type_traits>

#include "mhd_physics.hpp"

namespace mhd {

constexpr int TX = 64;
// partial layout: [NPART][nblocks]; 0: max (|v|+cf)/dx, 1: max (|v|+cf),
// 2..10: sums of the 9 conserved components
constexpr int NPART = 11;

template <typename T> struct StageArgs {
    const T *uin;   // state the fluxes are built from (Un or U1); with
                    // constrained transport its components 9..11 are the
                    // face field on each cell's lower x, y, z face
    T *flx;         // constrained transport with the mean edge EMF: [6][ncell]
                    // transverse field fluxes of each cell's lower faces
                    // (x: By, Bz; y: Bx, Bz; z: Bx, By); null with the
                    // upwind EMF, which does not use them
    const T *un;    // Un (later stages' combine); equals uin in stage 1
    T *uout;        // this stage's output (U1, U2 or U_next)
    double *part;   // last stage: NPART x nblocks partials
    int *flag;      // non-physical flag
    int nx, ny, nz; // interior cells
    long long nxy;  // nx*ny
    long long ncell;
    int per[3];     // periodic per axis
    int kz;         // planes per chunk
    int tiles_x, tiles_y, chunks;
    int nblocks;
    T dt;
    T idx[3];       // 1/dx per axis
    T damp;
    double gamma_d; // FP64 copies for the reductions
    double idx_d[3];
    Phys<T> ph;
};

// Logical block id from the hardware id.  Consecutive hardware ids are
// dispatched round-robin over the 8 XCDs; giving each XCD a contiguous
// range of logical ids keeps neighbouring tiles (shared halos) in one L2.
__device__ __forceinline__ int logical_block(int hw, int nblocks)
{
    if ((nblocks & 7) != 0) return hw;
    return (hw & 7) * (nblocks >> 3) + (hw >> 3);
}

// FP64 signal speeds of one conserved cell state (any T), for the CFL
// reduction: smax = max_d (|v_d| + c_f,d)/dx_d, cmax = max_d (|v_d| + c_f,d).
template <typename T, int NDIM>
__device__ __forceinline__ bool cell_speeds(const T *u, double gamma, const double *idx,
                                            double &smax, double &cmax)
{
    const double rho = (double)u[RHO];
    const double ir = 1.0 / rho;
    const double m[3] = {(double)u[MX], (double)u[MY], (double)u[MZ]};
    const double b[3] = {(double)u[BX], (double)u[BY], (double)u[BZ]};
    const double bsq = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double kin = 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir;
    const double p = (gamma - 1.0) * ((double)u[ENG] - kin - 0.5 * bsq);
    bool ok = (rho > 0.0) & (rho < 1e300) & (p > 0.0) & (p < 1e300);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        const double lam = __builtin_fabs(m[d] * ir) + fast_speed(p, bsq, b[d] * b[d], gamma, ir);
        smax = __builtin_fmax(smax, lam * idx[d]);
        cmax = __builtin_fmax(cmax, lam);
    }
    return ok;
}

// FP32 signal speeds of one FP32 cell state, used only to pick the cell
// whose FP64 speeds a thread reports: ls = max_d (|v_d| + c_f,d)/dx_d,
// lc = max_d (|v_d| + c_f,d).  The discriminant is formed from the
// transverse field, (a^2 - b^2)^2 + 4 a^2 b_t^2, a sum of non-negative terms;
// the estimate carries rounding of the order of ten FP32 ulps plus the FP32
// pressure's cancellation, which reaches |v| + c_f only through the sound
// speed (about gamma M / 4 ulps at Mach M).
// Returns false for rho <= 0, p <= 0 or non-finite values.
template <int NDIM>
__device__ __forceinline__ bool cell_speeds_f32(const float *u, float gamma, const float *idx, float &ls,
                                                float &lc)
{
    const float rho = u[RHO];
    const float ir = __builtin_amdgcn_rcpf(rho);
    const float m[3] = {u[MX], u[MY], u[MZ]};
    const float b[3] = {u[BX], u[BY], u[BZ]};
    const float bb[3] = {b[0] * b[0], b[1] * b[1], b[2] * b[2]};
    const float bsq = bb[0] + bb[1] + bb[2];
    const float kin = 0.5f * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir;
    const float p = (gamma - 1.0f) * (u[ENG] - kin - 0.5f * bsq);
    const bool ok = (rho > 0.0f) & (rho < 1e30f) & (p > 0.0f) & (p < 1e30f);
    const float a2 = gamma * p * ir;
    const float b2 = bsq * ir;
    const float dab = a2 - b2;
    ls = 0.0f;
    lc = 0.0f;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        const float bt2 = (bb[(d + 1) % 3] + bb[(d + 2) % 3]) * ir;
        const float disc = dab * dab + 4.0f * a2 * bt2;
        const float cf = __builtin_amdgcn_sqrtf(0.5f * (a2 + b2 + __builtin_amdgcn_sqrtf(disc)));
        const float lam = __builtin_fabsf(m[d] * ir) + cf;
        ls = __builtin_fmaxf(ls, lam * idx[d]);
        lc = __builtin_fmaxf(lc, lam);
    }
    return ok;
}

template <typename T>
__device__ __forceinline__ void load_cell(const T *__restrict__ U, long long ncell, long long c, T *u)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) u[q] = U[q * ncell + c];
}

// Wave64 sum / max of a double.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = __builtin_fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Waves per SIMD the kernels are compiled for.  FP32 PLM: 3, a budget of 168
// registers (stage 1 needs 127, so four 4-wave workgroups share a compute
// unit; the last stage 165, three).  FP32 WENO-Z: 2 (256 registers; its
// 8-row workgroups take 155 KB of LDS, one per compute unit).  FP64 PLM: 2
// (256 registers; the HLLD kernels spill some of them, and still run 11%
// faster than at one wave per SIMD without spills).  FP64 WENO-Z: 2 (140 KB
// of LDS, the fluxes laid over the primitive plane, allows one workgroup per
// compute unit: 4 rows with two waves each, the helper waves below; 256
// registers, some spilled: the 416^3 SSP-RK3 step ran 14% faster than with
// one 4-wave workgroup at 512 registers, before the last stage's reductions
// moved to the helpers).
template <typename T, int LIM> constexpr int stage_min_waves()
{
    return sizeof(T) == 4 ? (LIM == LIM_WENOZ ? 2 : 3) : 2;
}

// Waves per tile row.  FP64 WENO-Z's arrays leave room for one workgroup per
// compute unit; a second wave per row (a helper that owns no column) shares
// the halo conversions, the WENO-Z reconstructions and the x/y face fluxes
// of the plane, so that those phases run two waves per SIMD instead of one.
// The z march (register window, z faces) and the update stay with the
// column owners.
template <typename T, int LIM> constexpr int stage_row_waves()
{
    return (sizeof(T) == 8 && LIM == LIM_WENOZ) ? 2 : 1;
}

// Stage kinds of the Runge-Kutta integrators (KIND): 1 U1 = Un + dt L(Un)
// (first stage of both); 2 SSP-RK2 second and last stage
// (Un + U1 + dt L(U1))/2; 3 SSP-RK3 second stage 3/4 Un + 1/4 (U1 + dt L(U1));
// 4 SSP-RK3 last stage 1/3 Un + 2/3 (U2 + dt L(U2)).  The last stage damps
// psi and reduces the CFL maxima and the conservation sums.
constexpr bool last_stage(int kind) { return kind == 2 || kind == 4; }

template <typename T, int SOLVER, int LIM, int NDIM, int KIND, int TY, bool CT = false>
__global__ void __launch_bounds__(TX *TY *(stage_row_waves<T, LIM>()), (stage_min_waves<T, LIM>()))
stage_kernel(const StageArgs<T> a)
{
    constexpr bool WENO = LIM == LIM_WENOZ;
    // with constrained transport the cell field is final only after the
    // face update, which therefore takes the last stage's reductions
    constexpr bool LAST = last_stage(KIND) && !CT;
    static_assert(!CT || NDIM == 3, "constrained transport is three-dimensional");
    constexpr int H = WENO ? 3 : 2;        // stencil half width (ghost layers)
    constexpr int NW = TY * stage_row_waves<T, LIM>();  // waves: TY column owners, then helpers
    constexpr int NT = TX * NW;
    constexpr int HY = NDIM >= 2 ? H : 0;  // y halo width in LDS
    constexpr int PX = TX + 2 * H;         // LDS row pitch
    constexpr int PY = TY + 2 * HY;        // LDS rows
    constexpr int PLANE = PX * PY;         // LDS elements per component
    constexpr int NFX = TY * (TX + 1);     // x-face items
    constexpr int NFY = NDIM >= 2 ? (TY + 1) * TX : 0;
    constexpr int NCHX = (NFX + TX - 1) / TX;       // 64-wide chunks of x items
    constexpr int NCHUNK = NCHX + NFY / TX;          // NFY is a multiple of TX
    constexpr int NHX = 2 * H * TY;        // x-halo cells
    constexpr int NH = NHX + (NDIM >= 2 ? 2 * H * TX : 0);
    // WENO-Z reconstructs every cell once per direction (both of its face
    // values) before the face fluxes: x for cells -1 .. TX of each row, y for
    // rows -1 .. TY of each column; the values go to LDS edge arrays
    // E[2][NQ][rows][cells] (right/upper face first).
    constexpr int NXE = TX + 2;                          // cells per row with an x edge
    constexpr int NYE = TY + 2;                          // rows with a y edge
    constexpr int NRX = WENO ? TY * NXE : 0;             // x reconstruction items
    constexpr int NRY = (WENO && NDIM >= 2) ? NYE * TX : 0;
    constexpr int NRCH = (NRX + NRY + TX - 1) / TX;      // their 64-wide chunks
    // LDS: [P][FX][FY] and, for WENO-Z, [EX][EY]; when that exceeds the 160 KB
    // of a compute unit (FP64), FX and FY go over P once P is used, and the
    // next plane's loads wait for the update (one more barrier per plane)
    constexpr int SZP = NQ * PLANE;
    constexpr int SZFX = NQ * TY * (TX + 1);
    constexpr int SZFY = NDIM >= 2 ? NQ * (TY + 1) * TX : 0;
    constexpr int SZEX = WENO ? 2 * NQ * TY * NXE : 0;
    constexpr int SZEY = (WENO && NDIM >= 2) ? 2 * NQ * NYE * TX : 0;
    constexpr bool ALIAS = WENO && (SZP + SZFX + SZFY + SZEX + SZEY) * (int)sizeof(T) > 160 * 1024;
    constexpr int OFX = ALIAS ? 0 : SZP;
    constexpr int OFY = OFX + SZFX;
    constexpr int OEX = ALIAS ? (SZP > SZFX + SZFY ? SZP : SZFX + SZFY) : OFY + SZFY;
    constexpr int OEY = OEX + SZEX;
    constexpr int SZL0 = OEY + SZEY;
    // Last stage with helper waves: the column owners leave each plane's
    // results in LDS (OUTS[NQ][TY * TX]) and the helpers take their FP64
    // sums and signal speeds during the next plane's z-face phase, which
    // is the owners' alone; the owners then carry no reduction state
    // through the march.
    constexpr bool HELP_RED = LAST && stage_row_waves<T, LIM>() > 1;
    static_assert(!HELP_RED || sizeof(T) == 8, "helper reductions keep FP64 sums in T registers");
    constexpr int OOUT = SZL0;
    constexpr int SZL = OOUT + (HELP_RED ? NQ * TY * TX : 0);
    static_assert(SZL * (int)sizeof(T) <= 160 * 1024, "LDS of one compute unit");

    __shared__ T lds[SZL];
    // With helper waves (FP64 WENO-Z) the reconstruction chunks of a plane
    // are handed out through this counter, one more barrier after the plane
    // load letting the helpers start on them while the column owners form the
    // plane's z faces (the owners take what is left): 416^3 SSP-RK3 step
    // 47.8 -> 46.2 ms.  The chunk order changes no arithmetic.
    constexpr bool OVERLAP = WENO && stage_row_waves<T, LIM>() > 1 && NDIM == 3;
    __shared__ int chunk_next;
    T *const P = lds;
    T *const FXs = lds + OFX;
    T *const FYs = lds + OFY;
    T *const EX = lds + OEX;
    T *const EY = lds + OEY;
    T *const OUTS = lds + OOUT;

    const int t = threadIdx.x;
    const int tx = t & (TX - 1);
    const int ty = t / TX;  // tile row of a column owner (>= TY: helper)
    const int wave = __builtin_amdgcn_readfirstlane(ty);
    // With one wave per tile row every wave owns its row.  For the 3D FP32
    // kernels the owner test is folded at compile time: the compiler then
    // holds the PLM stages to 127 and 165 registers (four and three
    // workgroups per compute unit) instead of 138 and 168 with 8 spilled, and
    // the WENO-Z stages (one workgroup per unit either way) run 1-4% faster.
    // Elsewhere it is left to run time, which the compiler's allocation
    // favours (FP64 PLM: 0 and 24 spilled registers against 28 and 87; 2D
    // FP32 PLM: 127 against 129, a workgroup per compute unit more).
    constexpr bool ALL_OWN = stage_row_waves<T, LIM>() == 1 && sizeof(T) == 4 && NDIM == 3;
    const bool owner = ALL_OWN || wave < TY;  // wave-uniform
    const int lb = logical_block(blockIdx.x, a.nblocks);
    const int tile_x = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int tile_y = rest % a.tiles_y;
    const int chunk = rest / a.tiles_y;
    const int i0 = tile_x * TX, j0 = tile_y * TY;
    const int k0 = chunk * a.kz;
    const int k1 = min(k0 + a.kz, a.nz);
    const int i = i0 + tx, j = j0 + ty;
    const bool active = owner & (i < a.nx) & (j < a.ny);

    // own column (remapped so that columns just past the grid edge hold the
    // ghost values their active neighbours need)
    const long long own = (long long)remap_index(j, a.ny, a.per[1]) * a.nx +
                          remap_index(i, a.nx, a.per[0]);
    // halo cells of this thread (fixed over the march): LDS slot and offset
    constexpr int HPT = (NH + NT - 1) / NT;  // halo cells per thread
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
                const int rh = hy / TX, c = hy % TX;
                lx = c + H;
                ly = rh < H ? rh : TY + rh;
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
        load_cell(a.uin, a.ncell, c, u);
        ok &= cons_to_prim(u, a.ph, v);
    };
    auto slope9 = [&](const T *vm, const T *v0, const T *vp, T *s) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] = limited_slope<LIM>(v0[q] - vm[q], vp[q] - v0[q]);
    };

    // Flux through one face of the plane from its two states, stored (dst
    // may be null for padding items).  Constrained transport: fc is the cell
    // whose lower face this is (its face value is the normal field) and, for
    // the tile's own faces (mine), the two transverse field fluxes go to flx.
    auto flux_item = [&](auto dir, const T *VL, const T *VR, T *dst, int fstride, long long fc,
                         bool mine) {
        constexpr int D = decltype(dir)::value;
        T F[NQ];
        if constexpr (CT) {
            face_flux<T, SOLVER, true>(VL, VR, D, a.ph, F, a.uin[(9 + D) * a.ncell + fc]);
            if (mine && a.flx) {
                a.flx[(2 * D) * a.ncell + fc] = F[D == 0 ? BY : BX];
                a.flx[(2 * D + 1) * a.ncell + fc] = F[BZ];
            }
        } else {
            face_flux<T, SOLVER>(VL, VR, D, a.ph, F);
        }
        if (dst) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) dst[q * fstride] = F[q];
        }
    };
    // owner cell (in plane zk) of the lower face of tile cell (x, y), and
    // whether that cell is in the grid
    auto face_cell = [&](long long zk, int x, int y) -> long long {
        return zk + (long long)remap_index(j0 + y, a.ny, a.per[1]) * a.nx + remap_index(i0 + x, a.nx, a.per[0]);
    };
    auto in_grid = [&](int x, int y) -> bool { return (i0 + x < a.nx) & (j0 + y < a.ny); };
    // PLM face from the LDS stencil w0..w3 (stride apart; the face lies
    // between w1 and w2): limited slopes of w1 and w2, face states, flux.
    auto face_item = [&](auto dir, const T *base, int stride, T *dst, int fstride, long long fc,
                         bool mine) {
        T VL[NQ], VR[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T *pq = base + q * PLANE;
            const T w0 = pq[0], w1 = pq[stride], w2 = pq[2 * stride], w3 = pq[3 * stride];
            const T s1 = limited_slope<LIM>(w1 - w0, w2 - w1);
            const T s2 = limited_slope<LIM>(w2 - w1, w3 - w2);
            VL[q] = w1 + T(0.5) * s1;
            VR[q] = w2 - T(0.5) * s2;
        }
        flux_item(dir, VL, VR, dst, fstride, fc, mine);
    };

    // z window.  PLM: V(k), V(k+1) and the limited slope of V(k).  WENO-Z:
    // V(k-1) .. V(k+2) and ZT, the upper face value of cell k.  Fzm is the
    // flux through face k-1/2.
    constexpr int ZW = WENO ? 4 : 2;
    constexpr int ZC = WENO ? 1 : 0;       // window slot of plane k
    T Wz[ZW][NQ], D0[NQ], ZT[NQ], Fzm[NQ];
    // A helper wave keeps its running FP64 sums of the cells its row's owner
    // left in OUTS (same column) in Fzm and its maxima of the signal speeds
    // in ZT[0..1]: registers the owners hold through the march anyway and
    // the helpers have no other use for.  Cells outside the grid count
    // nothing.
    auto helper_fold = [&]() {
        const int row = wave - TY;
        if ((i < a.nx) & (j0 + row < a.ny)) {
            T u[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                u[q] = OUTS[q * TY * TX + row * TX + tx];
                Fzm[q] += u[q];
            }
            double smx = ZT[0], cmx = ZT[1];
            ok &= cell_speeds<T, NDIM>(u, a.gamma_d, a.idx_d, smx, cmx);
            ZT[0] = smx;
            ZT[1] = cmx;
        }
    };
    if (HELP_RED && !owner) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) Fzm[q] = ZT[q] = T(0);
    }
    if (NDIM == 3 && owner) {
        T VL[NQ], VR[NQ];
        if constexpr (WENO) {
            // cell k0-1 gives the lower state of face k0-1/2, cell k0 the
            // upper one and its own upper face value
            T Vm3[NQ], Vm2[NQ];
            prim_at(zoff(k0 - 3) + own, Vm3);
            prim_at(zoff(k0 - 2) + own, Vm2);
#pragma unroll
            for (int m = 0; m < 4; ++m) prim_at(zoff(k0 - 1 + m) + own, Wz[m]);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T lo;
                wenoz_pair(Vm3[q], Vm2[q], Wz[0][q], Wz[1][q], Wz[2][q], VL[q], lo);
                wenoz_pair(Vm2[q], Wz[0][q], Wz[1][q], Wz[2][q], Wz[3][q], ZT[q], VR[q]);
            }
        } else {
            T Vm2[NQ], Vm1[NQ], Dm1[NQ];
            prim_at(zoff(k0 - 2) + own, Vm2);
            prim_at(zoff(k0 - 1) + own, Vm1);
            prim_at(zoff(k0) + own, Wz[0]);
            prim_at(zoff(k0 + 1) + own, Wz[1]);
            slope9(Vm2, Vm1, Wz[0], Dm1);
            slope9(Vm1, Wz[0], Wz[1], D0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                VL[q] = Vm1[q] + T(0.5) * Dm1[q];
                VR[q] = Wz[0][q] - T(0.5) * D0[q];
            }
        }
        if constexpr (CT)
            face_flux<T, SOLVER, true>(VL, VR, 2, a.ph, Fzm, a.uin[11 * a.ncell + zoff(k0) + own]);
        else
            face_flux<T, SOLVER>(VL, VR, 2, a.ph, Fzm);
    } else if (owner) {
        prim_at(own, Wz[ZC]);
    }

    double smax = 0.0, cmax = 0.0;
    // FP32 states: the z index of this thread's cells with the largest FP32
    // estimates of the two maxima (their FP64 speeds are taken at the end)
    float best_s = -1.0f, best_c = -1.0f;
    int k_s = -1, k_c = -1;
    double sum[HELP_RED ? 1 : NQ];
#pragma unroll
    for (int q = 0; q < (HELP_RED ? 1 : NQ); ++q) sum[q] = 0.0;

    // The stage combine's inputs at the thread's own cell are loaded at the
    // top of the plane, so that their latency hides behind the face phases,
    // where registers allow: FP32 PLM (measured 2% faster).  FP64 PLM would
    // spill (25% slower), FP32 WENO-Z runs at two waves per SIMD (3% slower),
    // and FP64 WENO-Z with its helper waves spills 2.2x more (the 416^3 step
    // 55% slower); those load them at the update.
    constexpr bool PREFETCH = (sizeof(T) == 4) && !WENO;
    auto load_combine = [&](long long c, T *cin, T *cun) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            cin[q] = a.uin[q * a.ncell + c];
            cun[q] = KIND == 1 ? T(0) : a.un[q * a.ncell + c];
        }
    };

    for (int k = k0; k < k1; ++k) {
        const long long zk = zoff(k);
        T cin[NQ], cun[NQ];
        if (PREFETCH && active) load_combine(zk + own, cin, cun);
        // the fluxes of the previous plane sit where P goes; the helpers
        // read the previous plane's results
        if ((ALIAS || HELP_RED) && k > k0) __syncthreads();
        // (a) primitives of plane k into LDS: own column and halo cell
        if (owner) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) P[q * PLANE + own_slot] = Wz[ZC][q];
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
        if constexpr (OVERLAP) {
            // the plane is in LDS: the reconstructions may start
            if (t == 0) chunk_next = 0;
            __syncthreads();
        }
        // (the previous plane's results stay until this plane's update,
        // several barriers on)
        if (HELP_RED && !owner && k > k0) helper_fold();
        // (b) z-face k+1/2 from the register window
        T Fzp[NQ], D1[NQ];
        if (NDIM == 3 && owner) {
            T Vn[NQ], VL[NQ], VR[NQ];
            prim_at(zoff(k + ZW - ZC) + own, Vn);  // PLM: V(k+2); WENO-Z: V(k+3)
            if constexpr (WENO) {
                // cell k+1: its lower face value closes face k+1/2, its upper
                // one is carried to the next plane
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    VL[q] = ZT[q];
                    wenoz_pair(Wz[0][q], Wz[1][q], Wz[2][q], Wz[3][q], Vn[q], ZT[q], VR[q]);
                }
            } else {
                slope9(Wz[0], Wz[1], Vn, D1);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    VL[q] = Wz[0][q] + T(0.5) * D0[q];
                    VR[q] = Wz[1][q] - T(0.5) * D1[q];
                }
            }
            if constexpr (CT)
                face_flux<T, SOLVER, true>(VL, VR, 2, a.ph, Fzp, a.uin[11 * a.ncell + zoff(k + 1) + own]);
            else
                face_flux<T, SOLVER>(VL, VR, 2, a.ph, Fzp);
            // slide the window by one plane
#pragma unroll
            for (int m = 0; m + 1 < ZW; ++m) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) Wz[m][q] = Wz[m + 1][q];
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) Wz[ZW - 1][q] = Vn[q];
        }
        if constexpr (!OVERLAP) __syncthreads();
        if constexpr (WENO) {
            // (c0) WENO-Z face values of every cell the plane's faces need,
            // each from the five cells centred on it: x items for cells
            // -1 .. TX of each row, y items for rows -1 .. TY of each column.
            // Direction only changes addresses, so chunks mix the two.
            auto next_chunk = [&](int ch) -> int {
                if constexpr (OVERLAP) {
                    int c = 0;
                    if (tx == 0) c = atomicAdd(&chunk_next, 1);
                    return __builtin_amdgcn_readfirstlane(c);
                } else {
                    return ch + NW;
                }
            };
            for (int ch = OVERLAP ? next_chunk(0) : wave; ch < NRCH; ch = next_chunk(ch)) {
                const int it = ch * TX + tx;
                if (it < NRX + NRY) {
                    const T *src;
                    int stride;
                    T *dst;
                    int esize;
                    if (it < NRX) {
                        const int r = it / NXE, c = it - r * NXE;
                        src = &P[(r + HY) * PX + c];
                        stride = 1;
                        dst = &EX[r * NXE + c];
                        esize = NQ * TY * NXE;
                    } else {
                        const int iy = it - NRX;
                        const int r = iy / TX, c = iy - r * TX;
                        src = &P[r * PX + c + H];
                        stride = PX;
                        dst = &EY[r * TX + c];
                        esize = NQ * NYE * TX;
                    }
                    const int qs = esize / NQ;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const T *pq = src + q * PLANE;
                        T hi, lo;
                        wenoz_pair(pq[0], pq[stride], pq[2 * stride], pq[3 * stride], pq[4 * stride], hi, lo);
                        dst[q * qs] = hi;
                        dst[esize + q * qs] = lo;
                    }
                }
            }
            __syncthreads();
            // (c1) face fluxes from the edge values: x face f of row r between
            // cells f-1 and f, y face r of column c between rows r-1 and r;
            // (the fluxes overwrite P when the LDS is aliased)
            for (int ch = wave; ch < NCHUNK; ch += NW) {
                T VL[NQ], VR[NQ];
                if (ch < NCHX) {
                    const int it = ch * TX + tx;
                    const bool valid = it < NFX;
                    const int r = valid ? it / (TX + 1) : 0;
                    const int f = valid ? it - r * (TX + 1) : 0;
                    constexpr int QS = TY * NXE;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        VL[q] = EX[q * QS + r * NXE + f];
                        VR[q] = EX[NQ * QS + q * QS + r * NXE + f + 1];
                    }
                    flux_item(std::integral_constant<int, 0>{}, VL, VR,
                              valid ? &FXs[r * (TX + 1) + f] : nullptr, TY * (TX + 1), face_cell(zk, f, r),
                              valid && f < TX && in_grid(f, r));
                } else {
                    const int it = (ch - NCHX) * TX + tx;
                    const int r = it / TX, c = it - r * TX;
                    constexpr int QS = NYE * TX;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        VL[q] = EY[q * QS + r * TX + c];
                        VR[q] = EY[NQ * QS + q * QS + (r + 1) * TX + c];
                    }
                    flux_item(std::integral_constant<int, 1>{}, VL, VR, &FYs[r * TX + c], (TY + 1) * TX,
                              face_cell(zk, c, r), r < TY && in_grid(c, r));
                }
            }
        } else {
            // (c) x- and y-faces of the plane.  Items go out in 64-wide chunks,
            // one chunk per wave at a time; x items are padded to whole chunks so
            // every chunk is a single direction and the solver is inlined with a
            // compile-time frame.
            for (int ch = wave; ch < NCHUNK; ch += NW) {
                if (ch < NCHX) {
                    const int it = ch * TX + tx;
                    const bool valid = it < NFX;
                    const int r = valid ? it / (TX + 1) : 0;
                    const int f = valid ? it - r * (TX + 1) : 0;
                    // cells f-2 .. f+1 of row r
                    face_item(std::integral_constant<int, 0>{}, &P[(r + HY) * PX + f], 1,
                              valid ? &FXs[r * (TX + 1) + f] : nullptr, TY * (TX + 1), face_cell(zk, f, r),
                              valid && f < TX && in_grid(f, r));
                } else {
                    const int it = (ch - NCHX) * TX + tx;
                    const int r = it / TX, c = it - r * TX;
                    // rows r-2 .. r+1 of column c
                    face_item(std::integral_constant<int, 1>{}, &P[r * PX + c + H], PX, &FYs[r * TX + c],
                              (TY + 1) * TX, face_cell(zk, c, r), r < TY && in_grid(c, r));
                }
            }
        }
        __syncthreads();
        // (d) divergence and stage combine
        if (active) {
            const long long c = zk + own;
            T L[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const T *fx = &FXs[q * TY * (TX + 1) + ty * (TX + 1) + tx];
                T l = (fx[0] - fx[1]) * a.idx[0];
                if (NDIM >= 2) {
                    const T *fy = &FYs[q * (TY + 1) * TX + ty * TX + tx];
                    l += (fy[0] - fy[TX]) * a.idx[1];
                }
                if (NDIM == 3) l += (Fzm[q] - Fzp[q]) * a.idx[2];
                L[q] = l;
            }
            if (!PREFETCH) load_combine(c, cin, cun);
            T out[NQ];
            if (KIND == 1) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[q] = cin[q] + a.dt * L[q];
            } else if (KIND == 2) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[q] = T(0.5) * ((cun[q] + cin[q]) + a.dt * L[q]);
            } else if (KIND == 3) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[q] = T(0.75) * cun[q] + T(0.25) * (cin[q] + a.dt * L[q]);
            } else {
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[q] = cun[q] * T(1.0 / 3.0) + T(2.0 / 3.0) * (cin[q] + a.dt * L[q]);
            }
            if (LAST) out[PSI] *= a.damp;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                // constrained transport: the face update writes the cell field
                if (CT && q >= BX && q <= BZ) continue;
                __builtin_nontemporal_store(out[q], &a.uout[q * a.ncell + c]);  // not read again here
            }
            if (CT && a.flx) {
                // transverse field fluxes of this cell's lower z face
                a.flx[4 * a.ncell + c] = Fzm[BX];
                a.flx[5 * a.ncell + c] = Fzm[BY];
            }
            if constexpr (HELP_RED) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) OUTS[q * TY * TX + t] = out[q];
            } else if (LAST) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) sum[q] += (double)out[q];
                if constexpr (sizeof(T) == 8) {
                    ok &= cell_speeds<T, NDIM>(out, a.gamma_d, a.idx_d, smax, cmax);
                } else {
                    float ls, lc;
                    ok &= cell_speeds_f32<NDIM>(out, a.ph.gamma, a.idx, ls, lc);
                    k_s = ls > best_s ? k : k_s;
                    best_s = __builtin_fmaxf(best_s, ls);
                    k_c = lc > best_c ? k : k_c;
                    best_c = __builtin_fmaxf(best_c, lc);
                }
            }
        }
        if (NDIM == 3 && owner) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                Fzm[q] = Fzp[q];
                if constexpr (!WENO) D0[q] = D1[q];
            }
        }
    }

    if constexpr (LAST && sizeof(T) == 4) {
        // FP64 speeds of the selected cells, re-read from this thread's own
        // output (it stored them above)
        if (k_s >= 0) {
            T u[NQ];
            load_cell(a.uout, a.ncell, zoff(k_s) + own, u);
            ok &= cell_speeds<T, NDIM>(u, a.gamma_d, a.idx_d, smax, cmax);
        }
        if (k_c >= 0 && k_c != k_s) {
            T u[NQ];
            load_cell(a.uout, a.ncell, zoff(k_c) + own, u);
            ok &= cell_speeds<T, NDIM>(u, a.gamma_d, a.idx_d, smax, cmax);
        }
    }
    if (LAST) {
        // block reduction of the partials in a fixed order
        __syncthreads();
        double *red = reinterpret_cast<double *>(P);  // LDS reuse, TY * NPART doubles
        double vals[NPART];
        if constexpr (HELP_RED) {
            if (!owner) helper_fold();  // the chunk's last plane
            vals[0] = wave_max(ZT[0]);
            vals[1] = wave_max(ZT[1]);
#pragma unroll
            for (int q = 0; q < NQ; ++q) vals[2 + q] = wave_sum(Fzm[q]);
        } else {
            vals[0] = wave_max(smax);
            vals[1] = wave_max(cmax);
#pragma unroll
            for (int q = 0; q < NQ; ++q) vals[2 + q] = wave_sum(sum[q]);
        }
        // the row's reducing wave: its helper, or its owner
        if (tx == 0 && (HELP_RED ? !owner : owner)) {
            const int row = HELP_RED ? wave - TY : ty;
#pragma unroll
            for (int e = 0; e < NPART; ++e) red[row * NPART + e] = vals[e];
        }
        __syncthreads();
        if (t < NPART) {
            double r = red[t];
            for (int w = 1; w < TY; ++w) {
                const double x = red[w * NPART + t];
                r = t < 2 ? __builtin_fmax(r, x) : r + x;
            }
            a.part[(long long)t * a.nblocks + lb] = r;
        }
    }
    if (!ok) atomicOr(a.flag, 1);
}

} // namespace mhd
