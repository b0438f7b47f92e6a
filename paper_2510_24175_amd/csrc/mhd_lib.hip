// Host side of the C ABI declared in include/mhd.h: argument validation,
// context and scratch management, kernel dispatch on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mhd.h"
#include "mhd_adjoint.hpp"
#include "mhd_ct.hpp"
#include "mhd_reduce.hpp"
#include "mhd_stage.hpp"

using namespace mhd;

struct mhd_ctx {
    mhd_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    long long n[3] = {1, 1, 1};
    long long ncell = 0;
    size_t elem = 4;             // bytes per state element
    int ns = NQ;                 // state components (12 with constrained transport)
    void *u1_scratch = nullptr;  // stage-1 state when the caller passes none
    void *u2_scratch = nullptr;  // SSP-RK3 stage-2 state
    void *ct_flx = nullptr;      // constrained transport: [6] transverse field fluxes (mean EMF)
                                 // or cell velocities and fast speeds (upwind EMF)
    void *ct_emf = nullptr;      // constrained transport: [3] edge EMFs
    double *part = nullptr;      // NPART x part_cap block partials
    int part_cap = 0;
    double *result = nullptr;    // device NPART doubles: reductions of the last mhd_step output
    double *cfl_result = nullptr; // device NPART doubles: the last mhd_cfl_dt reduction
    int *flag = nullptr;         // device non-physical flag
    double *host_res = nullptr;  // pinned NPART doubles + flag word
    double *lam1 = nullptr;      // adjoint: FP64 stage cotangent
    bool have_step = false;
    double cell_volume = 1.0;
    double dx[3] = {1, 1, 1};
    std::vector<hipEvent_t> events; // 4 per timed step
    int timed_cap = 0, timed_steps = 0;
    // a transient context of mhd_step_noalloc: its buffers are the static
    // scratch, each step first clears the flag, and errors keep no text
    bool no_alloc = false;
    std::string err;
};

namespace {

constexpr int CFL_MAX_BLOCKS = 4096;
// rows of an upwind EMF tile (TX x 8 columns: 124 KB of LDS in FP64, one
// workgroup of 8 waves per compute unit; 62 KB in FP32, two)
template <typename T> constexpr int ct_emf_rows() { return 8; }

mhd_status fail(mhd_ctx *ctx, mhd_status st, const char *msg)
{
    if (ctx && !ctx->no_alloc) ctx->err = msg;
    return st;
}

mhd_status fail_hip(mhd_ctx *ctx, const char *what, hipError_t e)
{
    if (ctx && !ctx->no_alloc) ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return MHD_ERR_HIP;
}

#define HIP_TRY(ctx, call)                                \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return fail_hip((ctx), #call, e_); \
    } while (0)

// Stage tile rows per workgroup (one wave per row; two with FP64 WENO-Z, see
// stage_row_waves).  FP32 PLM: 4 rows, three
// workgroups (12 waves) per compute unit at the 168-VGPR budget; measured
// faster than 6 rows (two workgroups of 6 waves) by a third and than 8 rows
// (one workgroup of 8 waves) by 13%; an 8-row first stage at two workgroups
// of 8 waves (125 registers, a tenth fewer face items and half the halo
// conversions per cell) measured 2% slower, and a 6-row last stage at two
// workgroups of 6 waves (the same 12 waves per compute unit; 6 waves do not
// spread evenly over its 4 SIMDs) 60% slower.  FP32 WENO-Z: 8 rows, one workgroup of
// 8 waves and 155 KB of LDS per compute unit; the three-cell y halo costs
// half as much per cell as with 4 rows (measured 9% faster).  FP64 (register
// bound, WENO-Z at 140 KB of LDS): 4 rows.  1D: 1 row.
template <typename T, int LIM, int NDIM> constexpr int tile_rows()
{
    return NDIM == 1 ? 1 : (sizeof(T) == 4 && LIM == LIM_WENOZ ? 8 : 4);
}

struct Launch {
    int tiles_x, tiles_y, chunks, kz, nblocks;
};

// min_blocks: the grid size below which z chunks are shortened (each chunk
// pays a warm-up of a few planes); the forward stages run two or three
// workgroups per compute unit and want 2048, the adjoint runs one and
// wants 256: its warm-up is three full planes of z work, and one round of
// longer chunks measured 4% faster at 128^3 than two rounds of half-length
// ones.
Launch plan_stage(const mhd_ctx *ctx, int ty, long long min_blocks = 2048)
{
    Launch L;
    L.tiles_x = (int)((ctx->n[0] + TX - 1) / TX);
    L.tiles_y = (int)((ctx->n[1] + ty - 1) / ty);
    const long long tiles = (long long)L.tiles_x * L.tiles_y;
    int kz = 1;
    if (ctx->cfg.ndim == 3) {
        // long z chunks amortise the warm-up planes; shorter chunks when
        // the grid would otherwise leave compute units idle.  FP64 WENO-Z
        // (one 4-wave workgroup per compute unit) starts at 32 planes:
        // measured 7% faster at 416^3 and 10% with constrained transport at
        // 352^3 than 64; FP32 constrained transport at 16 planes, 2% faster
        // at 352^3 (FP32 GLM and PLM: no gain)
        const bool f64 = ctx->cfg.dtype == MHD_F64;
        kz = (f64 && ctx->cfg.limiter == MHD_WENOZ) ? 32 : ((!f64 && ctx->cfg.ct) ? 16 : 64);
        while (kz > 4 && tiles * ((ctx->n[2] + kz - 1) / kz) < min_blocks) kz >>= 1;
    }
    L.kz = kz;
    L.chunks = (int)((ctx->n[2] + kz - 1) / kz);
    L.nblocks = (int)(tiles * L.chunks);
    return L;
}

template <typename T> Phys<T> make_phys(const mhd_ctx *ctx, double ch)
{
    Phys<T> p;
    const double g = ctx->cfg.gamma;
    p.gamma = (T)g;
    p.gm1 = (T)(g - 1.0);
    p.inv_gm1 = (T)(1.0 / (g - 1.0));
    p.glm = ctx->cfg.glm ? 1 : 0;
    p.ch = (T)(p.glm ? ch : 0.0);
    p.ch2 = (T)(p.glm ? ch * ch : 0.0);
    p.half_ich = (T)(p.glm ? 0.5 / ch : 0.0);
    return p;
}

template <typename T, int SOLVER, int LIM, int NDIM>
mhd_status launch_step(mhd_ctx *ctx, const T *un, T *unext, T *u1, double dt, double ch, double damp)
{
    const bool rk3 = ctx->cfg.time_order == 3;
    constexpr int TY = tile_rows<T, LIM, NDIM>();
    constexpr int NTH = TX * TY * stage_row_waves<T, LIM>();
    const Launch L = plan_stage(ctx, TY);
    if (L.nblocks > ctx->part_cap) return fail(ctx, MHD_ERR_ARG, "grid too large for partials buffer");
    if (ctx->no_alloc) {
        // the static scratch keeps the last call's flag: this call reports
        // only what its own kernels see
        hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, ctx->stream, ctx->flag);
        HIP_TRY(ctx, hipGetLastError());
    }
    StageArgs<T> a;
    a.part = ctx->part;
    a.flag = ctx->flag;
    a.nx = (int)ctx->n[0];
    a.ny = (int)ctx->n[1];
    a.nz = (int)ctx->n[2];
    a.nxy = ctx->n[0] * ctx->n[1];
    a.ncell = ctx->ncell;
    for (int d = 0; d < 3; ++d) {
        a.per[d] = ctx->cfg.bc[d][0] == MHD_PERIODIC;
        a.idx[d] = (T)(1.0 / ctx->dx[d]);
        a.idx_d[d] = 1.0 / ctx->dx[d];
    }
    a.kz = L.kz;
    a.tiles_x = L.tiles_x;
    a.tiles_y = L.tiles_y;
    a.chunks = L.chunks;
    a.nblocks = L.nblocks;
    a.dt = (T)dt;
    a.damp = (T)damp;
    a.gamma_d = ctx->cfg.gamma;
    a.ph = make_phys<T>(ctx, ch);

    hipEvent_t *ev = nullptr;
    if (ctx->timed_steps < ctx->timed_cap) ev = &ctx->events[4 * ctx->timed_steps++];
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
    a.uin = un;
    a.un = un;
    a.uout = u1;
    hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, NDIM, 1, TY>), dim3(L.nblocks), dim3(NTH), 0,
                       ctx->stream, a);
    HIP_TRY(ctx, hipGetLastError());
    if (rk3) {
        T *u2 = (T *)ctx->u2_scratch;
        a.uin = u1;
        a.uout = u2;
        hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, NDIM, 3, TY>), dim3(L.nblocks), dim3(NTH), 0,
                           ctx->stream, a);
        HIP_TRY(ctx, hipGetLastError());
        if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
        a.uin = u2;
        a.uout = unext;
        hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, NDIM, 4, TY>), dim3(L.nblocks), dim3(NTH), 0,
                           ctx->stream, a);
        HIP_TRY(ctx, hipGetLastError());
    } else {
        if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
        a.uin = u1;
        a.uout = unext;
        hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, NDIM, 2, TY>), dim3(L.nblocks), dim3(NTH), 0,
                           ctx->stream, a);
        HIP_TRY(ctx, hipGetLastError());
    }
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream,
                       (const double *)ctx->part, L.nblocks, ctx->result);
    HIP_TRY(ctx, hipGetLastError());
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[3], ctx->stream));
    return MHD_OK;
}

// Constrained transport step (3D, periodic): per stage the stage kernel
// (fluxes with the faces' normal field, with the mean EMF the transverse
// field fluxes to scratch, cell update of rho, m, E), the edge EMFs (mean of
// those fluxes, or upwind from the stage's input state), and the face update
// with the cell field; the last face update reduces the CFL maxima and sums.
template <typename T, int SOLVER, int LIM>
mhd_status launch_step_ct(mhd_ctx *ctx, const T *un, T *unext, T *u1, double dt, double ch, double damp)
{
    constexpr int TY = tile_rows<T, LIM, 3>();
    constexpr int NTH = TX * TY * stage_row_waves<T, LIM>();
    const bool rk3 = ctx->cfg.time_order == 3;
    const Launch L = plan_stage(ctx, TY);
    StageArgs<T> a;
    a.part = ctx->part;
    a.flag = ctx->flag;
    a.flx = ctx->cfg.ct == 1 ? (T *)ctx->ct_flx : nullptr;  // the upwind EMF takes no fluxes
    a.nx = (int)ctx->n[0];
    a.ny = (int)ctx->n[1];
    a.nz = (int)ctx->n[2];
    a.nxy = ctx->n[0] * ctx->n[1];
    a.ncell = ctx->ncell;
    for (int d = 0; d < 3; ++d) {
        a.per[d] = 1;
        a.idx[d] = (T)(1.0 / ctx->dx[d]);
        a.idx_d[d] = 1.0 / ctx->dx[d];
    }
    a.kz = L.kz;
    a.tiles_x = L.tiles_x;
    a.tiles_y = L.tiles_y;
    a.chunks = L.chunks;
    a.nblocks = L.nblocks;
    a.dt = (T)dt;
    a.damp = (T)damp;
    a.gamma_d = ctx->cfg.gamma;
    a.ph = make_phys<T>(ctx, ch);
    CTArgs<T> c;
    c.un = un;
    c.flx = (const T *)ctx->ct_flx;
    c.emf = (T *)ctx->ct_emf;
    c.part = ctx->part;
    c.flag = ctx->flag;
    c.nx = a.nx;
    c.ny = a.ny;
    c.nz = a.nz;
    c.ncell = ctx->ncell;
    c.dt = (T)dt;
    for (int d = 0; d < 3; ++d) {
        c.idx[d] = a.idx[d];
        c.idx_d[d] = a.idx_d[d];
    }
    c.gamma_d = ctx->cfg.gamma;
    const int nb = (int)std::min<long long>((ctx->ncell + RED_THREADS - 1) / RED_THREADS, CFL_MAX_BLOCKS);
    c.nblocks = nb;
    // upwind EMF tiling: z chunks of up to 32 planes, shortened until the
    // pass has eight workgroups per compute unit
    CTTiles ug;
    ug.tiles_x = (a.nx + TX - 1) / TX;
    ug.tiles_y = (a.ny + ct_emf_rows<T>() - 1) / ct_emf_rows<T>();
    ug.kz = 32;
    while (ug.kz > 4 && (long long)ug.tiles_x * ug.tiles_y * ((a.nz + ug.kz - 1) / ug.kz) < 8 * 256) ug.kz >>= 1;
    ug.nblocks = ug.tiles_x * ug.tiles_y * ((a.nz + ug.kz - 1) / ug.kz);

    hipEvent_t *ev = nullptr;
    if (ctx->timed_steps < ctx->timed_cap) ev = &ctx->events[4 * ctx->timed_steps++];
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
    // one stage: uin -> uout with stage kind KIND
    auto stage = [&](auto kind, const T *uin, T *uout) -> mhd_status {
        constexpr int KIND = decltype(kind)::value;
        a.uin = uin;
        a.un = un;
        a.uout = uout;
        hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, 3, KIND, TY, true>), dim3(L.nblocks), dim3(NTH), 0,
                           ctx->stream, a);
        HIP_TRY(ctx, hipGetLastError());
        c.uin = uin;
        c.uout = uout;
        if (ctx->cfg.ct == 2)
            hipLaunchKernelGGL((ct_emf_upwind_kernel<T, ct_emf_rows<T>()>), dim3(ug.nblocks), dim3(TX * ct_emf_rows<T>()), 0,
                               ctx->stream, c, ug);
        else
            hipLaunchKernelGGL(ct_emf_kernel<T>, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, c);
        HIP_TRY(ctx, hipGetLastError());
        hipLaunchKernelGGL((ct_face_kernel<T, KIND, last_stage(KIND)>), dim3(nb), dim3(RED_THREADS), 0,
                           ctx->stream, c);
        HIP_TRY(ctx, hipGetLastError());
        return MHD_OK;
    };
    mhd_status st = stage(std::integral_constant<int, 1>{}, un, u1);
    if (st != MHD_OK) return st;
    if (rk3) {
        T *u2 = (T *)ctx->u2_scratch;
        st = stage(std::integral_constant<int, 3>{}, u1, u2);
        if (st != MHD_OK) return st;
        if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
        st = stage(std::integral_constant<int, 4>{}, u2, unext);
    } else {
        if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
        st = stage(std::integral_constant<int, 2>{}, u1, unext);
    }
    if (st != MHD_OK) return st;
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream,
                       (const double *)ctx->part, nb, ctx->result);
    HIP_TRY(ctx, hipGetLastError());
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[3], ctx->stream));
    return MHD_OK;
}

template <typename T, int SOLVER, int LIM>
mhd_status launch_step_nd(mhd_ctx *ctx, const void *un, void *unext, void *u1, double dt, double ch,
                          double damp)
{
    const T *a = (const T *)un;
    T *b = (T *)unext, *c = (T *)u1;
    if (ctx->cfg.ct) return launch_step_ct<T, SOLVER, LIM>(ctx, a, b, c, dt, ch, damp);
    switch (ctx->cfg.ndim) {
    case 1: return launch_step<T, SOLVER, LIM, 1>(ctx, a, b, c, dt, ch, damp);
    case 2: return launch_step<T, SOLVER, LIM, 2>(ctx, a, b, c, dt, ch, damp);
    default: return launch_step<T, SOLVER, LIM, 3>(ctx, a, b, c, dt, ch, damp);
    }
}

// Adjoint tile rows per workgroup: FP32 8 rows (one 512-thread workgroup
// per compute unit, 124.6 KB of LDS, y-face halo overhead 3/8); FP64 4 rows
// (153.5 KB of LDS); 1D: 1 row.
template <typename T, int NDIM> constexpr int adj_tile_rows()
{
    return NDIM == 1 ? 1 : (sizeof(T) == 4 ? 8 : 4);
}

template <typename T, int SOLVER, int LIM, int NDIM, int PASS>
mhd_status launch_adj_stage(mhd_ctx *ctx, const T *U, const double *lamp, const double *lam1,
                            double *out, double dt, double ch, double damp)
{
    constexpr int TY = adj_tile_rows<T, NDIM>();
    const Launch L = plan_stage(ctx, TY, 256);
    AdjStageArgs<T> a;
    a.U = U;
    a.lamp = lamp;
    a.lam1 = lam1;
    a.out = out;
    a.flag = ctx->flag;
    a.nx = (int)ctx->n[0];
    a.ny = (int)ctx->n[1];
    a.nz = (int)ctx->n[2];
    a.nxy = ctx->n[0] * ctx->n[1];
    a.ncell = ctx->ncell;
    for (int d = 0; d < 3; ++d) {
        a.per[d] = ctx->cfg.bc[d][0] == MHD_PERIODIC;
        a.idx[d] = 1.0 / ctx->dx[d];
    }
    a.kz = L.kz;
    a.tiles_x = L.tiles_x;
    a.tiles_y = L.tiles_y;
    a.chunks = L.chunks;
    a.nblocks = L.nblocks;
    a.dt = dt;
    a.damp = damp;
    a.gm1 = ctx->cfg.gamma - 1.0;
    a.ph = make_phys<T>(ctx, ch);
    hipLaunchKernelGGL((adj_stage_kernel<T, SOLVER, LIM, NDIM, PASS, TY>), dim3(L.nblocks), dim3(TX * TY), 0,
                       ctx->stream, a);
    HIP_TRY(ctx, hipGetLastError());
    return MHD_OK;
}

template <typename T, int SOLVER, int LIM, int NDIM>
mhd_status launch_adjoint(mhd_ctx *ctx, const T *un, const T *u1, const double *lamp, double *lamn,
                          double dt, double ch, double damp)
{
    if (!u1) {
        // recompute the stage-1 state into scratch with the forward kernel
        constexpr int TY = tile_rows<T, LIM, NDIM>();
        constexpr int NTH = TX * TY * stage_row_waves<T, LIM>();
        const Launch L = plan_stage(ctx, TY);
        StageArgs<T> a;
        a.part = ctx->part;
        a.flag = ctx->flag;
        a.nx = (int)ctx->n[0];
        a.ny = (int)ctx->n[1];
        a.nz = (int)ctx->n[2];
        a.nxy = ctx->n[0] * ctx->n[1];
        a.ncell = ctx->ncell;
        for (int d = 0; d < 3; ++d) {
            a.per[d] = ctx->cfg.bc[d][0] == MHD_PERIODIC;
            a.idx[d] = (T)(1.0 / ctx->dx[d]);
                a.idx_d[d] = 1.0 / ctx->dx[d];
        }
        a.kz = L.kz;
        a.tiles_x = L.tiles_x;
        a.tiles_y = L.tiles_y;
        a.chunks = L.chunks;
        a.nblocks = L.nblocks;
        a.dt = (T)dt;
        a.damp = (T)damp;
        a.gamma_d = ctx->cfg.gamma;
        a.ph = make_phys<T>(ctx, ch);
        a.uin = un;
        a.un = un;
        a.uout = (T *)ctx->u1_scratch;
        hipLaunchKernelGGL((stage_kernel<T, SOLVER, LIM, NDIM, 1, TY>), dim3(L.nblocks), dim3(NTH), 0,
                           ctx->stream, a);
        HIP_TRY(ctx, hipGetLastError());
        u1 = (const T *)ctx->u1_scratch;
    }
    // stage-2 pass: lam1 = mu/2 + (dt/2) J_L(U1)^T mu, mu = D lam'
    mhd_status st = launch_adj_stage<T, SOLVER, LIM, NDIM, 2>(ctx, u1, lamp, nullptr, ctx->lam1, dt, ch, damp);
    if (st != MHD_OK) return st;
    // stage-1 pass: lamn = mu/2 + lam1 + dt J_L(Un)^T lam1
    st = launch_adj_stage<T, SOLVER, LIM, NDIM, 1>(ctx, un, lamp, ctx->lam1, lamn, dt, ch, damp);
    if (st != MHD_OK) return st;
    return MHD_OK;
}

template <typename T, int SOLVER, int LIM>
mhd_status launch_adjoint_nd(mhd_ctx *ctx, const void *un, const void *u1, const double *lamp,
                             double *lamn, double dt, double ch, double damp)
{
    const T *a = (const T *)un, *b = (const T *)u1;
    switch (ctx->cfg.ndim) {
    case 1: return launch_adjoint<T, SOLVER, LIM, 1>(ctx, a, b, lamp, lamn, dt, ch, damp);
    case 2: return launch_adjoint<T, SOLVER, LIM, 2>(ctx, a, b, lamp, lamn, dt, ch, damp);
    default: return launch_adjoint<T, SOLVER, LIM, 3>(ctx, a, b, lamp, lamn, dt, ch, damp);
    }
}

// Compile-time scheme: state type, Riemann solver, limiter.
template <typename T_, int SOLVER_, int LIM_> struct Scheme {
    using T = T_;
    static constexpr int SOLVER = SOLVER_;
    static constexpr int LIM = LIM_;
};

template <typename T, int SOLVER, typename Fn> mhd_status with_recon(const mhd_ctx *ctx, Fn &&fn)
{
    switch (ctx->cfg.limiter) {
    case MHD_MC: return fn(Scheme<T, SOLVER, LIM_MC>{});
    case MHD_WENOZ: return fn(Scheme<T, SOLVER, LIM_WENOZ>{});
    default: return fn(Scheme<T, SOLVER, LIM_MINMOD>{});
    }
}

template <typename Fn> mhd_status with_scheme(const mhd_ctx *ctx, Fn &&fn)
{
    const bool hlld = ctx->cfg.riemann == MHD_HLLD;
    if (ctx->cfg.dtype == MHD_F32)
        return hlld ? with_recon<float, SOLVER_HLLD>(ctx, fn) : with_recon<float, SOLVER_HLL>(ctx, fn);
    return hlld ? with_recon<double, SOLVER_HLLD>(ctx, fn) : with_recon<double, SOLVER_HLL>(ctx, fn);
}

template <typename T>
mhd_status launch_cfl(mhd_ctx *ctx, const T *U)
{
    const int nb = (int)std::min<long long>((ctx->ncell + RED_THREADS - 1) / RED_THREADS, CFL_MAX_BLOCKS);
    const double i0 = 1.0 / ctx->dx[0], i1 = 1.0 / ctx->dx[1], i2 = 1.0 / ctx->dx[2];
    switch (ctx->cfg.ndim) {
    case 1:
        hipLaunchKernelGGL((cfl_kernel<T, 1>), dim3(nb), dim3(RED_THREADS), 0, ctx->stream, U,
                           ctx->ncell, ctx->cfg.gamma, i0, i1, i2, ctx->part, nb, ctx->flag);
        break;
    case 2:
        hipLaunchKernelGGL((cfl_kernel<T, 2>), dim3(nb), dim3(RED_THREADS), 0, ctx->stream, U,
                           ctx->ncell, ctx->cfg.gamma, i0, i1, i2, ctx->part, nb, ctx->flag);
        break;
    default:
        hipLaunchKernelGGL((cfl_kernel<T, 3>), dim3(nb), dim3(RED_THREADS), 0, ctx->stream, U,
                           ctx->ncell, ctx->cfg.gamma, i0, i1, i2, ctx->part, nb, ctx->flag);
    }
    HIP_TRY(ctx, hipGetLastError());
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream,
                       (const double *)ctx->part, nb, ctx->cfl_result);
    HIP_TRY(ctx, hipGetLastError());
    return MHD_OK;
}

// Copy the result words of one reduction (the step's or the standalone
// CFL's) back, wait, and report (and clear) the flag.
mhd_status sync_results(mhd_ctx *ctx, const double *result)
{
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_res, result, NPART * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_res + NPART, ctx->flag, sizeof(int), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    int flag;
    std::memcpy(&flag, ctx->host_res + NPART, sizeof(int));
    if (flag) {
        HIP_TRY(ctx, hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return fail(ctx, MHD_ERR_NONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or non-finite)");
    }
    return MHD_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Validates a configuration: MHD_ERR_ARG for invalid fields,
// MHD_ERR_UNSUPPORTED for the adjoint of WENO-Z or SSP-RK3 (not built).
mhd_status check_config(const mhd_config *c, const char *&why)
{
    if (!c) return why = "config is NULL", MHD_ERR_ARG;
    if (c->ndim < 1 || c->ndim > 3) return why = "ndim must be 1, 2 or 3", MHD_ERR_ARG;
    if (c->dtype != MHD_F32 && c->dtype != MHD_F64) return why = "bad dtype", MHD_ERR_ARG;
    if (c->riemann != MHD_HLL && c->riemann != MHD_HLLD) return why = "bad riemann", MHD_ERR_ARG;
    if (c->limiter != MHD_MINMOD && c->limiter != MHD_MC && c->limiter != MHD_WENOZ)
        return why = "bad limiter", MHD_ERR_ARG;
    if (c->time_order != 2 && c->time_order != 3) return why = "time_order must be 2 or 3", MHD_ERR_ARG;
    if (c->ct < 0 || c->ct > 2) return why = "ct must be 0, 1 or 2", MHD_ERR_ARG;
    if (c->glm != 0 && c->glm != 1) return why = "glm must be 0 or 1", MHD_ERR_ARG;
    if ((c->flags & ~MHD_FLAG_ADJOINT) != 0) return why = "unknown flag bits", MHD_ERR_ARG;
    long long cells = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < c->ndim) {
            if (c->n[d] < 2) return why = "active axes need n >= 2", MHD_ERR_ARG;
            if (!(c->hi[d] > c->lo[d]) || !std::isfinite(c->hi[d] - c->lo[d]))
                return why = "hi must exceed lo on active axes", MHD_ERR_ARG;
            for (int s = 0; s < 2; ++s)
                if (c->bc[d][s] != MHD_PERIODIC && c->bc[d][s] != MHD_OUTFLOW)
                    return why = "bad boundary kind", MHD_ERR_ARG;
            if ((c->bc[d][0] == MHD_PERIODIC) != (c->bc[d][1] == MHD_PERIODIC))
                return why = "periodic must apply to both faces of an axis", MHD_ERR_ARG;
        } else if (c->n[d] != 1) {
            return why = "inactive axes need n = 1", MHD_ERR_ARG;
        }
        if (c->n[d] > (1LL << 30)) return why = "axis too long", MHD_ERR_ARG;
        cells *= c->n[d];
    }
    if (cells > (1LL << 40)) return why = "grid too large", MHD_ERR_ARG;
    if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) return why = "gamma must exceed 1", MHD_ERR_ARG;
    if (!(c->cfl > 0.0 && c->cfl <= 1.0)) return why = "cfl must be in (0, 1]", MHD_ERR_ARG;
    if (!(c->glm_alpha >= 0.0) || !std::isfinite(c->glm_alpha))
        return why = "glm_alpha must be >= 0", MHD_ERR_ARG;
    if ((c->flags & MHD_FLAG_ADJOINT) && (c->limiter == MHD_WENOZ || c->time_order != 2 || c->ct))
        return why = "the adjoint covers PLM with SSP-RK2 and GLM only", MHD_ERR_UNSUPPORTED;
    if (c->ct) {
        if (c->glm) return why = "constrained transport replaces GLM (glm must be 0)", MHD_ERR_ARG;
        if (c->ndim != 3) return why = "constrained transport is three-dimensional", MHD_ERR_UNSUPPORTED;
        for (int d = 0; d < 3; ++d)
            if (c->bc[d][0] != MHD_PERIODIC)
                return why = "constrained transport needs periodic axes", MHD_ERR_UNSUPPORTED;
        if (c->n[0] * c->n[1] * c->n[2] >= (1LL << 31))
            return why = "constrained transport needs fewer than 2^31 cells", MHD_ERR_ARG;
    }
    return MHD_OK;
}

void destroy_events(mhd_ctx *ctx)
{
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    ctx->events.clear();
    ctx->timed_cap = ctx->timed_steps = 0;
}

// Static scratch of mhd_step_noalloc, one copy per device, held until the
// process ends: the per-block partials of the last stage (NPART x
// NOALLOC_MAX_BLOCKS doubles), the final reduction (NPART doubles) and the
// non-physical flag.  Host code never uses the symbol itself (in host code
// it is a stand-in, not a device address): the device address is looked up
// once per device with hipGetSymbolAddress and kept in noalloc_ptr.
constexpr int NOALLOC_MAX_BLOCKS = 16384;
constexpr size_t NOALLOC_PART_BYTES = (size_t)NPART * NOALLOC_MAX_BLOCKS * sizeof(double);
constexpr size_t NOALLOC_RESULT_OFF = NOALLOC_PART_BYTES;
constexpr size_t NOALLOC_FLAG_OFF = NOALLOC_RESULT_OFF + 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_FLAG_OFF + 256;
static_assert(NPART * sizeof(double) <= 256, "result words fit their slot");
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[NOALLOC_MAX_DEVICES];  // device address of scratch per device
bool noalloc_gfx950[NOALLOC_MAX_DEVICES];

// Device address of the static scratch on the current device (looked up on
// the first call per device, with that device current); MHD_ERR_NO_DEVICE
// when the device is not a gfx950.
mhd_status noalloc_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return MHD_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MHD_ERR_NO_DEVICE;
        noalloc_gfx950[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        if (!noalloc_gfx950[dev]) return MHD_ERR_NO_DEVICE;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MHD_ERR_HIP;
        noalloc_ptr[dev] = p;
    }
    if (!noalloc_gfx950[dev]) return MHD_ERR_NO_DEVICE;
    *out = (unsigned char *)noalloc_ptr[dev];
    return MHD_OK;
}

void free_ctx(mhd_ctx *ctx)
{
    destroy_events(ctx);
    if (ctx->u1_scratch) (void)hipFree(ctx->u1_scratch);
    if (ctx->u2_scratch) (void)hipFree(ctx->u2_scratch);
    if (ctx->ct_flx) (void)hipFree(ctx->ct_flx);
    if (ctx->ct_emf) (void)hipFree(ctx->ct_emf);
    if (ctx->part) (void)hipFree(ctx->part);
    if (ctx->result) (void)hipFree(ctx->result);
    if (ctx->cfl_result) (void)hipFree(ctx->cfl_result);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->host_res) (void)hipHostFree(ctx->host_res);
    if (ctx->lam1) (void)hipFree(ctx->lam1);
    delete ctx;
}

} // namespace

extern "C" {

const char *mhd_status_string(mhd_status st)
{
    switch (st) {
    case MHD_OK: return "ok";
    case MHD_ERR_ARG: return "invalid argument";
    case MHD_ERR_NO_DEVICE: return "no usable gfx950 device";
    case MHD_ERR_HIP: return "HIP runtime error";
    case MHD_ERR_NONPHYSICAL: return "non-physical state";
    case MHD_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

mhd_status mhd_timing_start(mhd_ctx *ctx, int32_t capacity)
{
    if (!ctx) return MHD_ERR_ARG;
    if (capacity < 1 || capacity > (1 << 20)) return fail(ctx, MHD_ERR_ARG, "capacity out of range");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    destroy_events(ctx);
    ctx->events.resize(4 * (size_t)capacity, nullptr);
    for (auto &e : ctx->events) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            e = nullptr;
            destroy_events(ctx);
            return fail_hip(ctx, "hipEventCreate", r);
        }
    }
    ctx->timed_cap = capacity;
    ctx->timed_steps = 0;
    return MHD_OK;
}

mhd_status mhd_timing_stop(mhd_ctx *ctx, double out[4])
{
    if (!ctx) return MHD_ERR_ARG;
    if (!out) return fail(ctx, MHD_ERR_ARG, "null buffer");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    out[0] = ctx->timed_steps;
    out[1] = out[2] = out[3] = 0.0;
    for (int s = 0; s < ctx->timed_steps; ++s) {
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->events[4 * s + k], ctx->events[4 * s + k + 1]));
            out[1 + k] += ms;
        }
    }
    destroy_events(ctx);
    return MHD_OK;
}

const char *mhd_last_error(const mhd_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

mhd_status mhd_init(const mhd_config *cfg, void *hip_stream, mhd_ctx **out)
{
    if (!out) return MHD_ERR_ARG;
    *out = nullptr;
    const char *why = "";
    const mhd_status cst = check_config(cfg, why);
    if (cst != MHD_OK) return cst;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MHD_ERR_NO_DEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MHD_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MHD_ERR_NO_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MHD_ERR_NO_DEVICE;
    // set-up of mhd_step_noalloc's static scratch on this device
    unsigned char *noalloc_base = nullptr;
    const mhd_status sst = noalloc_scratch(dev, &noalloc_base);
    if (sst != MHD_OK) return sst;

    mhd_ctx *ctx = new (std::nothrow) mhd_ctx();
    if (!ctx) return MHD_ERR_HIP;
    ctx->cfg = *cfg;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->device = dev;
    ctx->ncell = 1;
    ctx->cell_volume = 1.0;
    for (int d = 0; d < 3; ++d) {
        ctx->n[d] = cfg->n[d];
        ctx->ncell *= cfg->n[d];
        ctx->dx[d] = d < cfg->ndim ? (cfg->hi[d] - cfg->lo[d]) / (double)cfg->n[d] : 1.0;
        if (d < cfg->ndim) ctx->cell_volume *= ctx->dx[d];
    }
    ctx->elem = cfg->dtype == MHD_F32 ? 4 : 8;
    // partials capacity: the forward stage grid (the CFL kernel uses at most
    // CFL_MAX_BLOCKS); the adjoint writes no partials
    const int ty = cfg->ndim == 1 ? 1
                 : (cfg->dtype == MHD_F32 ? (cfg->limiter == MHD_WENOZ ? tile_rows<float, LIM_WENOZ, 3>()
                                                                       : tile_rows<float, LIM_MINMOD, 3>())
                                          : tile_rows<double, LIM_MINMOD, 3>());
    const Launch L = plan_stage(ctx, ty);
    ctx->part_cap = std::max(L.nblocks, CFL_MAX_BLOCKS);
    ctx->ns = cfg->ct ? 12 : NQ;
    hipError_t e = hipMalloc(&ctx->u1_scratch, (size_t)ctx->ns * ctx->ncell * ctx->elem);
    if (e == hipSuccess && cfg->time_order == 3)
        e = hipMalloc(&ctx->u2_scratch, (size_t)ctx->ns * ctx->ncell * ctx->elem);
    if (e == hipSuccess && cfg->ct == 1) e = hipMalloc(&ctx->ct_flx, (size_t)6 * ctx->ncell * ctx->elem);
    if (e == hipSuccess && cfg->ct) e = hipMalloc(&ctx->ct_emf, (size_t)3 * ctx->ncell * ctx->elem);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->part, (size_t)NPART * ctx->part_cap * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->result, NPART * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->cfl_result, NPART * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->flag, sizeof(int));
    if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->host_res, (NPART + 1) * sizeof(double));
    if (e == hipSuccess && (cfg->flags & MHD_FLAG_ADJOINT))
        e = hipMalloc((void **)&ctx->lam1, (size_t)NQ * ctx->ncell * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        free_ctx(ctx);
        return MHD_ERR_HIP;
    }
    *out = ctx;
    return MHD_OK;
}

void mhd_destroy(mhd_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
}

mhd_status mhd_set_stream(mhd_ctx *ctx, void *hip_stream)
{
    if (!ctx) return MHD_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return MHD_OK;
}

mhd_status mhd_prim_to_cons(mhd_ctx *ctx, const double *V, void *U)
{
    if (!ctx) return MHD_ERR_ARG;
    if (!V || !U) return fail(ctx, MHD_ERR_ARG, "null buffer");
    const int nb = (int)std::min<long long>((ctx->ncell + RED_THREADS - 1) / RED_THREADS, 8192);
    const double ig = 1.0 / (ctx->cfg.gamma - 1.0);
    const int nx = (int)ctx->n[0], ny = (int)ctx->n[1], nz = (int)ctx->n[2];
    if (ctx->cfg.ct && ctx->cfg.dtype == MHD_F32)
        hipLaunchKernelGGL(prim_to_cons_ct_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, V,
                           (float *)U, nx, ny, nz, ig);
    else if (ctx->cfg.ct)
        hipLaunchKernelGGL(prim_to_cons_ct_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, V,
                           (double *)U, nx, ny, nz, ig);
    else if (ctx->cfg.dtype == MHD_F32)
        hipLaunchKernelGGL(prim_to_cons_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, V,
                           (float *)U, ctx->ncell, ig);
    else
        hipLaunchKernelGGL(prim_to_cons_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, V,
                           (double *)U, ctx->ncell, ig);
    HIP_TRY(ctx, hipGetLastError());
    return MHD_OK;
}

mhd_status mhd_prim_to_cons_adjoint(mhd_ctx *ctx, const double *V, const double *lam_U, double *lam_V)
{
    if (!ctx) return MHD_ERR_ARG;
    if (!V || !lam_U || !lam_V) return fail(ctx, MHD_ERR_ARG, "null buffer");
    if (lam_U == lam_V) return fail(ctx, MHD_ERR_ARG, "lam_V must not alias lam_U");
    if (ctx->cfg.ct) return fail(ctx, MHD_ERR_UNSUPPORTED, "no adjoint with constrained transport");
    const int nb = (int)std::min<long long>((ctx->ncell + RED_THREADS - 1) / RED_THREADS, 8192);
    hipLaunchKernelGGL(prim_to_cons_adjoint_kernel, dim3(nb), dim3(RED_THREADS), 0, ctx->stream, V,
                       lam_U, lam_V, ctx->ncell, 1.0 / (ctx->cfg.gamma - 1.0));
    HIP_TRY(ctx, hipGetLastError());
    return MHD_OK;
}

mhd_status mhd_cfl_dt(mhd_ctx *ctx, const void *U, double out[2])
{
    if (!ctx) return MHD_ERR_ARG;
    if (!U || !out) return fail(ctx, MHD_ERR_ARG, "null buffer");
    mhd_status st = ctx->cfg.dtype == MHD_F32 ? launch_cfl<float>(ctx, (const float *)U)
                                               : launch_cfl<double>(ctx, (const double *)U);
    if (st != MHD_OK) return st;
    st = sync_results(ctx, ctx->cfl_result);
    if (st != MHD_OK) return st;
    out[0] = ctx->cfg.cfl / ctx->host_res[0];
    out[1] = ctx->host_res[1];
    return MHD_OK;
}

mhd_status mhd_step(mhd_ctx *ctx, const void *Un, void *U_next, void *U1_out, double dt, double c_h,
                    double damp)
{
    if (!ctx) return MHD_ERR_ARG;
    if (!Un || !U_next) return fail(ctx, MHD_ERR_ARG, "null buffer");
    if (Un == U_next || U1_out == Un || (U1_out && U1_out == U_next))
        return fail(ctx, MHD_ERR_ARG, "state buffers must not alias");
    if (!finite_pos(dt)) return fail(ctx, MHD_ERR_ARG, "dt must be finite and > 0");
    if (ctx->cfg.glm && !finite_pos(c_h)) return fail(ctx, MHD_ERR_ARG, "c_h must be finite and > 0");
    if (!(damp > 0.0 && damp <= 1.0)) return fail(ctx, MHD_ERR_ARG, "damp must be in (0, 1]");
    void *u1 = U1_out ? U1_out : ctx->u1_scratch;
    const mhd_status st = with_scheme(ctx, [&](auto sch) {
        using S = decltype(sch);
        return launch_step_nd<typename S::T, S::SOLVER, S::LIM>(ctx, Un, U_next, u1, dt, c_h, damp);
    });
    if (st == MHD_OK) ctx->have_step = true;
    return st;
}

mhd_status mhd_step_info(mhd_ctx *ctx, double out[11])
{
    if (!ctx) return MHD_ERR_ARG;
    if (!out) return fail(ctx, MHD_ERR_ARG, "null buffer");
    if (!ctx->have_step) return fail(ctx, MHD_ERR_ARG, "no step has run on this context");
    mhd_status st = sync_results(ctx, ctx->result);
    if (st != MHD_OK) return st;
    out[0] = ctx->cfg.cfl / ctx->host_res[0];
    out[1] = ctx->host_res[1];
    for (int q = 0; q < NQ; ++q) out[2 + q] = ctx->host_res[2 + q] * ctx->cell_volume;
    return MHD_OK;
}

mhd_status mhd_get_sums(mhd_ctx *ctx, double out[9])
{
    if (!ctx) return MHD_ERR_ARG;
    if (!out) return fail(ctx, MHD_ERR_ARG, "null buffer");
    if (!ctx->have_step) return fail(ctx, MHD_ERR_ARG, "no step has run on this context");
    mhd_status st = sync_results(ctx, ctx->result);
    if (st != MHD_OK) return st;
    for (int q = 0; q < NQ; ++q) out[q] = ctx->host_res[2 + q] * ctx->cell_volume;
    return MHD_OK;
}

mhd_status mhd_step_noalloc(const mhd_config *cfg, void *hip_stream, const void *Un, void *U_next,
                            void *U1_out, double dt, double c_h, double damp, double info[11])
{
    const char *why = "";
    const mhd_status cst = check_config(cfg, why);
    if (cst != MHD_OK) return cst;
    if (cfg->flags != 0) return MHD_ERR_ARG;
    if (cfg->time_order != 2 || cfg->ct) return MHD_ERR_UNSUPPORTED;
    if (!Un || !U_next || !U1_out) return MHD_ERR_ARG;
    if (Un == U_next || U1_out == Un || U1_out == U_next) return MHD_ERR_ARG;
    if (!finite_pos(dt)) return MHD_ERR_ARG;
    if (cfg->glm && !finite_pos(c_h)) return MHD_ERR_ARG;
    if (!(damp > 0.0 && damp <= 1.0)) return MHD_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MHD_ERR_NO_DEVICE;
    unsigned char *base = nullptr;
    const mhd_status sst = noalloc_scratch(dev, &base);
    if (sst != MHD_OK) return sst;

    // a transient context over the static scratch (no member allocates:
    // the event list stays empty and errors keep no text)
    mhd_ctx c;
    c.no_alloc = true;
    c.cfg = *cfg;
    c.stream = (hipStream_t)hip_stream;
    c.device = dev;
    c.ncell = 1;
    for (int d = 0; d < 3; ++d) {
        c.n[d] = cfg->n[d];
        c.ncell *= cfg->n[d];
        c.dx[d] = d < cfg->ndim ? (cfg->hi[d] - cfg->lo[d]) / (double)cfg->n[d] : 1.0;
        if (d < cfg->ndim) c.cell_volume *= c.dx[d];
    }
    c.elem = cfg->dtype == MHD_F32 ? 4 : 8;
    c.part = (double *)base;
    c.part_cap = NOALLOC_MAX_BLOCKS;
    c.result = (double *)(base + NOALLOC_RESULT_OFF);
    c.flag = (int *)(base + NOALLOC_FLAG_OFF);
    // launch_step refuses a stage grid beyond NOALLOC_MAX_BLOCKS with
    // MHD_ERR_ARG before it enqueues anything
    const mhd_status st = with_scheme(&c, [&](auto sch) {
        using S = decltype(sch);
        return launch_step_nd<typename S::T, S::SOLVER, S::LIM>(&c, Un, U_next, U1_out, dt, c_h, damp);
    });
    if (st != MHD_OK || !info) return st;
    double res[NPART];
    int flag = 0;
    if (hipMemcpyAsync(res, c.result, sizeof res, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipMemcpyAsync(&flag, c.flag, sizeof flag, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
        return MHD_ERR_HIP;
    if (flag) return MHD_ERR_NONPHYSICAL;
    info[0] = cfg->cfl / res[0];
    info[1] = res[1];
    for (int q = 0; q < NQ; ++q) info[2 + q] = res[2 + q] * c.cell_volume;
    return MHD_OK;
}

mhd_status mhd_step_adjoint(mhd_ctx *ctx, const void *Un, const void *U1, const double *lam_next,
                            double *lam_n, double dt, double c_h, double damp)
{
    if (!ctx) return MHD_ERR_ARG;
    if (!Un || !lam_next || !lam_n) return fail(ctx, MHD_ERR_ARG, "null buffer");
    if (lam_next == lam_n) return fail(ctx, MHD_ERR_ARG, "lam_n must not alias lam_next");
    if (!finite_pos(dt)) return fail(ctx, MHD_ERR_ARG, "dt must be finite and > 0");
    if (ctx->cfg.glm && !finite_pos(c_h)) return fail(ctx, MHD_ERR_ARG, "c_h must be finite and > 0");
    if (!(damp > 0.0 && damp <= 1.0)) return fail(ctx, MHD_ERR_ARG, "damp must be in (0, 1]");
    if (!(ctx->cfg.flags & MHD_FLAG_ADJOINT))
        return fail(ctx, MHD_ERR_ARG, "context was created without MHD_FLAG_ADJOINT");
    if ((const void *)lam_n == Un || (const void *)lam_n == U1)
        return fail(ctx, MHD_ERR_ARG, "lam_n must not alias a state buffer");
    return with_scheme(ctx, [&](auto sch) -> mhd_status {
        using S = decltype(sch);
        if constexpr (S::LIM == LIM_WENOZ)
            return fail(ctx, MHD_ERR_UNSUPPORTED, "no adjoint of WENO-Z");  // mhd_init refuses it first
        else
            return launch_adjoint_nd<typename S::T, S::SOLVER, S::LIM>(ctx, Un, U1, lam_next, lam_n, dt, c_h,
                                                                      damp);
    });
}

} // extern "C"
