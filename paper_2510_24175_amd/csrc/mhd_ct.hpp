// Constrained transport (Evans & Hawley 1988) on periodic 3D grids: the
// field lives on the cell faces (state components 9..11: bx, by, bz on each
// cell's lower x, y and z face), each Riemann problem takes its face's value
// as the normal field (the stage kernel), the edge EMFs are the arithmetic
// mean of the four face fluxes around each edge (Balsara & Spicer 1999) or
// the upwind EMFs of Londrillo & Del Zanna (2004), the faces advance by the
// discrete curl of the EMFs with the stage's Runge-Kutta combination, and
// the cell field is the mean of each cell's two faces along each axis.
//
// With E = -v x B the transverse field fluxes are F_x(By) = -Ez,
// F_x(Bz) = Ey, F_y(Bx) = Ez, F_y(Bz) = -Ex, F_z(Bx) = -Ey, F_z(By) = Ex.
// The stage kernel leaves them, for each cell's lower faces, in flx[6][ncell]
// (x: By, Bz; y: Bx, Bz; z: Bx, By); emf_kernel forms the EMFs on each cell's
// lower edges (Ex at (j-1/2, k-1/2), Ey at (i-1/2, k-1/2), Ez at
// (i-1/2, j-1/2)); face_kernel applies dB/dt = -curl E.  Both are
// element-wise passes (HBM-bound, no LDS) over a grid-stride range.  The
// upwind EMF instead takes the stage's input state itself (the stage kernel
// then stores no fluxes) in a z-marching tiled pass.
#pragma once

#include "mhd_reduce.hpp"

namespace mhd {

template <typename T> struct CTArgs {
    const T *un;    // Un (combine); components 9..11 its faces
    const T *uin;   // the stage's input state
    T *uout;        // the stage's output: faces and cell field written here
    const T *flx;   // [6][ncell] transverse field fluxes (stage kernel)
    T *emf;         // [3][ncell] edge EMFs
    double *part;   // last stage: NPART x nblocks partials
    int *flag;      // non-physical flag
    int nx, ny, nz;
    long long ncell;
    T dt;
    T idx[3];
    double gamma_d;
    double idx_d[3];
    int nblocks;
};

// periodic neighbour of a cell coordinate one step away
__device__ __forceinline__ int ct_wrap(int m, int n) { return m < 0 ? m + n : (m >= n ? m - n : m); }

// (i, j, k) of a cell index in 32-bit arithmetic (a constrained-transport
// context holds 15 or more state-sized arrays, so ncell < 2^31 on any device)
__device__ __forceinline__ void ct_coords(long long c, int nx, int ny, int &i, int &j, int &k)
{
    const unsigned cc = (unsigned)c, row = cc / (unsigned)nx;
    i = (int)(cc - row * (unsigned)nx);
    k = (int)(row / (unsigned)ny);
    j = (int)(row - (unsigned)k * (unsigned)ny);
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) ct_emf_kernel(const CTArgs<T> a)
{
    const long long nxy = (long long)a.nx * a.ny;
    const T *FxBy = a.flx, *FxBz = a.flx + a.ncell, *FyBx = a.flx + 2 * a.ncell;
    const T *FyBz = a.flx + 3 * a.ncell, *FzBx = a.flx + 4 * a.ncell, *FzBy = a.flx + 5 * a.ncell;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < a.ncell;
         c += (long long)gridDim.x * RED_THREADS) {
        int i, j, k;
        ct_coords(c, a.nx, a.ny, i, j, k);
        const long long xm = c - i + ct_wrap(i - 1, a.nx);
        const long long ym = c + (long long)(ct_wrap(j - 1, a.ny) - j) * a.nx;
        const long long zm = c + (long long)(ct_wrap(k - 1, a.nz) - k) * nxy;
        a.emf[c] = T(0.25) * ((FzBy[ym] + FzBy[c]) - (FyBz[zm] + FyBz[c]));
        a.emf[a.ncell + c] = T(0.25) * ((FxBz[zm] + FxBz[c]) - (FzBx[xm] + FzBx[c]));
        a.emf[2 * a.ncell + c] = T(0.25) * ((FyBx[xm] + FyBx[c]) - (FxBy[ym] + FxBy[c]));
    }
}

// Velocity (3) and fast magnetosonic speed along each axis (3) of cell c
// of the conserved state u (cell-centred field), for the upwind EMF.
template <typename T>
__device__ __forceinline__ void ct_cell_vc(const T *__restrict__ u, long long nc, long long c, T gamma, T gm1,
                                           T *v, T *cf)
{
    const T rho = u[c], ir = Num<T>::rcp(rho);
    const T m[3] = {u[nc + c], u[2 * nc + c], u[3 * nc + c]};
    const T b[3] = {u[5 * nc + c], u[6 * nc + c], u[7 * nc + c]};
    const T bsq = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const T pr = gm1 * (u[4 * nc + c] - T(0.5) * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir - T(0.5) * bsq);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[d] = m[d] * ir;
        cf[d] = fast_speed(pr, bsq, b[d] * b[d], gamma, ir);
    }
}

// Upwind EMF (upwind constrained transport of Londrillo & Del Zanna 2004,
// HLL averaging) of one edge along axis e, with (e, p, q) cyclic.  Four
// cells meet at the edge: the lower or upper one along p (a = 0, 1) and
// along q (b = 0, 1).  Each gives a state at the edge:
//   v^ab  = cell velocity + (1/2 - a) s_p(v) + (1/2 - b) s_q(v),
//   B_q^a = q-face field on side a + (1/2 - a) s_p(B_q),
//   B_p^b = p-face field on side b + (1/2 - b) s_q(B_p),
//   E^ab  = -(v_p^ab B_q^a - v_q^ab B_p^b),
// s the minmod slope along an axis.  With HLL bounds a_p+ = max(0, v_p +
// c_f,p), a_p- = max(0, c_f,p - v_p) over the four cells (likewise along q),
//   E = sum_ab w_p^a w_q^b E^ab + a_p+ a_p- (B_q^1 - B_q^0) / (a_p+ + a_p-)
//                              - a_q+ a_q- (B_p^1 - B_p^0) / (a_q+ + a_q-),
// w_p^0 = a_p+ / (a_p+ + a_p-), w_p^1 = a_p- / (a_p+ + a_p-): the HLL flux of
// B_q along p (F_p(B_q) = -E_e) and of B_p along q (F_q(B_p) = E_e); where
// the fields vary along p alone it is the one-dimensional HLL flux of B_q.
// Inputs: vp, vq the p and q velocity components of the 4 x 4 cell block
// [mp][mq], mp, mq = 0..3 for offsets -2..1 along p and q from the upper
// cell of the edge (corners unused); cp, cq the fast speeds along p and q
// of its four cells (mp, mq = 1, 2); fq[m] the q-face field of the cells at
// p offset m - 2, on the edge's q plane; fp[m] the p-face field of the
// cells at q offset m - 2.
template <typename T>
__device__ __forceinline__ T ct_upwind_edge(const T (&vp)[4][4], const T (&vq)[4][4], const T (&cp)[4][4],
                                            const T (&cq)[4][4], const T (&fq)[4], const T (&fp)[4])
{
    T ev[2][2][2];  // edge velocities (p, q components) from cell (a, b)
    T app = T(0), apm = T(0), aqp = T(0), aqm = T(0);
#pragma unroll
    for (int ca = 0; ca < 2; ++ca) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int mp = ca + 1, mq = cb + 1;  // block index of the cell
            const T hp = T(0.5) - T(ca), hq = T(0.5) - T(cb);
            const T spp = Num<T>::minmod(vp[mp][mq] - vp[mp - 1][mq], vp[mp + 1][mq] - vp[mp][mq]);
            const T sqp = Num<T>::minmod(vp[mp][mq] - vp[mp][mq - 1], vp[mp][mq + 1] - vp[mp][mq]);
            const T spq = Num<T>::minmod(vq[mp][mq] - vq[mp - 1][mq], vq[mp + 1][mq] - vq[mp][mq]);
            const T sqq = Num<T>::minmod(vq[mp][mq] - vq[mp][mq - 1], vq[mp][mq + 1] - vq[mp][mq]);
            ev[ca][cb][0] = vp[mp][mq] + hp * spp + hq * sqp;
            ev[ca][cb][1] = vq[mp][mq] + hp * spq + hq * sqq;
            app = Num<T>::max(app, vp[mp][mq] + cp[mp][mq]);
            apm = Num<T>::max(apm, cp[mp][mq] - vp[mp][mq]);
            aqp = Num<T>::max(aqp, vq[mp][mq] + cq[mp][mq]);
            aqm = Num<T>::max(aqm, cq[mp][mq] - vq[mp][mq]);
        }
    }
    // face fields at the edge, reconstructed along p (B_q) and q (B_p)
    T Bq[2], Bp[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const T h = T(0.5) - T(s2);
        const T f0 = fq[s2 + 1];
        Bq[s2] = f0 + h * Num<T>::minmod(f0 - fq[s2], fq[s2 + 2] - f0);
        const T g0 = fp[s2 + 1];
        Bp[s2] = g0 + h * Num<T>::minmod(g0 - fp[s2], fp[s2 + 2] - g0);
    }
    const T isp = Num<T>::rcp(app + apm), isq = Num<T>::rcp(aqp + aqm);
    const T wp[2] = {app * isp, apm * isp}, wq[2] = {aqp * isq, aqm * isq};
    T Em = T(0);
#pragma unroll
    for (int ca = 0; ca < 2; ++ca) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) Em += wp[ca] * wq[cb] * (ev[ca][cb][1] * Bp[cb] - ev[ca][cb][0] * Bq[ca]);
    }
    Em += app * apm * isp * (Bq[1] - Bq[0]) - aqp * aqm * isq * (Bp[1] - Bp[0]);
    return Em;
}

// Tiling of the upwind EMF pass: TX x TY column tiles, z chunks of kz planes.
struct CTTiles {
    int tiles_x, tiles_y, kz, nblocks;
};

// Upwind edge EMFs on each cell's lower edges (Ex at (j-1/2, k-1/2), Ey at
// (i-1/2, k-1/2), Ez at (i-1/2, j-1/2)), from the stage's input state.  A
// workgroup owns a tile of TX x TY columns (one thread per column) and
// marches along z over a chunk of planes.  The 4 x 4 blocks of the three
// edges of a cell span planes k-2 .. k+1 and, in each, rows and columns -2
// .. 1 around it: every plane's velocities and fast speeds are formed once
// per tile (with that halo) into LDS rings, velocities for planes k-2 ..
// k+1 and fast speeds for k-1 .. k+1 (one plane ahead, formed with the
// velocities), so that a plane's cells are converted once per tile instead
// of once per use.  The face field is read from global memory: its
// in-plane neighbours at plane k, and the cell's own x and y faces at planes
// k-2 .. k+1 from a register window slid with the march.
template <typename T, int TY>
__global__ void __launch_bounds__(TX *TY) ct_emf_upwind_kernel(const CTArgs<T> a, const CTTiles g)
{
    constexpr int PX = TX + 3, PY = TY + 3, PL = PX * PY;  // LDS plane: columns -2 .. TX, rows -2 .. TY
    constexpr int NT = TX * TY;
    constexpr int NIT = (PL + NT - 1) / NT;  // plane cells per thread
    __shared__ T Vr[4][3][PL];  // velocities; plane p in slot (p + 8) & 3
    __shared__ T Cr[3][3][PL];  // fast speeds; plane p in slot (p + 9) % 3

    const int t = threadIdx.x, tx = t % TX, ty = t / TX;
    const int lb = logical_block(blockIdx.x, g.nblocks);
    const int tile_x = lb % g.tiles_x, rest = lb / g.tiles_x;
    const int tile_y = rest % g.tiles_y, chunk = rest / g.tiles_y;
    const int i0 = tile_x * TX, j0 = tile_y * TY;
    const int k0 = chunk * g.kz, k1 = min(k0 + g.kz, a.nz);
    const long long nc = a.ncell, nxy = (long long)a.nx * a.ny;
    const T gamma = (T)a.gamma_d, gm1 = (T)(a.gamma_d - 1.0);

    // in-plane index of this thread's LDS plane cells (periodic images)
    int ioff[NIT];
#pragma unroll
    for (int m = 0; m < NIT; ++m) {
        const int it = t + m * NT;
        ioff[m] = 0;
        if (it < PL) {
            const int ly = it / PX, lx = it - ly * PX;
            const int gi = ((i0 + lx - 2) % a.nx + a.nx) % a.nx;
            const int gj = ((j0 + ly - 2) % a.ny + a.ny) % a.ny;
            ioff[m] = gj * a.nx + gi;
        }
    }
    // velocities and fast speeds of plane p (-2 <= p <= nz) into the rings
    auto load_plane = [&](int p) {
        const long long zo = (long long)ct_wrap(p, a.nz) * nxy;
        const int sv = (p + 8) & 3, sc = (p + 9) % 3;
#pragma unroll
        for (int m = 0; m < NIT; ++m) {
            const int it = t + m * NT;
            if (it < PL) {
                T v[3], cf[3];
                ct_cell_vc(a.uin, nc, zo + ioff[m], gamma, gm1, v, cf);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    Vr[sv][d][it] = v[d];
                    Cr[sc][d][it] = cf[d];
                }
            }
        }
    };

    const int i = i0 + tx, j = j0 + ty;
    const bool active = (i < a.nx) & (j < a.ny);
    const int ic = active ? i : 0, jc = active ? j : 0;
    const long long col = (long long)jc * a.nx + ic;
    int ox[4], oy[4];  // offsets of the x and y neighbours -2 .. 1 (periodic)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        ox[m] = ct_wrap(ic + m - 2, a.nx) - ic;
        oy[m] = (ct_wrap(jc + m - 2, a.ny) - jc) * a.nx;
    }
    const int base = (ty + 2) * PX + tx + 2;  // the cell in an LDS plane
    const T *bxg = a.uin + 9 * nc, *byg = a.uin + 10 * nc, *bzg = a.uin + 11 * nc;
    T bxw[4], byw[4];  // own x and y faces at planes k-2 .. k+1
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const long long zo = (long long)ct_wrap(k0 + m - 2, a.nz) * nxy;
        bxw[m] = bxg[zo + col];
        byw[m] = byg[zo + col];
    }
    for (int p = k0 - 2; p <= k0 + 1; ++p) load_plane(p);
    __syncthreads();

    for (int k = k0; k < k1; ++k) {
        if (active) {
            const long long c = (long long)k * nxy + col;
            const int sv[4] = {(k + 6) & 3, (k + 7) & 3, (k + 8) & 3, (k + 9) & 3};  // planes k-2 .. k+1
            const int sc[2] = {(k + 8) % 3, (k + 9) % 3};                          // planes k-1, k
            T vp[4][4], vq[4][4], cp[4][4], cq[4][4], fq[4], fp[4];
            auto corner = [](int mp, int mq) { return (mp == 0 || mp == 3) && (mq == 0 || mq == 3); };
            // Ex: p = y, q = z
#pragma unroll
            for (int mp = 0; mp < 4; ++mp) {
#pragma unroll
                for (int mq = 0; mq < 4; ++mq) {
                    vp[mp][mq] = vq[mp][mq] = cp[mp][mq] = cq[mp][mq] = T(0);
                    if (corner(mp, mq)) continue;
                    const int x = base + (mp - 2) * PX;
                    vp[mp][mq] = Vr[sv[mq]][1][x];
                    vq[mp][mq] = Vr[sv[mq]][2][x];
                    if (mp >= 1 && mp <= 2 && mq >= 1 && mq <= 2) {
                        cp[mp][mq] = Cr[sc[mq - 1]][1][x];
                        cq[mp][mq] = Cr[sc[mq - 1]][2][x];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                fq[m] = bzg[c + oy[m]];
                fp[m] = byw[m];
            }
            a.emf[c] = ct_upwind_edge(vp, vq, cp, cq, fq, fp);
            // Ey: p = z, q = x
#pragma unroll
            for (int mp = 0; mp < 4; ++mp) {
#pragma unroll
                for (int mq = 0; mq < 4; ++mq) {
                    vp[mp][mq] = vq[mp][mq] = cp[mp][mq] = cq[mp][mq] = T(0);
                    if (corner(mp, mq)) continue;
                    const int x = base + mq - 2;
                    vp[mp][mq] = Vr[sv[mp]][2][x];
                    vq[mp][mq] = Vr[sv[mp]][0][x];
                    if (mp >= 1 && mp <= 2 && mq >= 1 && mq <= 2) {
                        cp[mp][mq] = Cr[sc[mp - 1]][2][x];
                        cq[mp][mq] = Cr[sc[mp - 1]][0][x];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                fq[m] = bxw[m];
                fp[m] = bzg[c + ox[m]];
            }
            a.emf[nc + c] = ct_upwind_edge(vp, vq, cp, cq, fq, fp);
            // Ez: p = x, q = y
#pragma unroll
            for (int mp = 0; mp < 4; ++mp) {
#pragma unroll
                for (int mq = 0; mq < 4; ++mq) {
                    vp[mp][mq] = vq[mp][mq] = cp[mp][mq] = cq[mp][mq] = T(0);
                    if (corner(mp, mq)) continue;
                    const int x = base + (mp - 2) + (mq - 2) * PX;
                    vp[mp][mq] = Vr[sv[2]][0][x];
                    vq[mp][mq] = Vr[sv[2]][1][x];
                    if (mp >= 1 && mp <= 2 && mq >= 1 && mq <= 2) {
                        cp[mp][mq] = Cr[sc[1]][0][x];
                        cq[mp][mq] = Cr[sc[1]][1][x];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                fq[m] = byg[c + ox[m]];
                fp[m] = bxg[c + oy[m]];
            }
            a.emf[2 * nc + c] = ct_upwind_edge(vp, vq, cp, cq, fq, fp);
        }
        if (k + 1 < k1) {
            // plane k+2 goes where plane k-2 (velocities) and k-1 (fast
            // speeds) were
            __syncthreads();
            load_plane(k + 2);
            const long long zo = (long long)ct_wrap(k + 2, a.nz) * nxy;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                bxw[m] = bxw[m + 1];
                byw[m] = byw[m + 1];
            }
            bxw[3] = bxg[zo + col];
            byw[3] = byg[zo + col];
            __syncthreads();
        }
    }
}

// Stage combination of the Runge-Kutta kinds of the stage kernel.
template <int KIND, typename T> __device__ __forceinline__ T rk_combine(T un, T uin, T dtr)
{
    if (KIND == 1) return uin + dtr;
    if (KIND == 2) return T(0.5) * ((un + uin) + dtr);
    if (KIND == 3) return T(0.75) * un + T(0.25) * (uin + dtr);
    return un * T(1.0 / 3.0) + T(2.0 / 3.0) * (uin + dtr);
}

// Face update and cell field; the last stage also reduces the CFL maxima
// (FP64 speeds of every cell) and the FP64 sums of the 9 cell components
// into per-block partials.
template <typename T, int KIND, bool LAST>
__global__ void __launch_bounds__(RED_THREADS) ct_face_kernel(const CTArgs<T> a)
{
    const long long nxy = (long long)a.nx * a.ny, nc = a.ncell;
    const T *Ex = a.emf, *Ey = a.emf + nc, *Ez = a.emf + 2 * nc;
    double smax = 0.0, cmax = 0.0, sum[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
    bool ok = true;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < nc;
         c += (long long)gridDim.x * RED_THREADS) {
        int i, j, k;
        ct_coords(c, a.nx, a.ny, i, j, k);
        const long long dxp = ct_wrap(i + 1, a.nx) - i;               // +x neighbour offset
        const long long dyp = (long long)(ct_wrap(j + 1, a.ny) - j) * a.nx;
        const long long dzp = (long long)(ct_wrap(k + 1, a.nz) - k) * nxy;
        // new value of the lower face of axis d of cell e (e = c or a
        // neighbour of c; its +1 neighbours along the other axes wrap the
        // same way as c's, since e differs from c only along d)
        auto face_new = [&](int d, long long e) -> T {
            T r;
            if (d == 0) r = -((Ez[e + dyp] - Ez[e]) * a.idx[1] - (Ey[e + dzp] - Ey[e]) * a.idx[2]);
            else if (d == 1) r = -((Ex[e + dzp] - Ex[e]) * a.idx[2] - (Ez[e + dxp] - Ez[e]) * a.idx[0]);
            else r = -((Ey[e + dxp] - Ey[e]) * a.idx[0] - (Ex[e + dyp] - Ex[e]) * a.idx[1]);
            const long long f = (long long)(9 + d) * nc + e;
            return rk_combine<KIND>(a.un[f], a.uin[f], a.dt * r);
        };
        T b[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const long long up = d == 0 ? dxp : (d == 1 ? dyp : dzp);
            const T lo = face_new(d, c), hi = face_new(d, c + up);
            a.uout[(long long)(9 + d) * nc + c] = lo;
            b[d] = T(0.5) * (lo + hi);
            a.uout[(long long)(BX + d) * nc + c] = b[d];
        }
        if (LAST) {
            T u[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) u[q] = (q >= BX && q <= BZ) ? b[q - BX] : a.uout[(long long)q * nc + c];
#pragma unroll
            for (int q = 0; q < NQ; ++q) sum[q] += (double)u[q];
            ok &= cell_speeds<T, 3>(u, a.gamma_d, a.idx_d, smax, cmax);
        }
    }
    if (!ok) atomicOr(a.flag, 1);
    if (LAST) {
        __shared__ double red[RED_THREADS / 64][NPART];
        double vals[NPART];
        vals[0] = wave_max(smax);
        vals[1] = wave_max(cmax);
#pragma unroll
        for (int q = 0; q < NQ; ++q) vals[2 + q] = wave_sum(sum[q]);
        const int w = threadIdx.x / 64;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int e = 0; e < NPART; ++e) red[w][e] = vals[e];
        }
        __syncthreads();
        if (threadIdx.x < NPART) {
            const int e = threadIdx.x;
            double r = red[0][e];
            for (int x = 1; x < RED_THREADS / 64; ++x) r = e < 2 ? __builtin_fmax(r, red[x][e]) : r + red[x][e];
            a.part[(long long)e * a.nblocks + blockIdx.x] = r;
        }
    }
}

// V (double, [12][ncell] with the face field in 9..11) -> U (state type):
// faces rounded once, cell field = face means formed in FP64, E in FP64
// with that field.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
prim_to_cons_ct_kernel(const double *__restrict__ V, T *__restrict__ U, int nx, int ny, int nz,
                       double inv_gm1)
{
    const long long nxy = (long long)nx * ny, nc = nxy * nz;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < nc;
         c += (long long)gridDim.x * RED_THREADS) {
        int i, j, k;
        ct_coords(c, nx, ny, i, j, k);
        const long long up[3] = {ct_wrap(i + 1, nx) - i, (long long)(ct_wrap(j + 1, ny) - j) * nx,
                                 (long long)(ct_wrap(k + 1, nz) - k) * nxy};
        double b[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double lo = V[(9 + d) * nc + c], hi = V[(9 + d) * nc + c + up[d]];
            b[d] = 0.5 * (lo + hi);
            U[(9 + d) * nc + c] = (T)lo;
        }
        const double rho = V[c], vx = V[nc + c], vy = V[2 * nc + c], vz = V[3 * nc + c];
        const double E = V[4 * nc + c] * inv_gm1 + 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                         0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        U[c] = (T)rho;
        U[nc + c] = (T)(rho * vx);
        U[2 * nc + c] = (T)(rho * vy);
        U[3 * nc + c] = (T)(rho * vz);
        U[4 * nc + c] = (T)E;
        U[5 * nc + c] = (T)b[0];
        U[6 * nc + c] = (T)b[1];
        U[7 * nc + c] = (T)b[2];
        U[8 * nc + c] = (T)V[8 * nc + c];
    }
}

} // namespace mhd
