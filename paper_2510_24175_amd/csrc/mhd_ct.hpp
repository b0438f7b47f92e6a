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
// element-wise passes (HBM-bound, no LDS) over a grid-stride range.
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

// Per-cell inputs of the upwind EMF, from the stage's input state: velocity
// (3) and fast magnetosonic speed along each axis (3), to w[6][ncell].
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) ct_cell_speeds_kernel(const CTArgs<T> a, T *w)
{
    const long long nc = a.ncell;
    const T gamma = (T)a.gamma_d, gm1 = (T)(a.gamma_d - 1.0);
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < nc;
         c += (long long)gridDim.x * RED_THREADS) {
        const T rho = a.uin[c], ir = Num<T>::rcp(rho);
        const T m[3] = {a.uin[nc + c], a.uin[2 * nc + c], a.uin[3 * nc + c]};
        const T b[3] = {a.uin[5 * nc + c], a.uin[6 * nc + c], a.uin[7 * nc + c]};
        const T bsq = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        const T pr = gm1 * (a.uin[4 * nc + c] - T(0.5) * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir -
                            T(0.5) * bsq);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            w[(long long)d * nc + c] = m[d] * ir;
            w[(long long)(3 + d) * nc + c] = fast_speed(rho, pr, bsq, b[d] * b[d], gamma, ir);
        }
    }
}

// Upwind edge EMFs (upwind constrained transport of Londrillo & Del Zanna
// 2004, HLL averaging), on each cell's lower edges, from the cells'
// velocities and fast speeds (w, ct_cell_speeds_kernel) and the face field
// of the stage's input state.  For the EMF along axis e, with (e, p, q)
// cyclic, four cells meet at the edge: the lower or upper one along p
// (a = 0, 1) and along q (b = 0, 1).  Each gives a state at the edge:
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
// Each thread reads the velocities of the 12 cells of the 4 x 4 block around
// an edge (corners left out) for the states and their slopes.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) ct_emf_upwind_kernel(const CTArgs<T> a, const T *w)
{
    const long long nxy = (long long)a.nx * a.ny, nc = a.ncell;
    const int n3[3] = {a.nx, a.ny, a.nz};
    const long long st[3] = {1, a.nx, nxy};
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < nc;
         c += (long long)gridDim.x * RED_THREADS) {
        int co[3];
        ct_coords(c, a.nx, a.ny, co[0], co[1], co[2]);
        // offset of the cell m = -2 .. 1 steps away along each axis (periodic)
        long long off[3][4];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int m = -2; m <= 1; ++m) off[d][m + 2] = (long long)(ct_wrap(co[d] + m, n3[d]) - co[d]) * st[d];
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int p = (e + 1) % 3, q = (e + 2) % 3;
            const T *vpa = w + (long long)p * nc, *vqa = w + (long long)q * nc;
            const T *cpa = w + (long long)(3 + p) * nc, *cqa = w + (long long)(3 + q) * nc;
            // velocities along p and q of the 4 x 4 block (mp, mq) in -2 .. 1
            T vp[4][4], vq[4][4];
#pragma unroll
            for (int mp = 0; mp < 4; ++mp) {
#pragma unroll
                for (int mq = 0; mq < 4; ++mq) {
                    vp[mp][mq] = vq[mp][mq] = T(0);
                    if ((mp == 0 || mp == 3) && (mq == 0 || mq == 3)) continue;  // corners: not used
                    const long long x = c + off[p][mp] + off[q][mq];
                    vp[mp][mq] = vpa[x];
                    vq[mp][mq] = vqa[x];
                }
            }
            T ev[2][2][2];  // corner velocities (p, q components) of cell (a, b)
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
                    const long long x = c + off[p][mp] + off[q][mq];
                    const T cp = cpa[x], cq = cqa[x];
                    app = Num<T>::max(app, vp[mp][mq] + cp);
                    apm = Num<T>::max(apm, cp - vp[mp][mq]);
                    aqp = Num<T>::max(aqp, vq[mp][mq] + cq);
                    aqm = Num<T>::max(aqm, cq - vq[mp][mq]);
                }
            }
            // face fields at the edge: the q faces of the cells on either side
            // along p, reconstructed along p; the p faces on either side along
            // q, reconstructed along q
            T Bq[2], Bp[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const T h = T(0.5) - T(s2);
                const T *fq = a.uin + (long long)(9 + q) * nc;
                const T f0 = fq[c + off[p][s2 + 1]];
                Bq[s2] = f0 + h * Num<T>::minmod(f0 - fq[c + off[p][s2]], fq[c + off[p][s2 + 2]] - f0);
                const T *fp = a.uin + (long long)(9 + p) * nc;
                const T g0 = fp[c + off[q][s2 + 1]];
                Bp[s2] = g0 + h * Num<T>::minmod(g0 - fp[c + off[q][s2]], fp[c + off[q][s2 + 2]] - g0);
            }
            const T isp = Num<T>::rcp(app + apm), isq = Num<T>::rcp(aqp + aqm);
            const T wp[2] = {app * isp, apm * isp}, wq[2] = {aqp * isq, aqm * isq};
            T Em = T(0);
#pragma unroll
            for (int ca = 0; ca < 2; ++ca) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    Em += wp[ca] * wq[cb] * (ev[ca][cb][1] * Bp[cb] - ev[ca][cb][0] * Bq[ca]);
            }
            Em += app * apm * isp * (Bq[1] - Bq[0]) - aqp * aqm * isq * (Bp[1] - Bp[0]);
            a.emf[(long long)e * nc + c] = Em;
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
