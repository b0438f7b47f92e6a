// Constrained transport (Evans & Hawley 1988) on periodic 3D grids: the
// field lives on the cell faces (state components 9..11: bx, by, bz on each
// cell's lower x, y and z face), each Riemann problem takes its face's value
// as the normal field (the stage kernel), the edge EMFs are the arithmetic
// mean of the four face fluxes around each edge (Balsara & Spicer 1999), the
// faces advance by the discrete curl of the EMFs with the stage's
// Runge-Kutta combination, and the cell field is the mean of each cell's two
// faces along each axis.
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
