// Standalone CFL reduction, the deterministic final pass over block
// partials, and the primitive -> conserved map.
#pragma once

#include "mhd_stage.hpp"

namespace mhd {

constexpr int RED_THREADS = 256;

// Per-block FP64 maxima of (|v_d|+c_f,d)/dx_d and |v_d|+c_f,d over a
// grid-stride range of cells; partials [2][nblocks] (sums left zero).
template <typename T, int NDIM>
__global__ void __launch_bounds__(RED_THREADS)
cfl_kernel(const T *__restrict__ U, long long ncell, double gamma, double idx0, double idx1,
           double idx2, double *part, int nblocks, int *flag)
{
    const double idx[3] = {idx0, idx1, idx2};
    double smax = 0.0, cmax = 0.0;
    bool ok = true;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * RED_THREADS) {
        T u[NQ];
        load_cell(U, ncell, c, u);
        ok &= cell_speeds<T, NDIM>(u, gamma, idx, smax, cmax);
    }
    if (!ok) atomicOr(flag, 1);
    __shared__ double red[2][RED_THREADS / 64];
    smax = wave_max(smax);
    cmax = wave_max(cmax);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = smax;
        red[1][w] = cmax;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double r = red[threadIdx.x][0];
        for (int k = 1; k < RED_THREADS / 64; ++k) r = __builtin_fmax(r, red[threadIdx.x][k]);
        part[(long long)threadIdx.x * nblocks + blockIdx.x] = r;
        for (int e = 2 + threadIdx.x; e < NPART; e += 2) part[(long long)e * nblocks + blockIdx.x] = 0.0;
    }
}

// Clears the non-physical flag (a kernel rather than a memset, so that a
// caller may capture it in a HIP graph).
__global__ void clear_flag_kernel(int *flag) { *flag = 0; }

// One workgroup folds nblocks partials into out[NPART] in a fixed order:
// each thread runs over a strided subset sequentially, then a fixed tree.
__global__ void __launch_bounds__(RED_THREADS)
final_reduce_kernel(const double *__restrict__ part, int nblocks, double *out)
{
    __shared__ double red[NPART][RED_THREADS];
    const int t = threadIdx.x;
    double acc[NPART];
#pragma unroll
    for (int e = 0; e < NPART; ++e) acc[e] = 0.0;
    for (int b = t; b < nblocks; b += RED_THREADS) {
        acc[0] = __builtin_fmax(acc[0], part[b]);
        acc[1] = __builtin_fmax(acc[1], part[(long long)nblocks + b]);
#pragma unroll
        for (int e = 2; e < NPART; ++e) acc[e] += part[(long long)e * nblocks + b];
    }
#pragma unroll
    for (int e = 0; e < NPART; ++e) red[e][t] = acc[e];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] = __builtin_fmax(red[0][t], red[0][t + s]);
            red[1][t] = __builtin_fmax(red[1][t], red[1][t + s]);
#pragma unroll
            for (int e = 2; e < NPART; ++e) red[e][t] += red[e][t + s];
        }
        __syncthreads();
    }
    if (t < NPART) out[t] = red[t][0];
}

// V (double primitives) -> U (state type): E in FP64, one rounding.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
prim_to_cons_kernel(const double *__restrict__ V, T *__restrict__ U, long long ncell,
                    double inv_gm1)
{
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * RED_THREADS) {
        double v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = V[q * ncell + c];
        const double rho = v[RHO];
        const double E = v[PRS] * inv_gm1 + 0.5 * rho * (v[VX] * v[VX] + v[VY] * v[VY] + v[VZ] * v[VZ]) +
                         0.5 * (v[BX] * v[BX] + v[BY] * v[BY] + v[BZ] * v[BZ]);
        U[c] = (T)rho;
        U[1 * ncell + c] = (T)(rho * v[VX]);
        U[2 * ncell + c] = (T)(rho * v[VY]);
        U[3 * ncell + c] = (T)(rho * v[VZ]);
        U[4 * ncell + c] = (T)E;
        U[5 * ncell + c] = (T)v[BX];
        U[6 * ncell + c] = (T)v[BY];
        U[7 * ncell + c] = (T)v[BZ];
        U[8 * ncell + c] = (T)v[PSI];
    }
}

// lam_V = (dU/dV)^T lam_U for U(V) above (all FP64).
__global__ void __launch_bounds__(RED_THREADS)
prim_to_cons_adjoint_kernel(const double *__restrict__ V, const double *__restrict__ lu,
                            double *__restrict__ lv, long long ncell, double inv_gm1)
{
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * RED_THREADS) {
        double v[NQ], l[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            v[q] = V[q * ncell + c];
            l[q] = lu[q * ncell + c];
        }
        const double rho = v[RHO];
        const double vsq = v[VX] * v[VX] + v[VY] * v[VY] + v[VZ] * v[VZ];
        // U = (rho, rho v, p/(g-1) + rho|v|^2/2 + |B|^2/2, B, psi)
        lv[c] = l[RHO] + l[MX] * v[VX] + l[MY] * v[VY] + l[MZ] * v[VZ] + l[ENG] * 0.5 * vsq;
        lv[1 * ncell + c] = l[MX] * rho + l[ENG] * rho * v[VX];
        lv[2 * ncell + c] = l[MY] * rho + l[ENG] * rho * v[VY];
        lv[3 * ncell + c] = l[MZ] * rho + l[ENG] * rho * v[VZ];
        lv[4 * ncell + c] = l[ENG] * inv_gm1;
        lv[5 * ncell + c] = l[BX] + l[ENG] * v[BX];
        lv[6 * ncell + c] = l[BY] + l[ENG] * v[BY];
        lv[7 * ncell + c] = l[BZ] + l[ENG] * v[BZ];
        lv[8 * ncell + c] = l[PSI];
    }
}

} // namespace mhd
