// Device helpers shared by the step kernels of libpimd.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "pimd_internal.h"

namespace pimd {

// --------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(unsigned long long c[4], unsigned long long k0,
                                              unsigned long long k1)
{
    const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const unsigned long long lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const unsigned long long n0 = hi1 ^ c[1] ^ k0;
        const unsigned long long n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}

__device__ __forceinline__ double u01(unsigned long long w)
{
    // top 53 bits + 1, times 2^-53: uniform on (0, 1], exact in FP64
    return ((double)(w >> 11) + 1.0) * 1.1102230246251565404e-16;
}

// Three N(0,1) deviates for atom i, mode k, step s: counter (i, k, s, 0),
// key (seed, 0); (z0, z1) from (u0, u1), z2 from (u2, u3).
__device__ __forceinline__ void gauss3(unsigned long long seed, unsigned long long i,
                                       unsigned long long k, unsigned long long s, double z[3])
{
    unsigned long long c[4] = {i, k, s, 0ULL};
    philox4x64_10(c, seed, 0ULL);
    const double r0 = sqrt(-2.0 * log(u01(c[0])));
    const double r2 = sqrt(-2.0 * log(u01(c[2])));
    double s1, c1;
    sincospi(2.0 * u01(c[1]), &s1, &c1);
    z[0] = r0 * c1;
    z[1] = r0 * s1;
    z[2] = r2 * cospi(2.0 * u01(c[3]));
}

// --------------------------------------------------------------------------
// Block reductions (fixed order).
// --------------------------------------------------------------------------
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *red /* [kBlock*NV] */)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * kBlock + t] = v[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q * kBlock + t] += red[q * kBlock + t + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = red[q * kBlock];
    __syncthreads();
}

__device__ inline double block_max(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = fmax(red[t], red[t + w]);
        __syncthreads();
    }
    v = red[0];
    __syncthreads();
    return v;
}

}  // namespace pimd
