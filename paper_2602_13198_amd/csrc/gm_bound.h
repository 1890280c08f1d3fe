// Register-limited FP64 bound of the tracking kernel: dependent chains of
// FP64 fused multiply-adds at a fixed number of waves per SIMD.
//
// The tracker's FP64 state keeps it at a few waves per SIMD, and most of its
// arithmetic (software exp, log, cbrt and division sequences, the push) is
// a chain of dependent operations.  This kernel runs `CHAINS` independent
// FMA chains per lane with the same waves per SIMD, so its attained rate is
// what FP64 vector code of that occupancy and dependency depth can reach on
// the chip.  The occupancy is pinned by the launch: grid = CUs x waves
// blocks of 256 threads, each block reserving enough LDS that no more than
// `waves` blocks (one wave per SIMD each) fit on a CU.
#pragma once
#include "gm_common.h"

namespace gm {

template <int CHAINS>
__global__ __launch_bounds__(256) void fma_chain_kernel(double m, double a, long long iters, double *out)
{
#pragma clang fp contract(off)
    extern __shared__ double lds_reserve[];
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c)   // (1 + 1e-9 t) + 1e-3 c, each operation rounded on its own
        acc[c] = (1.0 + 1e-9 * (double)t) + 1e-3 * (double)c;
#pragma unroll 8
    for (long long i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = __fma_rn(acc[c], m, a);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += acc[c];
    if (iters < 0) lds_reserve[threadIdx.x] = s;   // never taken; keeps the reservation referenced
    out[t] = s;
}

}  // namespace gm
