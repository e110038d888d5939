// Fixed-order workgroup reduction shared by the bias kernels.
#pragma once
#include "sx_internal.h"

namespace sx {

// Sum N doubles over a workgroup of kBlock threads: a butterfly inside each
// wavefront, then the wavefronts in index order (the same order whatever
// the schedule); the result is in thread 0.  Ends with a barrier, so lds
// may be reused right after.
template <int N>
__device__ __forceinline__ void block_sum0(double (&v)[N], double *lds /* N * kBlock/64 */)
{
    // fixed tree: wave butterfly, then waves in index order; result in thread 0
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[wv * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = lds[k];
            for (int q = 1; q < kBlock / 64; ++q) s += lds[q * N + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

}  // namespace sx
