// Hill sum over ONE hill list shared by many query points (walkers sharing
// a bias, or arbitrary evaluation points such as training and
// certification samples of a surrogate).  Metadynamics bias, Sec. 2.1.5.
//
// Unlike the private-list sum, every hill is reused by every query, so the
// work is bound by VALU arithmetic, not by HBM:
//   * grid x: hill chunks (a multiple of 256 hills, sized so that chunks x
//     query blocks fill the chip); grid y: blocks of kBlock*Q queries;
//   * a workgroup stages its chunk in LDS, 256 hills at a time (SoA, one
//     hill per lane per stage), and every lane evaluates its Q queries
//     against every staged hill (LDS broadcast reads, no bank conflicts);
//   * the displacement, the periodic wrap, the quadratic form and every sum
//     are FP64 (the same VALU rate as unpacked FP32 on CDNA4); only the
//     exponential is FP32 (v_exp_f32): summing the products e * dxi in FP32
//     loses digits where the terms of dV/dxi cancel;
//   * each (chunk, query) partial has one writer; the finalize kernel sums a
//     query's chunks in chunk order (bitwise deterministic), forms dV/dxi,
//     and appends one hill per walker for a deposition step, in walker order.
#include "sx_internal.h"

namespace sx {
namespace {

constexpr int kStage = kBlock;  // hills staged in LDS at a time

template <int D, int Q>
__global__ void __launch_bounds__(kBlock) k_hill_shared(SharedArgs a)
{
    __shared__ float s_c[D][kStage];
    __shared__ float s_h[kStage];
    const int32_t n = *a.count;
    const int64_t h0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t q0 = ((int64_t)blockIdx.y * kBlock + threadIdx.x) * Q;
    // with a query list only its first *qcount entries are live; a
    // workgroup past them leaves before its first barrier (uniform test)
    const int64_t nq = a.qlist ? (int64_t)*a.qcount : a.nq;
    if ((int64_t)blockIdx.y * kBlock * Q >= nq) return;
    double xi[Q][D];
    bool live[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        live[q] = q0 + q < nq;
        const int64_t row = !live[q] ? 0 : (a.qlist ? (int64_t)a.qlist[q0 + q] : q0 + q);
#pragma unroll
        for (int d = 0; d < D; ++d) xi[q][d] = live[q] ? a.xi[row * D + d] : 0.0;
    }
    double acc[Q][1 + D];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[q][j] = 0.0;
    const int64_t hend = min((int64_t)n, h0 + a.chunk);
    // exponent scale log2(e) / (2 sigma^2) in FP64: the quadratic form and the
    // sums are FP64 (full VALU rate here); only the exponential is FP32
    double a2[D];
#pragma unroll
    for (int d = 0; d < D; ++d) a2[d] = 0.7213475204444817 * a.inv_sig2[d];
    for (int64_t s0 = h0; s0 < hend; s0 += kStage) {
        const int64_t k = s0 + threadIdx.x;
        const bool ok = k < hend;
#pragma unroll
        for (int d = 0; d < D; ++d) s_c[d][threadIdx.x] = ok ? a.c[d][k] : 0.f;
        s_h[threadIdx.x] = ok ? a.h[k] : 0.f;  // zero height: no contribution
        __syncthreads();
        const int m = (int)min((int64_t)kStage, hend - s0);
        for (int j0 = 0; j0 < m; j0 += 4) {
#pragma unroll
            for (int j = j0; j < j0 + 4; ++j) {
                double c[D];
#pragma unroll
                for (int d = 0; d < D; ++d) c[d] = (double)s_c[d][j];
                const float h = s_h[j];  // j >= m: staged as zero height
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double x[D], qd = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        x[d] = xi[q][d] - c[d];
                        if (a.period[d] > 0.0) x[d] = fma(-a.period[d], rint(x[d] * a.inv_period[d]), x[d]);
                        qd = fma(x[d] * a2[d], x[d], qd);
                    }
                    const double e = (double)(h * __builtin_amdgcn_exp2f(-(float)qd));
                    acc[q][0] += e;
#pragma unroll
                    for (int d = 0; d < D; ++d) acc[q][1 + d] = fma(e, x[d], acc[q][1 + d]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!live[q]) continue;
        double *p = a.partial + ((int64_t)blockIdx.x * a.nq + q0 + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) p[j] = acc[q][j];
    }
}

template <int N>
__device__ __forceinline__ void block_sum0(double (&v)[N], double *lds)
{
    // fixed tree: wave butterfly, then waves in index order; result in thread 0
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[(threadIdx.x >> 6) * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = lds[k];
            for (int q = 1; q < kBlock / 64; ++q) s += lds[q * N + k];
            v[k] = s;
        }
}

// per query: V, dV/dxi, outputs and (all or none) the appended hill;
// w is the query's row (its walker, or its entry of the query list)
template <int D>
__device__ __forceinline__ void shared_finish(const SharedArgs &a, int64_t w, const double (&acc)[1 + D])
{
    const double V = acc[0];
    bool finite = isfinite(V);
    if (a.V_ws) a.V_ws[w] = V;
    if (a.V_out) a.V_out[w] = V;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double dv = -acc[1 + d] * a.inv_sig2[d];
        finite = finite && isfinite(dv);
        if (a.dV_ws) a.dV_ws[w * D + d] = dv;
        if (a.dV_out) a.dV_out[w * D + d] = dv;
        if (a.xi_out) a.xi_out[w * D + d] = a.xi[w * D + d];
    }
    if (!finite && a.flags) atomicOr(a.flags, kFlagNonFinite);
    bool dep = a.deposit == 2;
    if (a.deposit == 1 && a.stride > 0) dep = (*a.dstep - 1) % a.stride == 0;
    if (dep) {
        // all walkers append in walker order at count + w (all or none);
        // the count moves in the next kernel, after every lane read it
        const int32_t n = *a.count;
        if ((int64_t)n + a.nq <= a.cap) {
            const int64_t k = (int64_t)n + w;
#pragma unroll
            for (int d = 0; d < D; ++d) a.c[d][k] = (float)a.xi[w * D + d];
            a.h[k] = (float)(a.inv_kdT > 0.0 ? a.height * exp(-V * a.inv_kdT) : a.height);
        } else if (w == 0) {
            atomicOr(a.flags, kFlagCapacity);
        }
    }
}

// few chunks: one lane per query sums its chunks in order
template <int D>
__global__ void __launch_bounds__(kBlock) k_hill_shared_finalize(SharedArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (a.qlist ? (int64_t)*a.qcount : a.nq)) return;
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0;
    for (int ch = 0; ch < a.nchunk; ++ch) {
        const double *p = a.partial + ((int64_t)ch * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
    shared_finish<D>(a, a.qlist ? (int64_t)a.qlist[q] : q, acc);
}

// many chunks: one workgroup per query, lanes stride over the chunks and a
// fixed reduction tree combines them (deterministic)
template <int D>
__global__ void __launch_bounds__(kBlock) k_hill_shared_finalize_wg(SharedArgs a)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    const int64_t q = blockIdx.x;
    if (q >= (a.qlist ? (int64_t)*a.qcount : a.nq)) return;  // uniform per workgroup
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0;
    for (int ch = threadIdx.x; ch < a.nchunk; ch += kBlock) {
        const double *p = a.partial + ((int64_t)ch * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
    block_sum0<1 + D>(acc, lds);
    if (threadIdx.x == 0) shared_finish<D>(a, a.qlist ? (int64_t)a.qlist[q] : q, acc);
}

// the count of a shared list advances after the finalize kernel (kernel
// boundary = every lane has read the old count)
__global__ void k_shared_count(SharedArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bool dep = a.deposit == 2;
    if (a.deposit == 1 && a.stride > 0) dep = (*a.dstep - 1) % a.stride == 0;
    if (dep && (int64_t)*a.count + a.nq <= a.cap) *a.count = (int32_t)(*a.count + a.nq);
}

__global__ void k_set_step(int64_t *dstep, int64_t step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dstep = step >= 0 ? step + 1 : *dstep + 1;
}

template <int D>
hipError_t launch_shared_d(const SharedArgs &a, hipStream_t s)
{
    if (a.count_step) {
        hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, a.dstep, a.step);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // queries per lane: 1 for small query sets (more workgroups), 4 for many
    const int Q = a.nq >= 65536 ? 4 : 1;
    dim3 grid(a.nchunk, (unsigned)((a.nq + kBlock * Q - 1) / (kBlock * Q)));
    if (Q == 4)
        hipLaunchKernelGGL((k_hill_shared<D, 4>), grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_hill_shared<D, 1>), grid, dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nchunk >= 32)
        hipLaunchKernelGGL((k_hill_shared_finalize_wg<D>), dim3((unsigned)a.nq), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_hill_shared_finalize<D>), dim3((unsigned)((a.nq + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.deposit) {
        hipLaunchKernelGGL(k_shared_count, dim3(1), dim3(64), 0, s, a);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

void shared_split(int64_t cap, int64_t nq, int32_t &chunk, int32_t &nchunk)
{
    const int Q = nq >= 65536 ? 4 : 1;
    const int64_t nqb = std::max<int64_t>(1, (nq + (int64_t)kBlock * Q - 1) / ((int64_t)kBlock * Q));
    const int64_t stages = std::max<int64_t>(1, (cap + kStage - 1) / kStage);
    int64_t nc = std::min<int64_t>(stages, std::max<int64_t>(1, (2048 + nqb - 1) / nqb));
    const int64_t per = (stages + nc - 1) / nc;  // stages per chunk
    chunk = (int32_t)(per * kStage);
    nchunk = (int32_t)((cap + chunk - 1) / chunk);
    if (nchunk < 1) nchunk = 1;
}

hipError_t launch_hill_shared(const SharedArgs &a, hipStream_t s)
{
    switch (a.D) {
    case 1: return launch_shared_d<1>(a, s);
    case 2: return launch_shared_d<2>(a, s);
    case 3: return launch_shared_d<3>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sx
