// Hill sum over ONE hill list shared by many query points (walkers sharing
// a bias, or arbitrary evaluation points such as training and
// certification samples of a surrogate).  Metadynamics bias, Sec. 2.1.5.
//
// Unlike the private-list sum, every hill is reused by every query, so the
// work is bound by VALU arithmetic, not by HBM:
//   * grid x: hill chunks (multiples of 256 hills, sized so that chunks x
//     query blocks fill the chip); grid y: blocks of 64 Q queries;
//   * the four wavefronts of a workgroup hold the same 64 Q queries (Q per
//     lane) and split every staged group of 256 hills in four, so a small
//     query set (a step's walkers) still gives several wavefronts per
//     SIMD; a fixed-order LDS reduction joins the four;
//   * staging converts each hill once: centres to FP64, scaled by
//     s_d = sqrt(log2(e) / (2 sigma_d^2)), so that a (hill, query) pair costs
//     the scaled displacement and its periodic wrap (FP64), the quadratic
//     form (FP64 FMAs), one v_exp_f32, and FP64 sums of e and e * dx: about
//     17 VALU operations for two CVs.  Summing the products e * dxi in FP32
//     would lose digits where the terms of dV/dxi cancel;
//   * periodicity is a template parameter (all, none, or per CV);
//   * each (chunk, query) partial has one writer; the finalize kernel sums a
//     query's chunks in chunk order (bitwise deterministic), forms dV/dxi,
//     and appends one hill per walker for a deposition step, in walker order.
#include "sx_internal.h"
#include "dev_gather.h"

namespace sx {
namespace {

constexpr int kStage = kBlock;  // hills staged in LDS at a time (one per lane)
constexpr int kQueryLanes = 64;  // queries of a block per Q

enum { kPerNone = 0, kPerAll = 1, kPerMixed = 2 };

template <int D, int Q, int PER>
__global__ void __launch_bounds__(kBlock) k_hill_shared(SharedArgs a)
{
    __shared__ double s_c[D][kStage];
    __shared__ float s_h[kStage];
    __shared__ double s_red[3][Q * (1 + D)][kQueryLanes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the step counter moves here (the finalize, which may deposit, reads it)
    if (a.count_step && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    const int32_t n = *a.count;
    const int64_t qb0 = (int64_t)blockIdx.y * kQueryLanes * Q;
    const int64_t nq = a.nq;
    double sc[D], per[D], iper[D];
    bool wrap[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        sc[d] = sqrt(0.7213475204444817 * a.inv_sig2[d]);  // log2(e) / 2 = 0.72134...
        wrap[d] = PER == kPerAll || (PER == kPerMixed && a.period[d] > 0.0);
        per[d] = a.period[d] * sc[d];
        iper[d] = a.inv_period[d] / sc[d];
    }
    double xs[Q][D];
    bool live[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t q = qb0 + lane + (int64_t)kQueryLanes * i;
        live[i] = q < nq;
#pragma unroll
        for (int d = 0; d < D; ++d) xs[i][d] = live[i] ? a.xi[q * D + d] * sc[d] : 0.0;
    }
    double acc[Q][1 + D];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[i][j] = 0.0;
    const int64_t h0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t hend = min((int64_t)n, h0 + a.chunk);
    for (int64_t s0 = h0; s0 < hend; s0 += kStage) {
        const int64_t k = s0 + threadIdx.x;
        const bool ok = k < hend;
#pragma unroll
        for (int d = 0; d < D; ++d) s_c[d][threadIdx.x] = ok ? (double)a.c[d][k] * sc[d] : 0.0;
        s_h[threadIdx.x] = ok ? a.h[k] : 0.f;  // zero height: no contribution
        __syncthreads();
        // this wavefront's quarter of the staged hills
        const int m = (int)min((int64_t)kStage, hend - s0);
        const int j0 = wave * 64, j1 = min(j0 + 64, m);
        for (int jb = j0; jb < j1; jb += 4) {
#pragma unroll
            for (int j = jb; j < jb + 4; ++j) {  // j < j0 + 64 <= kStage; past m: zero height
                double c[D];
#pragma unroll
                for (int d = 0; d < D; ++d) c[d] = s_c[d][j];
                const float h = s_h[j];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    double x[D], qd = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        x[d] = xs[i][d] - c[d];
                        if (wrap[d]) x[d] = fma(-per[d], rint(x[d] * iper[d]), x[d]);
                        qd = fma(x[d], x[d], qd);
                    }
                    const double e = (double)(h * __builtin_amdgcn_exp2f(-(float)qd));
                    acc[i][0] += e;
#pragma unroll
                    for (int d = 0; d < D; ++d) acc[i][1 + d] = fma(e, x[d], acc[i][1 + d]);
                }
            }
        }
        __syncthreads();
    }
    // join the four wavefronts in a fixed order (0 + 1 + 2 + 3)
    if (wave > 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int j = 0; j <= D; ++j) s_red[wave - 1][i * (1 + D) + j][lane] = acc[i][j];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int j = 0; j <= D; ++j) acc[i][j] += s_red[w][i * (1 + D) + j][lane];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!live[i]) continue;
        const int64_t q = qb0 + lane + (int64_t)kQueryLanes * i;
        double *p = a.partial + ((int64_t)blockIdx.x * a.nq + q) * 4;
        p[0] = acc[i][0];
#pragma unroll
        for (int d = 0; d < D; ++d) p[1 + d] = acc[i][1 + d] / sc[d];  // back to CV units
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
// w is the query's row (its walker, or its evaluation point)
template <int D>
__device__ __forceinline__ void shared_finish(const SharedArgs &a, int64_t w, const double (&acc)[1 + D],
                                              double (&dv)[D])
{
    const double V = acc[0];
    bool finite = isfinite(V);
    if (a.V_ws) a.V_ws[w] = V;
    if (a.V_out) a.V_out[w] = V;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        dv[d] = -acc[1 + d] * a.inv_sig2[d];
        finite = finite && isfinite(dv[d]);
        if (a.dV_ws) a.dV_ws[w * D + d] = dv[d];
        if (a.dV_out) a.dV_out[w * D + d] = dv[d];
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

// few chunks: one lane per query sums its chunks in order (no fallback mode)
template <int D>
__global__ void __launch_bounds__(kBlock) k_hill_shared_finalize(SharedArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0;
    for (int ch = 0; ch < a.nchunk; ++ch) {
        const double *p = a.partial + ((int64_t)ch * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
    double dv[D];
    shared_finish<D>(a, q, acc, dv);
    if (a.do_forces) {  // coefficients -dV/dxi; this lane owns the walker's atoms
        double coef[D];
#pragma unroll
        for (int d = 0; d < D; ++d) coef[d] = -dv[d];
        const float *Jw = a.J + q * a.nslots * 3;
        for (int u = 0; u < a.tabs.U; ++u) gather_atom(a.tabs, Jw, (int32_t)q, coef, a.F, u);
    }
}

// many chunks, or fallback sums: one workgroup per query (walker), lanes
// stride over the chunks and a fixed reduction tree combines them
// (deterministic); then the walker's force gather
template <int D>
__global__ void __launch_bounds__(kBlock) k_hill_shared_finalize_wg(SharedArgs a)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ double s_coef[D];
    const int64_t w = blockIdx.x, q = w;  // fallback mode: records per walker
    if (a.fb && !a.fb[w]) return;           // uniform per workgroup
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0;
    for (int ch = threadIdx.x; ch < a.nchunk; ch += kBlock) {
        const double *p = a.partial + ((int64_t)ch * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
    block_sum0<1 + D>(acc, lds);
    if (threadIdx.x == 0) {
        double dv[D];
        shared_finish<D>(a, w, acc, dv);
#pragma unroll
        for (int d = 0; d < D; ++d) s_coef[d] = -dv[d];
    }
    if (!a.do_forces) return;  // uniform
    __syncthreads();
    gather_forces(a.tabs, a.J + w * a.nslots * 3, (int32_t)w, s_coef, a.F);
}

// The same in one wavefront, for steps that gather forces through the
// table in kernel-argument form: every load is requested before the first
// wait (each lane's first chunk record -- lanes past the count re-read the
// last one and drop it, nchunk >= 1 -- the CV values, the deposit's count
// and step, and a table row per lane with its Jacobian rows and force; lanes
// past U re-read row U - 1 and store nothing); the records are summed
// lane-strided and combined by a butterfly (every lane ends with the same
// bits); lane 0 writes the outputs and deposits, lane u < U adds atom u's
// force.  No LDS, no barrier.
template <int D>
__global__ void __launch_bounds__(64) k_hill_shared_finalize_wave(SharedArgs a)
{
    const int64_t w = blockIdx.x, q = w;  // fallback mode: records per walker
    const int lane = threadIdx.x;
    if (a.fb && !a.fb[w]) return;  // uniform per workgroup
    const int nch = a.nchunk;
    double r0[1 + D];
    {
        const double *p = a.partial + ((int64_t)min(lane, nch - 1) * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) r0[j] = p[j];
    }
    double xi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xi[d] = a.xi[w * D + d];
    const bool dep_cnt = a.deposit == 1 && a.stride > 0;
    const int64_t dstep = dep_cnt ? *a.dstep : 0;
    const int32_t cnt = a.deposit ? *a.count : 0;
    SmallGather sg{0.f, 0.f, 0.f, nullptr};
    int nent = 0;
    int32_t cvq[kSmallPer];
    float jr[kSmallPer][3];
    small_rows(a.small, a.J + w * a.nslots * 3, a.F, a.tabs.atom_off[w], min(lane, a.small.U - 1), sg, nent, cvq, jr);
    // the first record kept or replaced by +0.0 through a bit mask, which
    // uses the loaded value on every lane (a select lets the load move
    // under a branch)
    const long long keep = lane < nch ? -1LL : 0LL;
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0 + __longlong_as_double(__double_as_longlong(r0[j]) & keep);
    for (int ch = lane + 64; ch < nch; ch += 64) {  // the same order as one loop from ch = lane
        const double *p = a.partial + ((int64_t)ch * a.nq + q) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j <= D; ++j)
        for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    double dv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) dv[d] = -acc[1 + d] * a.inv_sig2[d];
    if (lane == 0) {
        const double V = acc[0];
        bool finite = isfinite(V);
        if (a.V_ws) a.V_ws[w] = V;
        if (a.V_out) a.V_out[w] = V;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            finite = finite && isfinite(dv[d]);
            if (a.dV_ws) a.dV_ws[w * D + d] = dv[d];
            if (a.dV_out) a.dV_out[w * D + d] = dv[d];
            if (a.xi_out) a.xi_out[w * D + d] = xi[d];
        }
        if (!finite && a.flags) atomicOr(a.flags, kFlagNonFinite);
        bool dep = a.deposit == 2;
        if (dep_cnt) dep = (dstep - 1) % a.stride == 0;
        if (dep) {  // as shared_finish: walker order at count + w, all or none
            if ((int64_t)cnt + a.nq <= a.cap) {
                const int64_t k = (int64_t)cnt + w;
#pragma unroll
                for (int d = 0; d < D; ++d) a.c[d][k] = (float)xi[d];
                a.h[k] = (float)(a.inv_kdT > 0.0 ? a.height * exp(-V * a.inv_kdT) : a.height);
            } else if (w == 0) {
                atomicOr(a.flags, kFlagCapacity);
            }
        }
    }
    if (lane < a.small.U) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
        for (int qq = 0; qq < kSmallPer; ++qq) {
            double cf = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) cf = cvq[qq] == d ? -dv[d] : cf;
            fx += qq < nent ? cf * (double)jr[qq][0] : 0.0;
            fy += qq < nent ? cf * (double)jr[qq][1] : 0.0;
            fz += qq < nent ? cf * (double)jr[qq][2] : 0.0;
        }
        sg.dst[0] = sg.f0 + (float)fx;
        sg.dst[a.F.sk] = sg.f1 + (float)fy;
        sg.dst[2 * a.F.sk] = sg.f2 + (float)fz;
    }
}

// Fallback sums of a surrogate step (the few walkers outside certified
// cells): workgroup (c, y) sums chunk c of kQmChunk hills for its walkers,
// lanes over hills with float4 loads all issued before use (the chunk is
// read from L2 once per workgroup and kept in registers for all of its
// walkers), a fixed-order reduction, one partial record per (chunk,
// walker); the finalize kernel then sums a walker's chunks in order.
// COMPACT (at most kQmCompactMax queries): gridDim.y = min(queries,
// kQmSlots) rows, row y taking the flagged walkers of rank y, y + rows, ...
// in walker order, so the grid does not grow with the walkers the network
// serves; otherwise row y is walker y and leaves at once unless flagged.
// A walker's records do not depend on which workgroup formed them.
constexpr int kQmChunk = 4096;               // hills per workgroup
constexpr int kQmGroups = kQmChunk / (4 * kBlock);  // float4 groups per lane
constexpr int kQmSlots = 32;                 // workgroup rows of the compacted grid
constexpr int kQmCompactMax = 1024;          // largest query count it serves
constexpr int kQmPerRow = kQmCompactMax / kQmSlots;  // walkers one row takes at most

template <int D, int PER, bool COMPACT>
__global__ void __launch_bounds__(kBlock) k_hill_shared_qm(SharedArgs a)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ int32_t s_list[COMPACT ? kQmPerRow : 1];
    __shared__ int32_t s_nw;
    if (a.count_step && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    int nw = 1;
    if (COMPACT) {
        // wavefront 0 ranks the flagged walkers in order and lists this row's
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const unsigned long long below = (1ull << lane) - 1ull;
            int base = 0, mine = 0;
            for (int64_t b0 = 0; b0 < a.nq; b0 += 64) {
                const int64_t ww = b0 + lane;
                const bool f = ww < a.nq && a.fb[ww];
                const unsigned long long m = __ballot(f);
                const bool take = f && (base + __popcll(m & below)) % (int)gridDim.y == (int)blockIdx.y;
                const unsigned long long mt = __ballot(take);
                if (take) s_list[mine + __popcll(mt & below)] = (int32_t)ww;  // < kQmPerRow: at most nq / rows
                mine += __popcll(mt);
                base += __popcll(m);
            }
            if (lane == 0) s_nw = mine;
        }
        __syncthreads();
        nw = s_nw;
    } else if (!a.fb[blockIdx.y]) {
        return;  // uniform per workgroup
    }
    if (nw == 0) return;  // uniform
    const int32_t n = *a.count;
    const int64_t h0 = (int64_t)blockIdx.x * kQmChunk;
    if (h0 >= n) {  // uniform: a chunk past the count adds zero (the finalize sums every chunk)
        for (int iw = 0; iw < nw; ++iw) {
            const int64_t w = COMPACT ? (int64_t)s_list[iw] : (int64_t)blockIdx.y;
            if (threadIdx.x <= D) a.partial[((int64_t)blockIdx.x * a.nq + w) * 4 + threadIdx.x] = 0.0;
        }
        return;
    }
    double sc[D], per[D], iper[D];
    bool wrap[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        sc[d] = sqrt(0.7213475204444817 * a.inv_sig2[d]);
        wrap[d] = PER == kPerAll || (PER == kPerMixed && a.period[d] > 0.0);
        per[d] = a.period[d] * sc[d];
        iper[d] = a.inv_period[d] / sc[d];
    }
    // groups of 4 hills; the list's storage is padded to a multiple of 4
    // floats and 16-byte aligned: a group past the count reads group 0 and
    // gets zero heights
    float4 cv[kQmGroups][D], hv[kQmGroups];
    int64_t kk[kQmGroups];
#pragma unroll
    for (int it = 0; it < kQmGroups; ++it) {
        const int64_t k = h0 + 4 * ((int64_t)it * kBlock + threadIdx.x);
        kk[it] = k;
        const int64_t ks = k < n ? k : 0;
#pragma unroll
        for (int d = 0; d < D; ++d) cv[it][d] = *reinterpret_cast<const float4 *>(a.c[d] + ks);
        hv[it] = *reinterpret_cast<const float4 *>(a.h + ks);
    }
    for (int iw = 0; iw < nw; ++iw) {
        const int64_t w = COMPACT ? (int64_t)s_list[iw] : (int64_t)blockIdx.y;
        double xs[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xs[d] = a.xi[w * D + d] * sc[d];
        double acc[1 + D];
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] = 0.0;
#pragma unroll
        for (int it = 0; it < kQmGroups; ++it) {
            const int64_t k = kk[it];
            const float hh[4] = {k < n ? hv[it].x : 0.f, k + 1 < n ? hv[it].y : 0.f, k + 2 < n ? hv[it].z : 0.f,
                                 k + 3 < n ? hv[it].w : 0.f};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double x[D], qd = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const float4 &c4 = cv[it][d];
                    const float c = j == 0 ? c4.x : (j == 1 ? c4.y : (j == 2 ? c4.z : c4.w));
                    x[d] = xs[d] - (double)c * sc[d];
                    if (wrap[d]) x[d] = fma(-per[d], rint(x[d] * iper[d]), x[d]);
                    qd = fma(x[d], x[d], qd);
                }
                const double e = (double)(hh[j] * __builtin_amdgcn_exp2f(-(float)qd));
                acc[0] += e;
#pragma unroll
                for (int d = 0; d < D; ++d) acc[1 + d] = fma(e, x[d], acc[1 + d]);
            }
        }
        block_sum0<1 + D>(acc, lds);  // ends with a barrier: lds is free for the next walker
        if (threadIdx.x == 0) {
            double *p = a.partial + ((int64_t)blockIdx.x * a.nq + w) * 4;
            p[0] = acc[0];
#pragma unroll
            for (int d = 0; d < D; ++d) p[1 + d] = acc[1 + d] / sc[d];  // back to CV units
        }
    }
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

// the one-wavefront finalize: forces through the kernel-argument table of
// walkers (one query per walker, its records at query w)
bool small_finalize(const SharedArgs &a)
{
    return a.do_forces && a.small.on && a.small.U > 0 && a.nchunk >= 1 && a.tabs.W == a.nq;
}

template <int D>
hipError_t launch_shared_d(const SharedArgs &a, hipStream_t s)
{
    if (a.fb) {  // fallback walkers of a surrogate step: query-major sums, finalize per walker
        SharedArgs b = a;
        b.chunk = kQmChunk;
        b.nchunk = (int32_t)std::max<int64_t>(1, (a.cap + kQmChunk - 1) / kQmChunk);
        bool any = false, all = true;
        for (int d = 0; d < D; ++d) {
            any = any || a.period[d] > 0.0;
            all = all && a.period[d] > 0.0;
        }
        const int per = all ? kPerAll : (any ? kPerMixed : kPerNone);
        if (a.nq <= kQmCompactMax) {
            const dim3 g(b.nchunk, (unsigned)std::min<int64_t>(a.nq, kQmSlots));
            if (per == kPerAll) hipLaunchKernelGGL((k_hill_shared_qm<D, kPerAll, true>), g, dim3(kBlock), 0, s, b);
            else if (per == kPerNone) hipLaunchKernelGGL((k_hill_shared_qm<D, kPerNone, true>), g, dim3(kBlock), 0, s, b);
            else hipLaunchKernelGGL((k_hill_shared_qm<D, kPerMixed, true>), g, dim3(kBlock), 0, s, b);
        } else {
            const dim3 g(b.nchunk, (unsigned)a.nq);
            if (per == kPerAll) hipLaunchKernelGGL((k_hill_shared_qm<D, kPerAll, false>), g, dim3(kBlock), 0, s, b);
            else if (per == kPerNone) hipLaunchKernelGGL((k_hill_shared_qm<D, kPerNone, false>), g, dim3(kBlock), 0, s, b);
            else hipLaunchKernelGGL((k_hill_shared_qm<D, kPerMixed, false>), g, dim3(kBlock), 0, s, b);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (small_finalize(b))
            hipLaunchKernelGGL((k_hill_shared_finalize_wave<D>), dim3((unsigned)a.nq), dim3(64), 0, s, b);
        else
            hipLaunchKernelGGL((k_hill_shared_finalize_wg<D>), dim3((unsigned)a.nq), dim3(kBlock), 0, s, b);
        return hipGetLastError();
    }
    // queries per lane: 1 for small query sets (more workgroups), 4 for many
    const int Q = a.nq >= 65536 ? 4 : 1;
    dim3 grid(a.nchunk, (unsigned)((a.nq + kQueryLanes * Q - 1) / (kQueryLanes * Q)));
    bool any = false, all = true;
    for (int d = 0; d < D; ++d) {
        any = any || a.period[d] > 0.0;
        all = all && a.period[d] > 0.0;
    }
    const int per = all ? kPerAll : (any ? kPerMixed : kPerNone);
#define SX_SHARED_LAUNCH(QQ, PP) hipLaunchKernelGGL((k_hill_shared<D, QQ, PP>), grid, dim3(kBlock), 0, s, a)
    if (Q == 4) {
        if (per == kPerAll) SX_SHARED_LAUNCH(4, kPerAll);
        else if (per == kPerNone) SX_SHARED_LAUNCH(4, kPerNone);
        else SX_SHARED_LAUNCH(4, kPerMixed);
    } else {
        if (per == kPerAll) SX_SHARED_LAUNCH(1, kPerAll);
        else if (per == kPerNone) SX_SHARED_LAUNCH(1, kPerNone);
        else SX_SHARED_LAUNCH(1, kPerMixed);
    }
#undef SX_SHARED_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nchunk >= 32 && small_finalize(a))
        hipLaunchKernelGGL((k_hill_shared_finalize_wave<D>), dim3((unsigned)a.nq), dim3(64), 0, s, a);
    else if (a.nchunk >= 32)
        hipLaunchKernelGGL((k_hill_shared_finalize_wg<D>), dim3((unsigned)a.nq), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_hill_shared_finalize<D>), dim3((unsigned)((a.nq + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.deposit == 2 || (a.deposit == 1 && a.stride > 0)) {
        hipLaunchKernelGGL(k_shared_count, dim3(1), dim3(64), 0, s, a);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

void shared_split(int64_t cap, int64_t nq, int32_t &chunk, int32_t &nchunk, int32_t target)
{
    const int Q = nq >= 65536 ? 4 : 1;
    const int64_t nqb = std::max<int64_t>(1, (nq + (int64_t)kQueryLanes * Q - 1) / ((int64_t)kQueryLanes * Q));
    const int64_t stages = std::max<int64_t>(1, (cap + kStage - 1) / kStage);
    // about `target` workgroups (chunks x query blocks), at least one stage each
    int64_t nc = std::min<int64_t>(stages, std::max<int64_t>(1, (target + nqb - 1) / nqb));
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
