// Bias kernels: the metadynamics hill sum with well-tempered deposition
// (Sec. 2.1.5) and the atomic-free force gather that adds a bias to the
// engine's forces (Sec. 2).
//
// Hill sum over private hill lists (one list per walker), two kernels:
//   A  k_hill_tiles: a static table of tiles (walker, first hill), each
//      1024 * U hills of one walker's capacity.  A tile at or past the
//      walker's current hill count leaves at once, so the work follows the
//      hills deposited so far, not the space reserved for them.  Hills are
//      stored SoA in float32 (centres c[d][k], heights h[k]); every lane
//      issues its non-temporal float4 loads of a batch of 4 groups before
//      using any of them (clamped to the group of the walker's last hill and masked by
//      its count, so no branch sits between the loads), which keeps enough
//      bytes in flight to stream HBM.
//      When every CV is a dihedral the tile's workgroup computes its
//      walker's xi itself (FP64) while its hill loads are in flight, so no
//      separate CV kernel runs.  The displacement and its periodic wrap are
//      formed in FP64 (the same VALU rate as FP32 on CDNA4 without packed
//      math), the Gaussian in FP32 with the hardware exp2, the sums in FP64
//      per group of 4 hills.  Each tile writes its partial (V, sum e D_d) to
//      its own record.
//   B  k_hill_finalize: one workgroup per walker reduces that walker's live
//      tile records in tile order (bitwise deterministic whatever the schedule),
//      forms dV/dxi, writes the outputs, deposits the well-tempered hill and
//      gathers the force onto the walker's atoms.  The kernel boundary is the
//      only cross-workgroup synchronisation: no fences, no atomics.
#include "dev_cv.h"
#include "dev_gather.h"
#include "dev_reduce.h"

namespace sx {
namespace {


// Gaussian term of one hill: returns h exp(-sum_d D_d^2/(2 sigma_d^2)) and
// the wrapped displacements D_d (float).  The difference xi - c and its
// minimum image are formed in FP64 so that D_d carries only the final
// rounding to float.
template <int D>
__device__ __forceinline__ float hill_term(const double (&xi)[D], const float (&c)[D], float h, const HillArgs &a,
                                           float (&dl)[D])
{
    float q = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double x = xi[d] - (double)c[d];
        x = fma(-a.period[d], rint(x * a.inv_period[d]), x);
        dl[d] = (float)x;
        q = fmaf(dl[d] * a.a2[d], dl[d], q);
    }
    return h * __builtin_amdgcn_exp2f(-q);
}

// Streaming load of one float4 group of a hill list: non-temporal, so the
// list (read once per step, far larger than the L2) does not displace the
// small tables, records and positions that the step's kernels reuse.
typedef float nt_f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4 *p)
{
    const nt_f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f32x4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float comp(const float4 &v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

constexpr int kBatch = 8;  // float4 groups loaded per lane before use

// Dihedral `cv` (CV index d) of the tile's walker, FP64.  Writes xi to the
// workgroup's LDS slot; the walker's first tile also keeps xi and the
// Jacobian rows in the workspace for kernel B.
// Loads through the constant address space: the value is the same for the
// whole workgroup and does not change while the kernel runs, so it comes
// through the scalar cache into SGPRs.
template <typename T>
__device__ __forceinline__ T ld_uniform(const T *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) T *)(p);
#else
    return *p;
#endif
}

// Lane d (< D) of wave 0 evaluates dihedral d of the tile's walker (FP64):
// first its four positions are requested (atom indices selected from the
// kernel arguments with selects, not loads), then -- after the hill loads
// of the tile are in flight -- the angle is computed.  The walker's first
// tile also keeps xi and the Jacobian rows in the workspace for kernel B.
template <int D>
__device__ __forceinline__ int32_t dihedral_atom(const CvSet &cs, int d, int q)
{
    int32_t at = cs.cv[0].atom[q];
#pragma unroll
    for (int dd = 1; dd < D; ++dd) at = d == dd ? cs.cv[dd].atom[q] : at;
    return at;
}

// Raw coordinates of a dihedral's four atoms as loaded (T: the position
// type); conversion waits until the values are used, so the loads stay in
// flight while the hill loads are issued.
template <typename T>
struct RawAtoms {
    T v[12];
};

template <int D, typename T>
__device__ __forceinline__ void fetch_dihedral_atoms(const CvSet &cs, const PosView &pos, int64_t aoff,
                                                     RawAtoms<T> &ra)
{
    const int d = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const T *p = static_cast<const T *>(pos.ptr) + (aoff + dihedral_atom<D>(cs, d, q)) * pos.sa;
        ra.v[3 * q + 0] = p[0];
        ra.v[3 * q + 1] = p[pos.sk];
        ra.v[3 * q + 2] = p[2 * pos.sk];
    }
}

template <int D, typename T>
__device__ __forceinline__ void finish_dihedral(const HillArgs &a, const CvSet &cs, const TileRec &tr,
                                                const RawAtoms<T> &ra, double *s_xi)
{
    const int d = threadIdx.x;
    T v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        v[k] = ra.v[k];
        asm volatile("" : "+v"(v[k]));  // keep the use (and the wait) here, after the hill loads
    }
    double3 r[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = make_double3((double)v[3 * q], (double)v[3 * q + 1], (double)v[3 * q + 2]);
    if (tr.h0 == 0 && a.do_forces) {
        int32_t slot0 = cs.cv[0].slot0;
#pragma unroll
        for (int dd = 1; dd < D; ++dd) slot0 = d == dd ? cs.cv[dd].slot0 : slot0;
        const double phi = dihedral_fp64<true>(r, g);
        s_xi[d] = phi;
        a.xi_save[(int64_t)tr.w * D + d] = phi;
        float *J = a.J + ((int64_t)tr.w * a.nslots + slot0) * 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            J[q * 3 + 0] = (float)g[q].x;
            J[q * 3 + 1] = (float)g[q].y;
            J[q * 3 + 2] = (float)g[q].z;
        }
    } else {
        const double phi = dihedral_fp64<false>(r, g);
        s_xi[d] = phi;
        if (tr.h0 == 0) a.xi_save[(int64_t)tr.w * D + d] = phi;
    }
}

// Kernel A.  One tile per loop trip (persistent when the grid is smaller
// than the tile count).  Load pattern per lane and batch: UB float4 of each
// centre array and of the heights at float4 index q0 + u * kBlock, from
// uniform (scalar) base pointers with 32-bit lane offsets; the scheduling
// barrier keeps every load of the batch ahead of the arithmetic.
// One tile: partial (V, sum e D_d) of hills [h0, h0 + 1024 U) of one walker,
// stored as the tile's record and left in thread 0's `sum`.
template <int D, int U, bool FUSE, typename T>
__device__ __forceinline__ void hill_tile(const HillArgs &a, const CvSet &cs, const PosView &pos, int t, double *lds,
                                          double *s_xi, double (&sum)[1 + D])
{
    constexpr int UB = U < kBatch ? U : kBatch;
        const TileRec tr = ld_uniform(a.tiles + t);
        const int64_t aoff = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(tr.aoff_hi) << 32) |
                                       (uint32_t)__builtin_amdgcn_readfirstlane(tr.aoff_lo));
        const int32_t w = tr.w;
        const int32_t n = ld_uniform(a.count + w);
        // a tile at or past the walker's hill count has nothing to add and
        // leaves on a uniform branch (kernel B reads only the live tiles);
        // the first tile always runs: it also evaluates fused CVs
        if (tr.h0 > 0 && tr.h0 >= n) return;
        const int64_t hb = (int64_t)tr.hb4 * 4;
        const float4 *cb[D];
#pragma unroll
        for (int d = 0; d < D; ++d) cb[d] = reinterpret_cast<const float4 *>(a.c[d] + hb);
        const float4 *hp = reinterpret_cast<const float4 *>(a.h + hb);
        const uint32_t q0 = (uint32_t)(tr.h0 / kHillsPerLoad) + threadIdx.x;
        // loads are clamped to the float4 group of the last live hill (group
        // 0 of an empty list), so no lane streams the empty capacity; the
        // tile record's klast bounds the walker's capacity
        const uint32_t qlast = min((uint32_t)(tr.klast / kHillsPerLoad),
                                   n > 0 ? (uint32_t)(n - 1) / kHillsPerLoad : 0u);
        // fused CVs: lane d of wave 0 requests the positions of dihedral d
        // before the hill loads, computes the angle (FP64) while those are
        // in flight, and meets the other waves at the barrier below
        const bool cv_lane = FUSE && (int)threadIdx.x < D;
        RawAtoms<T> ra;
        if (cv_lane) fetch_dihedral_atoms<D, T>(cs, pos, aoff, ra);
        __builtin_amdgcn_sched_barrier(0);
        double xi[D];
        double acc[1 + D];
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] = 0.0;
#pragma unroll
        for (int ub = 0; ub < U; ub += UB) {
            float4 cv[UB][D], hv[UB];
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                const uint32_t qi = min(q0 + (uint32_t)((ub + q) * kBlock), qlast);
#pragma unroll
                for (int d = 0; d < D; ++d) cv[q][d] = ld_stream(&cb[d][qi]);
                hv[q] = ld_stream(&hp[qi]);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (ub == 0) {
                if (FUSE) {
                    if (cv_lane) finish_dihedral<D, T>(a, cs, tr, ra, s_xi);
                    __syncthreads();
#pragma unroll
                    for (int d = 0; d < D; ++d) xi[d] = s_xi[d];
                } else {
#pragma unroll
                    for (int d = 0; d < D; ++d) xi[d] = a.xi[(int64_t)w * D + d];
                }
            }
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                const int32_t k = (int32_t)(q0 + (uint32_t)((ub + q) * kBlock)) * kHillsPerLoad;
                float sv = 0.f, sg[D];
#pragma unroll
                for (int d = 0; d < D; ++d) sg[d] = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float c[D], dl[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) c[d] = comp(cv[q][d], i);
                    float e = hill_term<D>(xi, c, comp(hv[q], i), a, dl);
                    e = (k + i < n) ? e : 0.f;
                    sv += e;
#pragma unroll
                    for (int d = 0; d < D; ++d) sg[d] = fmaf(e, dl[d], sg[d]);
                }
                acc[0] += (double)sv;
#pragma unroll
                for (int d = 0; d < D; ++d) acc[1 + d] += (double)sg[d];
            }
        }
        block_sum0<1 + D>(acc, lds);
        if (threadIdx.x == 0) {
            double *p = a.partial + (int64_t)t * 4;
#pragma unroll
            for (int j = 0; j <= D; ++j) p[j] = acc[j];
        }
#pragma unroll
        for (int j = 0; j <= D; ++j) sum[j] = acc[j];
}

// One workgroup per tile: the tile record is read before any store, so it
// comes through the scalar cache.
template <int D, int U, bool FUSE, typename T>
__global__ void __launch_bounds__(kBlock) k_hill_tiles(HillArgs a, CvSet cs, PosView pos)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ double s_xi[D];
    if (a.count_step && blockIdx.x == 0 && threadIdx.x == 0) *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    double sum[1 + D];
    hill_tile<D, U, FUSE, T>(a, cs, pos, blockIdx.x, lds, s_xi, sum);
}

// Persistent grid: each workgroup strides over the tiles.
template <int D, int U, bool FUSE, typename T>
__global__ void __launch_bounds__(kBlock) k_hill_tiles_persist(HillArgs a, CvSet cs, PosView pos)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ double s_xi[D];
    if (a.count_step && blockIdx.x == 0 && threadIdx.x == 0) *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        double sum[1 + D];
        hill_tile<D, U, FUSE, T>(a, cs, pos, __builtin_amdgcn_readfirstlane(t), lds, s_xi, sum);
        __syncthreads();  // lds / s_xi reuse by the next tile
    }
}

// Tiles of a walker that kernel A ran: those starting below its hill count
// (at least the first).  Kernel A saw the same count: nothing changes it
// between the two kernels.
__device__ __forceinline__ int32_t live_tiles(const HillArgs &a, const WalkerRec &wr, int32_t cnt)
{
    const int32_t T = a.tile_units * kTileUnit;
    return min(wr.nt, max(1, (cnt + T - 1) / T));
}

// Kernel B's work once the walker's sum is in thread 0's acc: V, dV/dxi and
// the outputs, the deposit (thread 0), then the forces (every thread; the
// small table's rows were requested by lanes u < U before the sum).
template <int D>
__device__ __forceinline__ void finalize_tail(const HillArgs &a, int32_t w, const WalkerRec &wr, int32_t cnt0,
                                              int64_t next_step, const double (&acc)[1 + D], const double *s_xi,
                                              double *s_coef, bool small_lane, const SmallGather &sg, int nent,
                                              const int32_t (&cvq)[kSmallPer], const float (&jr)[kSmallPer][3])
{
    if (threadIdx.x == 0) {
        const double V = acc[0];
        bool finite = isfinite(V);
        a.V_ws[w] = V;
        if (a.V_out) a.V_out[w] = V;
        if (a.xi_out)
#pragma unroll
            for (int d = 0; d < D; ++d) a.xi_out[(int64_t)w * D + d] = s_xi[d];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double dv = -acc[1 + d] * a.inv_sig2[d];
            finite = finite && isfinite(dv);
            a.dV_ws[(int64_t)w * D + d] = dv;
            if (a.dV_out) a.dV_out[(int64_t)w * D + d] = dv;
            s_coef[d] = -dv;
        }
        if (!finite) atomicOr(a.flags, kFlagNonFinite);
        bool dep = a.deposit == 2;
        if (a.deposit == 1 && a.stride > 0) dep = (next_step - 1) % a.stride == 0;  // kernel A set the counter
        if (dep) {
            const int32_t cnt = cnt0;
            if (cnt < wr.cap) {
                const int64_t k = (int64_t)wr.hb4 * 4 + cnt;
#pragma unroll
                for (int d = 0; d < D; ++d) a.c[d][k] = (float)s_xi[d];
                a.h[k] = (float)(a.inv_kdT > 0.0 ? a.height * exp(-V * a.inv_kdT) : a.height);
                a.count[w] = cnt + 1;
            } else {
                atomicOr(a.flags, kFlagCapacity);
            }
        }
    }
    __syncthreads();
    if (!a.do_forces) return;
    if (a.small.on) {
        if (small_lane) {
            double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
            for (int q = 0; q < kSmallPer; ++q) {
                const double cf = s_coef[cvq[q]];
                fx += q < nent ? cf * (double)jr[q][0] : 0.0;
                fy += q < nent ? cf * (double)jr[q][1] : 0.0;
                fz += q < nent ? cf * (double)jr[q][2] : 0.0;
            }
            sg.dst[0] = sg.f0 + (float)fx;
            sg.dst[a.F.sk] = sg.f1 + (float)fy;
            sg.dst[2 * a.F.sk] = sg.f2 + (float)fz;
        }
    } else {
        gather_forces(a.tabs, a.J + (int64_t)w * a.nslots * 3, w, s_coef, a.F);
    }
}

template <int D, bool FUSE>
__global__ void __launch_bounds__(kBlock) k_hill_finalize(HillArgs a, CvSet cs, PosView pos)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ double s_coef[kMaxCv];
    __shared__ double s_xi[kMaxBiasDim];
    const int32_t w = blockIdx.x;
    const WalkerRec wr = ld_uniform(a.wrec + w);
    // values thread 0 needs after the reduction, requested up front; the
    // step counter was set by kernel A and is constant during this kernel
    const int64_t next_step = a.deposit == 1 ? ld_uniform(a.dstep) : 0;
    const int32_t cnt0 = ld_uniform(a.count + w);
    const int32_t nlive = live_tiles(a, wr, cnt0);
    // small gather table: lane u < U requests its atom's force and the
    // Jacobian rows it will combine before the reduction, so that only the
    // multiply-adds and the stores follow the barrier
    const bool small_lane = a.do_forces && a.small.on && (int)threadIdx.x < a.small.U;
    SmallGather sg{0.f, 0.f, 0.f, nullptr};
    int nent = 0;
    int32_t cvq[kSmallPer];
    float jr[kSmallPer][3];
    if (small_lane)
        small_rows(a.small, a.J + (int64_t)w * a.nslots * 3, a.F, wr.aoff, threadIdx.x, sg, nent, cvq, jr);
    if ((int)threadIdx.x < D) s_xi[threadIdx.x] = (FUSE ? a.xi_save : a.xi)[(int64_t)w * D + threadIdx.x];
    double acc[1 + D];
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0;
    for (int i = threadIdx.x; i < nlive; i += kBlock) {
        const double *p = a.partial + (int64_t)(wr.t0 + i) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
    block_sum0<1 + D>(acc, lds);  // also orders the s_xi writes
    finalize_tail<D>(a, w, wr, cnt0, next_step, acc, s_xi, s_coef, small_lane, sg, nent, cvq, jr);
}

// The same finalize in one wavefront, for steps that gather forces through a
// table small enough for the kernel arguments (at most 32 touched atoms, 8
// slots each): the tile records are summed by a fixed butterfly across the
// wavefront (every lane ends with the same bits, as each lane adds in the
// same order), every lane forms dV/dxi itself, lane 0 writes the outputs and
// deposits, and lane u < U gathers atom u's force -- no LDS and no barrier
// on the path.
template <int D, bool FUSE>
__global__ void __launch_bounds__(64) k_hill_finalize_wave(HillArgs a, CvSet cs, PosView pos)
{
    const int32_t w = blockIdx.x;
    const int lane = threadIdx.x;
    const WalkerRec wr = ld_uniform(a.wrec + w);
    const int64_t next_step = a.deposit == 1 ? ld_uniform(a.dstep) : 0;
    const int32_t cnt0 = ld_uniform(a.count + w);  // scalar: no vector wait
    const int32_t nlive = live_tiles(a, wr, cnt0);
    const bool small_lane = lane < a.small.U;  // launched only when forces are gathered
    SmallGather sg{0.f, 0.f, 0.f, nullptr};
    int nent = 0;
    int32_t cvq[kSmallPer];
    float jr[kSmallPer][3];
    // requested before anything waits, with no branch between the loads:
    // the first tile record of each lane (lanes past the walker's live tiles
    // re-read a record inside its table, nt >= 1, and drop it), the CV values, and a
    // small-table row per lane (lanes past U re-read row U - 1 and store
    // nothing)
    double acc[1 + D];
    double r0[1 + D];
    {
        const double *p = a.partial + (int64_t)(wr.t0 + min(lane, wr.nt - 1)) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) r0[j] = p[j];
    }
    double xi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xi[d] = (FUSE ? a.xi_save : a.xi)[(int64_t)w * D + d];
    small_rows(a.small, a.J + (int64_t)w * a.nslots * 3, a.F, wr.aoff, min(lane, a.small.U - 1), sg, nent, cvq, jr);
    // the record is kept or replaced by +0.0 through a bit mask, which uses
    // the loaded value on every lane (a select lets the load move under a branch)
    const long long keep = lane < nlive ? -1LL : 0LL;
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = 0.0 + __longlong_as_double(__double_as_longlong(r0[j]) & keep);
    for (int i = lane + 64; i < nlive; i += 64) {  // the same order as one loop from i = lane
        const double *p = a.partial + (int64_t)(wr.t0 + i) * 4;
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j <= D; ++j)
        for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    // every lane now holds the sums; take lane 0's bits so all agree
#pragma unroll
    for (int j = 0; j <= D; ++j) acc[j] = __shfl(acc[j], 0, 64);
    double coef[D];
#pragma unroll
    for (int d = 0; d < D; ++d) coef[d] = acc[1 + d] * a.inv_sig2[d];  // -dV/dxi
    if (lane == 0) {
        const double V = acc[0];
        bool finite = isfinite(V);
        a.V_ws[w] = V;
        if (a.V_out) a.V_out[w] = V;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double dv = -coef[d];
            finite = finite && isfinite(dv);
            a.dV_ws[(int64_t)w * D + d] = dv;
            if (a.dV_out) a.dV_out[(int64_t)w * D + d] = dv;
            if (a.xi_out) a.xi_out[(int64_t)w * D + d] = xi[d];
        }
        if (!finite) atomicOr(a.flags, kFlagNonFinite);
        bool dep = a.deposit == 2;
        if (a.deposit == 1 && a.stride > 0) dep = (next_step - 1) % a.stride == 0;  // kernel A set the counter
        if (dep) {
            if (cnt0 < wr.cap) {
                const int64_t k = (int64_t)wr.hb4 * 4 + cnt0;
#pragma unroll
                for (int d = 0; d < D; ++d) a.c[d][k] = (float)xi[d];
                a.h[k] = (float)(a.inv_kdT > 0.0 ? a.height * exp(-V * a.inv_kdT) : a.height);
                a.count[w] = cnt0 + 1;
            } else {
                atomicOr(a.flags, kFlagCapacity);
            }
        }
    }
    if (small_lane) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
        for (int q = 0; q < kSmallPer; ++q) {
            double cf = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) cf = cvq[q] == d ? coef[d] : cf;
            fx += q < nent ? cf * (double)jr[q][0] : 0.0;
            fy += q < nent ? cf * (double)jr[q][1] : 0.0;
            fz += q < nent ? cf * (double)jr[q][2] : 0.0;
        }
        sg.dst[0] = sg.f0 + (float)fx;
        sg.dst[a.F.sk] = sg.f1 + (float)fy;
        sg.dst[2 * a.F.sk] = sg.f2 + (float)fz;
    }
}

// The whole step in one launch when all the hills are one tile (one walker
// whose capacity fits a tile): the workgroup sums the tile, then does kernel
// B's work on its own sum -- the same bits kernel B would form from the one
// record -- with the Jacobian rows and CV values it wrote itself (visible to
// it after the sum's barriers) and the step counter it set itself.
template <int D, int U, bool FUSE, typename T>
__global__ void __launch_bounds__(kBlock) k_hill_step_one_tile(HillArgs a, CvSet cs, PosView pos)
{
    __shared__ double lds[(1 + D) * (kBlock / 64)];
    __shared__ double s_xi[kMaxBiasDim];
    __shared__ double s_coef[kMaxCv];
    int64_t next_step = 0;  // thread 0 alone decides the deposit
    if (threadIdx.x == 0) {
        if (a.count_step) {
            next_step = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
            *a.dstep = next_step;
        } else if (a.deposit == 1) {
            next_step = *a.dstep;
        }
    }
    double acc[1 + D];
    hill_tile<D, U, FUSE, T>(a, cs, pos, 0, lds, s_xi, acc);
    const WalkerRec wr = ld_uniform(a.wrec);
    const int32_t cnt0 = ld_uniform(a.count);  // what the tile saw: only the deposit below changes it
    const bool small_lane = a.do_forces && a.small.on && (int)threadIdx.x < a.small.U;
    SmallGather sg{0.f, 0.f, 0.f, nullptr};
    int nent = 0;
    int32_t cvq[kSmallPer];
    float jr[kSmallPer][3];
    if (small_lane) small_rows(a.small, a.J, a.F, wr.aoff, threadIdx.x, sg, nent, cvq, jr);
    if (!FUSE) {
        if ((int)threadIdx.x < D) s_xi[threadIdx.x] = a.xi[threadIdx.x];
        __syncthreads();
    }
    finalize_tail<D>(a, 0, wr, cnt0, next_step, acc, s_xi, s_coef, small_lane, sg, nent, cvq, jr);
}

template <int D, bool FUSE, typename T>
hipError_t launch_step_one_tile(const HillArgs &a, const CvSet &cs, const PosView &pos, hipStream_t s)
{
    switch (a.tile_units) {
    case 1: hipLaunchKernelGGL((k_hill_step_one_tile<D, 1, FUSE, T>), dim3(1), dim3(kBlock), 0, s, a, cs, pos); break;
    case 2: hipLaunchKernelGGL((k_hill_step_one_tile<D, 2, FUSE, T>), dim3(1), dim3(kBlock), 0, s, a, cs, pos); break;
    case 4: hipLaunchKernelGGL((k_hill_step_one_tile<D, 4, FUSE, T>), dim3(1), dim3(kBlock), 0, s, a, cs, pos); break;
    case 8: hipLaunchKernelGGL((k_hill_step_one_tile<D, 8, FUSE, T>), dim3(1), dim3(kBlock), 0, s, a, cs, pos); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int D, bool FUSE, typename T>
hipError_t launch_tiles(const HillArgs &a, const CvSet &cs, const PosView &pos, int32_t g, hipStream_t s)
{
    const bool persist = g < a.ntiles;
#define SX_TILE_CASE(UU)                                                                                          \
    case UU:                                                                                                      \
        if (persist)                                                                                              \
            hipLaunchKernelGGL((k_hill_tiles_persist<D, UU, FUSE, T>), dim3(g), dim3(kBlock), 0, s, a, cs, pos); \
        else                                                                                                      \
            hipLaunchKernelGGL((k_hill_tiles<D, UU, FUSE, T>), dim3(g), dim3(kBlock), 0, s, a, cs, pos);         \
        break;
    switch (a.tile_units) {
        SX_TILE_CASE(1)
        SX_TILE_CASE(2)
        SX_TILE_CASE(4)
        SX_TILE_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef SX_TILE_CASE
    return hipGetLastError();
}

template <int D, bool FUSE>
hipError_t launch_hill_d(const HillArgs &a, const CvSet &cs, const PosView &pos, int32_t grid, hipStream_t s,
                         int which)
{
    const int g = (grid > 0 && grid < a.ntiles) ? grid : a.ntiles;
    if (which == 3 && a.ntiles == 1)
        return (FUSE && pos.f64) ? launch_step_one_tile<D, FUSE, double>(a, cs, pos, s)
                                 : launch_step_one_tile<D, FUSE, float>(a, cs, pos, s);
    if (which & 1) {
        hipError_t e = (FUSE && pos.f64) ? launch_tiles<D, FUSE, double>(a, cs, pos, g, s)
                                         : launch_tiles<D, FUSE, float>(a, cs, pos, g, s);
        if (e != hipSuccess) return e;
    }
    if (which & 2) {
        if (a.small.on && a.do_forces && a.small.U > 0)
            hipLaunchKernelGGL((k_hill_finalize_wave<D, FUSE>), dim3(a.tabs.W), dim3(64), 0, s, a, cs, pos);
        else
            hipLaunchKernelGGL((k_hill_finalize<D, FUSE>), dim3(a.tabs.W), dim3(kBlock), 0, s, a, cs, pos);
    }
    return hipGetLastError();
}

template <int D>
hipError_t launch_hill_dd(const HillArgs &a, const CvSet &cs, const PosView &pos, int32_t grid, hipStream_t s,
                          int which)
{
    return a.fuse ? launch_hill_d<D, true>(a, cs, pos, grid, s, which)
                  : launch_hill_d<D, false>(a, cs, pos, grid, s, which);
}

// One lane per (walker, touched atom): out += sign * sum_s coef[w][cv(s)] J_s.
__global__ void __launch_bounds__(kBlock) k_gather(WalkerTabs t, const float *J, int32_t nslots, int32_t D,
                                                    const double *coef, double sign, ForceView out)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)t.W * t.U) return;
    const int32_t w = (int32_t)(gid / t.U), u = (int32_t)(gid % t.U);
    const int64_t jb = (int64_t)w * nslots;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int q = t.inv_ptr[u]; q < t.inv_ptr[u + 1]; ++q) {
        const int32_t s = t.inv_slot[q];
        const double cf = sign * coef[(int64_t)w * D + t.slot_cv[s]];
        const float *js = J + (jb + s) * 3;
        fx += cf * (double)js[0];
        fy += cf * (double)js[1];
        fz += cf * (double)js[2];
    }
    float *f = out.ptr + (t.atom_off[w] + t.touched[u]) * out.sa;
    f[0] += (float)fx;
    f[out.sk] += (float)fy;
    f[2 * out.sk] += (float)fz;
}

__global__ void k_copy_f64(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

hipError_t launch_hill_private(const HillArgs &a, const CvSet &cs, const PosView &pos, int32_t grid, hipStream_t s,
                               int which)
{
    switch (a.D) {
    case 1: return launch_hill_dd<1>(a, cs, pos, grid, s, which);
    case 2: return launch_hill_dd<2>(a, cs, pos, grid, s, which);
    case 3: return launch_hill_dd<3>(a, cs, pos, grid, s, which);
    default: return hipErrorInvalidValue;
    }
}


hipError_t launch_gather(const WalkerTabs &t, const float *J, int32_t nslots, int32_t D, const double *coef,
                         double coef_sign, ForceView out, hipStream_t s)
{
    const int64_t n = (int64_t)t.W * t.U;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, t, J, nslots, D,
                       coef, coef_sign, out);
    return hipGetLastError();
}

hipError_t launch_copy_xi(const double *src, double *dst, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_zero_bytes(void *p, int64_t nbytes, hipStream_t s)
{
    const int64_t n = nbytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

}  // namespace sx
