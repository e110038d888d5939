// Metadynamics bias kept on a grid (Sec. 2.1.5: the bias may be stored on a
// pre-defined grid, trading accuracy for speed).  Each hill list has a grid
// holding, at every node, the list's bias V and its gradient dV/dxi; a CV
// value reads them back by multilinear interpolation over the 2^D nodes of
// its cell (V and each gradient component interpolated on their own).
// Outside the range of a non-periodic CV there is no bias.
//
//   k_grid_step     one workgroup per walker: the read-back, the outputs, the
//                   well-tempered deposit into the hill list (height from
//                   the read-back V) and the force gather; k_grid_step_wave
//                   is the same in one wavefront when forces go through the
//                   table in kernel-argument form.
//   k_grid_add      one workgroup per grid: the hills the step appended
//                   (FP64, list order) added to every node, then the list's
//                   count advanced; the workgroup of grid 0 also advances
//                   the device step counter.  With rebuild set, many
//                   workgroups per grid refill it from the whole list.
//   k_grid_eval     the read-back at arbitrary points.
//
// Node sums run in FP64 in the order the hills sit in the list, so a grid
// holds the exact hill sum at its nodes up to the rounding of exp.
#include "sx_internal.h"
#include "dev_cv.h"
#include "dev_gather.h"

namespace sx {
namespace {

constexpr int kAddBlock = 1024;

// The cell of xi: lower and upper node per CV and the fractions t; false
// outside the range of a non-periodic CV (its nodes are then set to 0).
__device__ __forceinline__ bool grid_cell(const GridArgs &g, const double *xi, int32_t (&i0)[kMaxBiasDim],
                                          int32_t (&i1)[kMaxBiasDim], double (&t)[kMaxBiasDim])
{
    bool inside = true;
#pragma unroll
    for (int d = 0; d < kMaxBiasDim; ++d) {  // compile-time indices (registers)
        if (d >= g.D) continue;
        const double u = (xi[d] - g.lo[d]) / g.delta[d];
        double fl = floor(u);
        t[d] = u - fl;
        if (g.per[d]) {
            int64_t k = (int64_t)fl % g.nbins[d];
            if (k < 0) k += g.nbins[d];
            i0[d] = (int32_t)k;
            i1[d] = i0[d] + 1 == g.nbins[d] ? 0 : i0[d] + 1;
        } else {
            if (!(u >= 0.0 && u <= (double)g.nbins[d])) {
                inside = false;
                i0[d] = i1[d] = 0;
                continue;
            }
            int32_t k = (int32_t)fl;
            if (k == g.nbins[d]) {  // xi == hi: the last cell, weight 1 on its far node
                k = g.nbins[d] - 1;
                t[d] = 1.0;
            }
            i0[d] = k;
            i1[d] = k + 1;
        }
    }
    return inside;
}

// Corner c of the cell: its node index and multilinear weight.  Corner c
// takes node i1 of CV d when bit D - 1 - d of c is set (first CV the most
// significant).
__device__ __forceinline__ int64_t grid_corner(const GridArgs &g, int c, const int32_t (&i0)[kMaxBiasDim],
                                               const int32_t (&i1)[kMaxBiasDim], const double (&t)[kMaxBiasDim],
                                               double &wgt)
{
    int64_t idx = 0;
    wgt = 1.0;
#pragma unroll
    for (int d = 0; d < kMaxBiasDim; ++d) {
        if (d >= g.D) continue;
        const bool hi = (c >> (g.D - 1 - d)) & 1;
        const int32_t n0 = i0[d], n1 = i1[d];  // select values, not addresses (keeps the arrays in registers)
        idx = idx * g.n[d] + (hi ? n1 : n0);
        wgt *= hi ? t[d] : 1.0 - t[d];
    }
    return idx;
}

// The interpolated (V, dV/dxi) of grid l at xi, corners summed in order;
// false (and zeros) outside the range of a non-periodic CV.
__device__ bool grid_read(const GridArgs &g, int32_t l, const double *xi, double &V, double (&G)[kMaxBiasDim])
{
    int32_t i0[kMaxBiasDim], i1[kMaxBiasDim];
    double t[kMaxBiasDim];
    const bool inside = grid_cell(g, xi, i0, i1, t);
    V = 0.0;
    for (int d = 0; d < kMaxBiasDim; ++d) G[d] = 0.0;
    if (!inside) return false;
    const double *Vg = g.V + (int64_t)l * g.N;
    const double *Gg = g.G + (int64_t)l * g.D * g.N;
    for (int c = 0; c < (1 << g.D); ++c) {
        double wgt;
        const int64_t idx = grid_corner(g, c, i0, i1, t, wgt);
        V += wgt * Vg[idx];
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d)
            if (d < g.D) G[d] += wgt * Gg[(int64_t)d * g.N + idx];
    }
    return true;
}

__global__ void __launch_bounds__(kBlock) k_grid_step(GridArgs g)
{
    __shared__ double s_coef[kMaxCv];
    const int32_t w = blockIdx.x;
    const int32_t l = g.shared ? 0 : w;
    if (threadIdx.x == 0) {
        double xi[kMaxBiasDim], V, G[kMaxBiasDim];
        for (int d = 0; d < g.D; ++d) xi[d] = g.xi[(int64_t)w * g.D + d];
        const bool inside = grid_read(g, l, xi, V, G);
        bool finite = isfinite(V);
        g.V_ws[w] = V;
        if (g.V_out) g.V_out[w] = V;
        for (int d = 0; d < g.D; ++d) {
            finite = finite && isfinite(G[d]);
            g.dV_ws[(int64_t)w * g.D + d] = G[d];
            if (g.dV_out) g.dV_out[(int64_t)w * g.D + d] = G[d];
            if (g.xi_out) g.xi_out[(int64_t)w * g.D + d] = xi[d];
            s_coef[d] = -G[d];
        }
        if (!finite) atomicOr(g.flags, kFlagNonFinite);
        // the step number after this one: the step kernel reads the device
        // counter (only where a deposit depends on it), the add kernel that
        // follows advances it
        bool dep = g.deposit == 2;
        if (g.deposit == 1 && g.stride > 0) {
            const int64_t next_step = g.step >= 0 ? g.step + 1 : *g.dstep + 1;
            dep = (next_step - 1) % g.stride == 0;
        }
        if (dep && (inside || g.shared)) {
            // outside the grid nothing is deposited, except that a walker
            // keeps its slot of a shared list (walker order) with a hill of
            // height 0, which adds nothing to the bias
            const double h = !inside ? 0.0 : g.inv_kdT > 0.0 ? g.height * exp(-V * g.inv_kdT) : g.height;
            const WalkerRec wr = g.wrec[l];
            const int64_t hb = (int64_t)wr.hb4 * 4;
            const int32_t cnt = g.count[l];
            const int32_t nnew = g.shared ? g.tabs.W : 1;
            if ((int64_t)cnt + nnew <= wr.cap) {
                const int64_t k = hb + cnt + (g.shared ? w : 0);
                for (int d = 0; d < g.D; ++d) g.c[d][k] = (float)xi[d];
                g.h[k] = (float)h;
                if (!g.shared || w == 0) g.pend[l] = nnew;
            } else {
                atomicOr(g.flags, kFlagCapacity);
            }
        }
    }
    __syncthreads();
    if (g.count_in_step && w == 0 && threadIdx.x == 0) *g.dstep = g.step >= 0 ? g.step + 1 : *g.dstep + 1;
    if (g.do_forces) gather_forces(g.tabs, g.J + (int64_t)w * g.nslots * 3, w, s_coef, g.F);
}

// The same step in one wavefront, for steps that gather forces through the
// table in kernel-argument form.  Every lane finds the cell (the same
// values), lane c < 2^D loads corner c's V and dV/dxi, and every lane sums
// the corner terms in corner order through shuffles (the serial order and
// bits of grid_read); xi, the list's count and record and each lane's table
// row with its Jacobian rows and force are requested before any wait (lanes
// past 2^D or U re-read corner 0 or row U - 1 and drop it).  Lane 0 writes
// the outputs and deposits, lane u < U adds atom u's force.
__global__ void __launch_bounds__(64) k_grid_step_wave(GridArgs g)
{
    __shared__ float s_J[4 * kMaxBiasDim][3];  // fused CVs: the walker's Jacobian slots
    const int32_t w = blockIdx.x;
    const int32_t l = g.shared ? 0 : w;
    const int lane = threadIdx.x;
    const bool dep_cnt = g.deposit == 1 && g.stride > 0;
    const int64_t dstep = dep_cnt && g.step < 0 ? *g.dstep : 0;
    const int32_t cnt = g.deposit ? g.count[l] : 0;
    // no deposit in this configuration: the counter moves here (nothing reads it in this kernel)
    if (g.count_in_step && w == 0 && lane == 0) *g.dstep = g.step >= 0 ? g.step + 1 : *g.dstep + 1;
    const WalkerRec wr = g.wrec[l];
    const int64_t aoff = g.tabs.atom_off[w];
    SmallGather sg{0.f, 0.f, 0.f, nullptr};
    int nent = 0;
    int32_t cvq[kSmallPer];
    float jr[kSmallPer][3];
    double xi[kMaxBiasDim];
    if (g.fuse_cv) {
        // lane d < D evaluates dihedral d of the walker in FP64 (atom indices
        // and slots selected from the kernel arguments by value); its value
        // goes to every lane, its four gradient rows to LDS and the workspace
        int32_t at[4], slot0 = g.cs.cv[0].slot0;
#pragma unroll
        for (int q = 0; q < 4; ++q) at[q] = g.cs.cv[0].atom[q];
#pragma unroll
        for (int d = 1; d < kMaxBiasDim; ++d)
            if (lane == d && d < g.D) {
                slot0 = g.cs.cv[d].slot0;
#pragma unroll
                for (int q = 0; q < 4; ++q) at[q] = g.cs.cv[d].atom[q];
            }
        double xd = 0.0;
        if (lane < g.D) {
            double3 r[4], gr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = ld_pos(g.pos, aoff + at[q]);
            xd = dihedral_fp64<true>(r, gr);
            g.xi_ws[(int64_t)w * g.D + lane] = xd;
            float *js = g.J_ws + ((int64_t)w * g.nslots + slot0) * 3;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float gx = (float)gr[q].x, gy = (float)gr[q].y, gz = (float)gr[q].z;
                js[3 * q] = gx;
                js[3 * q + 1] = gy;
                js[3 * q + 2] = gz;
                s_J[slot0 + q][0] = gx;
                s_J[slot0 + q][1] = gy;
                s_J[slot0 + q][2] = gz;
            }
        }
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d) xi[d] = __shfl(xd, min(d, g.D - 1), 64);
        // this lane's table row and force (the Jacobian rows come from LDS)
        const int u = min(lane, g.small.U - 1);
        nent = g.small.nent[u];
        sg.dst = g.F.ptr + (aoff + g.small.touched[u]) * g.F.sa;
        sg.f0 = sg.dst[0];
        sg.f1 = sg.dst[g.F.sk];
        sg.f2 = sg.dst[2 * g.F.sk];
        int32_t e[kSmallPer];
#pragma unroll
        for (int q = 0; q < kSmallPer; ++q) e[q] = g.small.ent[u][q];
        __syncthreads();  // s_J written (one wavefront)
#pragma unroll
        for (int q = 0; q < kSmallPer; ++q) {
            const int32_t slot = e[q] & 0xFFFFF;  // < 4 D: every CV a dihedral
            cvq[q] = e[q] >> 20;
            jr[q][0] = s_J[slot][0];
            jr[q][1] = s_J[slot][1];
            jr[q][2] = s_J[slot][2];
        }
    } else {
        // xi over the largest CV count with the index clamped to the last
        // CV (in bounds, the extra entries unused), so the loads are issued
        // together
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d) xi[d] = g.xi[(int64_t)w * g.D + min(d, g.D - 1)];
        small_rows(g.small, g.J + (int64_t)w * g.nslots * 3, g.F, aoff, min(lane, g.small.U - 1), sg, nent, cvq, jr);
    }
    int32_t i0[kMaxBiasDim], i1[kMaxBiasDim];
    double t[kMaxBiasDim];
    const bool inside = grid_cell(g, xi, i0, i1, t);
    const int nc = 1 << g.D;
    double wgt;
    const int64_t idx = grid_corner(g, lane < nc ? lane : 0, i0, i1, t, wgt);
    const double *Vg = g.V + (int64_t)l * g.N;
    const double *Gg = g.G + (int64_t)l * g.D * g.N;
    const double tv = wgt * Vg[idx];
    double tg[kMaxBiasDim];
#pragma unroll
    for (int d = 0; d < kMaxBiasDim; ++d) tg[d] = d < g.D ? wgt * Gg[(int64_t)min(d, g.D - 1) * g.N + idx] : 0.0;
    double V = 0.0, G[kMaxBiasDim] = {0.0, 0.0, 0.0};
    for (int c = 0; c < nc; ++c) {
        V += __shfl(tv, c, 64);
        for (int d = 0; d < kMaxBiasDim; ++d) G[d] += __shfl(tg[d], c, 64);
    }
    if (!inside) {
        V = 0.0;
        for (int d = 0; d < kMaxBiasDim; ++d) G[d] = 0.0;
    }
    if (lane == 0) {
        bool finite = isfinite(V);
        g.V_ws[w] = V;
        if (g.V_out) g.V_out[w] = V;
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d) {
            if (d >= g.D) continue;
            finite = finite && isfinite(G[d]);
            g.dV_ws[(int64_t)w * g.D + d] = G[d];
            if (g.dV_out) g.dV_out[(int64_t)w * g.D + d] = G[d];
            if (g.xi_out) g.xi_out[(int64_t)w * g.D + d] = xi[d];
        }
        if (!finite) atomicOr(g.flags, kFlagNonFinite);
        const int64_t next_step = g.step >= 0 ? g.step + 1 : dstep + 1;
        bool dep = g.deposit == 2;
        if (dep_cnt) dep = (next_step - 1) % g.stride == 0;
        if (dep && (inside || g.shared)) {  // as k_grid_step
            const double h = !inside ? 0.0 : g.inv_kdT > 0.0 ? g.height * exp(-V * g.inv_kdT) : g.height;
            const int64_t hb = (int64_t)wr.hb4 * 4;
            const int32_t nnew = g.shared ? g.tabs.W : 1;
            if ((int64_t)cnt + nnew <= wr.cap) {
                const int64_t k = hb + cnt + (g.shared ? w : 0);
#pragma unroll
                for (int d = 0; d < kMaxBiasDim; ++d)
                    if (d < g.D) g.c[d][k] = (float)xi[d];
                g.h[k] = (float)h;
                if (!g.shared || w == 0) g.pend[l] = nnew;
            } else {
                atomicOr(g.flags, kFlagCapacity);
            }
        }
    }
    if (lane < g.small.U) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
        for (int q = 0; q < kSmallPer; ++q) {
            double cf = 0.0;
#pragma unroll
            for (int d = 0; d < kMaxBiasDim; ++d) cf = (d < g.D && cvq[q] == d) ? -G[d] : cf;
            fx += q < nent ? cf * (double)jr[q][0] : 0.0;
            fy += q < nent ? cf * (double)jr[q][1] : 0.0;
            fz += q < nent ? cf * (double)jr[q][2] : 0.0;
        }
        sg.dst[0] = sg.f0 + (float)fx;
        sg.dst[g.F.sk] = sg.f1 + (float)fy;
        sg.dst[2 * g.F.sk] = sg.f2 + (float)fz;
    }
}

// hills [k0, k1) of list l onto nodes [first, N) of its grid, node stride
// `stride`; rebuild: the nodes start from zero
__device__ void add_hills(const GridArgs &g, int32_t l, int32_t k0, int32_t k1, bool rebuild, int64_t first,
                          int64_t stride)
{
    const int64_t hb = (int64_t)g.wrec[l].hb4 * 4;
    double *Vg = g.V + (int64_t)l * g.N;
    double *Gg = g.G + (int64_t)l * g.D * g.N;
    for (int64_t node = first; node < g.N; node += stride) {
        double x[kMaxBiasDim];
        int64_t r = node;
        for (int d = g.D - 1; d >= 0; --d) {
            const int64_t i = r % g.n[d];
            r /= g.n[d];
            x[d] = g.lo[d] + (double)i * g.delta[d];
        }
        double v = rebuild ? 0.0 : Vg[node];
        double gd[kMaxBiasDim];
        for (int d = 0; d < g.D; ++d) gd[d] = rebuild ? 0.0 : Gg[(int64_t)d * g.N + node];
        for (int32_t j = k0; j < k1; ++j) {
            double q = 0.0, dl[kMaxBiasDim];
            for (int d = 0; d < g.D; ++d) {
                double u = x[d] - (double)g.c[d][hb + j];
                if (g.period[d] > 0.0) u -= g.period[d] * rint(u / g.period[d]);
                dl[d] = u;
                q += u * u * (0.5 * g.inv_sig2[d]);
            }
            const double e = (double)g.h[hb + j] * exp(-q);
            v += e;
            for (int d = 0; d < g.D; ++d) gd[d] -= e * dl[d] * g.inv_sig2[d];
        }
        Vg[node] = v;
        for (int d = 0; d < g.D; ++d) Gg[(int64_t)d * g.N + node] = gd[d];
    }
}

// After k_grid_step: one workgroup per grid (gridDim.x = L).
__global__ void __launch_bounds__(kAddBlock) k_grid_add(GridArgs g)
{
    const int32_t l = blockIdx.x;
    const int32_t k0 = g.count[l], nnew = g.pend[l];
    if (nnew > 0) add_hills(g, l, k0, k0 + nnew, false, threadIdx.x, kAddBlock);
    __syncthreads();  // every node has read the window before it moves
    if (threadIdx.x == 0) {
        if (nnew > 0) {
            g.count[l] = k0 + nnew;
            g.pend[l] = 0;
        }
        if (l == 0 && g.count_step) *g.dstep = g.step >= 0 ? g.step + 1 : *g.dstep + 1;
    }
}

// Rebuild grids l0 + blockIdx.x from their whole lists; the gridDim.y
// workgroups of a grid split its nodes.
__global__ void __launch_bounds__(kAddBlock) k_grid_rebuild(GridArgs g, int32_t l0)
{
    const int32_t l = l0 + blockIdx.x;
    add_hills(g, l, 0, g.count[l], true, (int64_t)blockIdx.y * kAddBlock + threadIdx.x,
              (int64_t)gridDim.y * kAddBlock);
}

__global__ void __launch_bounds__(kBlock) k_grid_eval(GridArgs g, int32_t l, const double *xi, int64_t n, double *V,
                                                        double *dV)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v, G[kMaxBiasDim];
    grid_read(g, l, xi + i * g.D, v, G);
    V[i] = v;
    if (dV)
        for (int d = 0; d < g.D; ++d) dV[i * g.D + d] = G[d];
}

__global__ void __launch_bounds__(kBlock) k_scale_f64(double *x, int64_t n, double a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= a;
}

}  // namespace

hipError_t launch_scale_f64(double *x, int64_t n, double a, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, n, a);
    return hipGetLastError();
}

// A configuration that never deposits (deposit off, or on a stride of 0)
// has nothing for the add kernel but the step counter: the step kernel then
// advances it and the add kernel is not launched.
hipError_t launch_grid_step(const GridArgs &g0, hipStream_t s)
{
    GridArgs g = g0;
    const bool add = !(g.deposit == 0 || (g.deposit == 1 && g.stride <= 0));
    g.count_in_step = add ? 0 : g.count_step;
    if (g.tabs.W < 1 || g.L < 1) return hipErrorInvalidValue;
    const bool wave = g.do_forces && g.small.on && g.small.U > 0;
    if (g.fuse_cv && !wave) return hipErrorInvalidValue;  // only the wavefront step evaluates CVs
    if (wave)
        hipLaunchKernelGGL(k_grid_step_wave, dim3(g.tabs.W), dim3(64), 0, s, g);
    else
        hipLaunchKernelGGL(k_grid_step, dim3(g.tabs.W), dim3(kBlock), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !add) return e;
    hipLaunchKernelGGL(k_grid_add, dim3(g.L), dim3(kAddBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_grid_rebuild(const GridArgs &g, int32_t l0, int32_t nl, hipStream_t s)
{
    if (nl < 1 || l0 < 0 || l0 + nl > g.L) return hipErrorInvalidValue;
    const int64_t nb = std::min<int64_t>((g.N + kAddBlock - 1) / kAddBlock, 1024);
    hipLaunchKernelGGL(k_grid_rebuild, dim3(nl, (unsigned)nb), dim3(kAddBlock), 0, s, g, l0);
    return hipGetLastError();
}

hipError_t launch_grid_eval(const GridArgs &g, int32_t l, const double *xi, int64_t n, double *V, double *dV,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (l < 0 || l >= g.L) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grid_eval, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, l, xi, n, V,
                       dV);
    return hipGetLastError();
}

}  // namespace sx
