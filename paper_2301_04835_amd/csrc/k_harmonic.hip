// Harmonic biasing (Sec. 2.1.1) and the samples of umbrella sampling /
// umbrella integration (Sec. 2.1.2): walker w is a window with centre
// xi0_w; its bias is sum_d k_d D_d^2 / 2 with D = xi - xi0_w (minimum image
// for a periodic CV), dV/dxi = k D, and the force -sum_d k_d D_d dxi_d/dx is
// gathered onto its atoms.  Each step may add the sample to the window's
// FP64 sums (count, sum D, sum D D^T), from which its mean and covariance
// and the mean force k (xi0 - <xi>) follow.
#include "sx_internal.h"
#include "dev_cv.h"
#include "dev_gather.h"

namespace sx {
namespace {

// one workgroup per walker; thread 0 owns the window's bookkeeping and
// requests its centre and running sums before anything waits.  With fuse_cv
// thread d < D first evaluates dihedral d (FP64) from the positions: its
// value into LDS and the workspace, its gradient rows into the workspace's
// Jacobian, which the gather below reads after the barrier.
__global__ void __launch_bounds__(kBlock) k_harmonic(HarmonicArgs a)
{
    __shared__ double s_coef[kMaxCv];
    __shared__ double s_xi[kMaxBiasDim];
    const int32_t w = blockIdx.x;
    // thread 0's window data requested before anything waits
    double x0[kMaxBiasDim], s1p[kMaxBiasDim], s2p[kMaxBiasDim][kMaxBiasDim];
    int64_t np0 = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d) {
            x0[d] = d < a.D ? a.xi0[(int64_t)w * a.D + d] : 0.0;
            s1p[d] = (a.accumulate && d < a.D) ? a.s1[(int64_t)w * a.D + d] : 0.0;
#pragma unroll
            for (int e = 0; e < kMaxBiasDim; ++e)
                s2p[d][e] = (a.accumulate && d < a.D && e < a.D) ? a.s2[((int64_t)w * a.D + d) * a.D + e] : 0.0;
        }
        if (a.accumulate) np0 = a.n[w];
    }
    if (a.fuse_cv) {
        if ((int)threadIdx.x < a.D) {
            const CvDesc &cv = a.cs.cv[threadIdx.x];
            const int64_t aoff = a.tabs.atom_off[w];
            double3 r[4], gr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = ld_pos(a.pos, aoff + cv.atom[q]);
            const double x = dihedral_fp64<true>(r, gr);
            s_xi[threadIdx.x] = x;
            a.xi_ws[(int64_t)w * a.D + threadIdx.x] = x;
            float *js = a.J_ws + ((int64_t)w * a.nslots + cv.slot0) * 3;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                js[3 * q] = (float)gr[q].x;
                js[3 * q + 1] = (float)gr[q].y;
                js[3 * q + 2] = (float)gr[q].z;
            }
        }
        __syncthreads();  // s_xi, and the Jacobian rows the gather reads
    }
    if (threadIdx.x == 0) {
        double Dv[kMaxBiasDim], V = 0.0;
        bool finite = true;
#pragma unroll
        for (int d = 0; d < kMaxBiasDim; ++d) {
            if (d >= a.D) break;
            const double x = a.fuse_cv ? s_xi[d] : a.xi[(int64_t)w * a.D + d];
            double t = x - x0[d];
            if (a.period[d] > 0.0) t -= a.period[d] * rint(t / a.period[d]);
            Dv[d] = t;
            const double g = a.k[d] * t;
            V += 0.5 * g * t;
            finite = finite && isfinite(g);
            a.dV_ws[(int64_t)w * a.D + d] = g;
            if (a.dV_out) a.dV_out[(int64_t)w * a.D + d] = g;
            if (a.xi_out) a.xi_out[(int64_t)w * a.D + d] = x;
            s_coef[d] = -g;
        }
        a.V_ws[w] = V;
        if (a.V_out) a.V_out[w] = V;
        if (!finite || !isfinite(V)) atomicOr(a.flags, kFlagNonFinite);
        if (a.accumulate) {
            a.n[w] = np0 + 1;
#pragma unroll
            for (int d = 0; d < kMaxBiasDim; ++d) {
                if (d >= a.D) break;
                a.s1[(int64_t)w * a.D + d] = s1p[d] + Dv[d];
#pragma unroll
                for (int e = 0; e < kMaxBiasDim; ++e)
                    if (e < a.D) a.s2[((int64_t)w * a.D + d) * a.D + e] = s2p[d][e] + Dv[d] * Dv[e];
            }
        }
        if (w == 0 && a.count_step) *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    }
    __syncthreads();
    if (a.do_forces) gather_forces(a.tabs, a.J + (int64_t)w * a.nslots * 3, w, s_coef, a.F);
}

}  // namespace

hipError_t launch_harmonic(const HarmonicArgs &a, hipStream_t s)
{
    if (a.tabs.W < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_harmonic, dim3(a.tabs.W), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace sx
