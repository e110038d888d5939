// Adaptive biasing force (Sec. 2.1.4, after Darve et al. 2008): one
// workgroup per walker.  Per touched atom i the Jacobian rows j_d (slots of
// one atom and one CV summed) give, in FP64 over the workgroup,
//   G = sum_i m_i^-1 j_d . j_e     and   u = sum_i m_i^-1 j_d . q_i .
// Projected-force estimator: unit masses, q = the system force, and
// theta = -G^-1 u.  Momentum estimator: q = the momentum, G^-1 u = W p (the
// CV-space momentum, W = (J M^-1 J^T)^-1 J M^-1), and
// theta = b_prev - (W p - (W p)_prev) / dt, b_prev the bias of the previous
// step (no sample on a walker's first step).  The bias of the bin of xi is
// Fsum / max(N, N_thr) from the samples before this step (with FUNN: the
// gradient of the network fitted to the mean forces, evaluated at xi, inside
// the grid's range); then N += 1, Fsum += theta, and the bias force is
// gathered onto the atoms.
#include "sx_internal.h"
#include "dev_gather.h"
#include "dev_reduce.h"

namespace sx {
namespace {

__global__ void __launch_bounds__(kBlock) k_abf(AbfArgs a)
{
    constexpr int MD = kMaxBiasDim;
    __shared__ double lds[(MD * MD + MD) * (kBlock / 64)];
    __shared__ double s_coef[kMaxCv];
    const int32_t w = blockIdx.x;
    const int D = a.D;
    const WalkerTabs &t = a.tabs;
    const int64_t jb = (int64_t)w * a.nslots, ab = t.atom_off[w];
    double acc[MD * MD + MD];
#pragma unroll
    for (int j = 0; j < MD * MD + MD; ++j) acc[j] = 0.0;
    for (int u = threadIdx.x; u < t.U; u += blockDim.x) {
        double jv[MD][3];
#pragma unroll
        for (int d = 0; d < MD; ++d) jv[d][0] = jv[d][1] = jv[d][2] = 0.0;
        for (int q = t.inv_ptr[u]; q < t.inv_ptr[u + 1]; ++q) {
            const int32_t s = t.inv_slot[q];
            const int d = t.slot_cv[s];
            const float *js = a.J + (jb + s) * 3;
#pragma unroll
            for (int dd = 0; dd < MD; ++dd)
                if (dd == d) {
                    jv[dd][0] += js[0];
                    jv[dd][1] += js[1];
                    jv[dd][2] += js[2];
                }
        }
        const int64_t atom = ab + t.touched[u];
        const float *fp = static_cast<const float *>(a.Fsys.ptr) + atom * a.Fsys.sa;
        const double f[3] = {fp[0], fp[a.Fsys.sk], fp[2 * a.Fsys.sk]};
        const double im = a.estimator == 1 ? a.inv_mass[atom] : 1.0;
#pragma unroll
        for (int d = 0; d < MD; ++d) {
#pragma unroll
            for (int e = 0; e < MD; ++e)
                acc[d * MD + e] += im * (jv[d][0] * jv[e][0] + jv[d][1] * jv[e][1] + jv[d][2] * jv[e][2]);
            acc[MD * MD + d] += im * (jv[d][0] * f[0] + jv[d][1] * f[1] + jv[d][2] * f[2]);
        }
    }
    block_sum0<MD * MD + MD>(acc, lds);
    if (threadIdx.x == 0) {
        // solve G x = u by Gaussian elimination with partial pivoting
        double G[MD][MD + 1];
        for (int d = 0; d < D; ++d) {
            for (int e = 0; e < D; ++e) G[d][e] = acc[d * MD + e];
            G[d][D] = acc[MD * MD + d];
        }
        for (int col = 0; col < D; ++col) {
            int piv = col;
            for (int r = col + 1; r < D; ++r)
                if (fabs(G[r][col]) > fabs(G[piv][col])) piv = r;
            if (piv != col)
                for (int e = 0; e <= D; ++e) {
                    double tmp = G[col][e];
                    G[col][e] = G[piv][e];
                    G[piv][e] = tmp;
                }
            for (int r = col + 1; r < D; ++r) {
                const double fct = G[r][col] / G[col][col];
                for (int e = col; e <= D; ++e) G[r][e] -= fct * G[col][e];
            }
        }
        double x[MD];
        for (int d = D - 1; d >= 0; --d) {
            double s = G[d][D];
            for (int e = d + 1; e < D; ++e) s -= G[d][e] * x[e];
            x[d] = s / G[d][d];
        }
        double theta[MD] = {0.0, 0.0, 0.0};
        bool sample = true;
        if (a.estimator == 1) {
            sample = a.has_prev[w] != 0;
            for (int d = 0; d < D; ++d)
                theta[d] = a.b_prev[(int64_t)w * D + d] - (x[d] - a.Wp_prev[(int64_t)w * D + d]) / a.dt;
        } else {
            for (int d = 0; d < D; ++d) theta[d] = -x[d];
        }
        // bin of xi (row-major, first CV slowest)
        int64_t k = 0;
        bool inr = true;
        for (int d = 0; d < D; ++d) {
            const double xv = a.xi[(int64_t)w * D + d];
            int64_t i = (int64_t)floor((xv - a.lo[d]) / a.delta[d]);
            if (a.periodic[d]) {
                i %= a.nbins[d];
                if (i < 0) i += a.nbins[d];
            } else if (i < 0 || i >= a.nbins[d]) {
                inr = false;
            }
            k = k * a.nbins[d] + i;
        }
        bool finite = true;
        for (int d = 0; d < D; ++d) finite = finite && isfinite(theta[d]) && isfinite(x[d]);
        if (!finite) atomicOr(a.flags, kFlagNonFinite);
        double b[MD] = {0.0, 0.0, 0.0};
        if (inr && finite) {
            uint32_t *Nk = a.N + (int64_t)w * a.nbins_total + k;
            double *Fk = a.Fsum + ((int64_t)w * a.nbins_total + k) * D;
            const uint32_t cnt = *Nk;
            const double den = (double)max((int64_t)cnt, (int64_t)a.n_threshold);
            for (int d = 0; d < D; ++d)
                b[d] = a.b_ext ? a.b_ext[(int64_t)w * D + d] : den > 0.0 ? Fk[d] / den : 0.0;
            if (sample) {
                *Nk = cnt + 1u;
                for (int d = 0; d < D; ++d) Fk[d] += theta[d];
            }
        }
        if (a.estimator == 1) {  // for the next step: this step's W p and bias
            for (int d = 0; d < D; ++d) {
                a.Wp_prev[(int64_t)w * D + d] = x[d];
                a.b_prev[(int64_t)w * D + d] = b[d];
            }
            a.has_prev[w] = 1;
        }
        for (int d = 0; d < D; ++d) {
            s_coef[d] = b[d];
            if (a.dV_out) a.dV_out[(int64_t)w * D + d] = -b[d];
            if (a.xi_out) a.xi_out[(int64_t)w * D + d] = a.xi[(int64_t)w * D + d];
        }
        if (a.V_out) a.V_out[w] = 0.0;
        if (w == 0) *a.dstep = a.step >= 0 ? a.step + 1 : *a.dstep + 1;
    }
    __syncthreads();
    gather_forces(t, a.J + jb * 3, w, s_coef, a.F);
}

}  // namespace

hipError_t launch_abf(const AbfArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_abf, dim3(a.tabs.W), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace sx
