// Adaptive biasing force (Sec. 2.1.4): one workgroup per walker.  Per
// touched atom i the Jacobian rows j_d (FP64; slots of one atom and one CV
// summed) give, in FP64 over the workgroup,
//   G = sum_i m_i^-1 j_d . j_e     and   u = sum_i m_i^-1 j_d . q_i .
// Momentum estimator (the one of Darve et al. that the paper cites):
// q = the momentum, G^-1 u = W p (the CV-space momentum,
// W = (J M^-1 J^T)^-1 J M^-1), and theta = b_prev - (W p - (W p)_prev) / dt,
// b_prev the bias of the previous step (no sample on a walker's first step).
// Projected-force estimator, for inputs without dynamics: unit masses,
// q = the system force, theta = -G^-1 u; it omits the divergence term
// k_B T div(J^T (J J^T)^-1) that the mean force of a nonlinear CV carries
// (zero for linear CVs).  The bias of the bin of xi is
// Fsum / max(N, N_thr) from the samples before this step (with FUNN: the
// gradient of the network fitted to the mean forces, evaluated at xi, inside
// the grid's range); then N += 1, Fsum += theta, and the bias force is
// gathered onto the atoms.  In the two-launch form the first launch also
// sums the all-pairs coordination numbers' values from the CV kernel's block
// records (unless FUNN needs xi earlier), which saves the value kernel's
// launch.
#include "sx_internal.h"
#include "dev_gather.h"
#include "dev_reduce.h"

namespace sx {
namespace {

constexpr int MD = kMaxBiasDim;
constexpr int NA = MD * MD + MD;  // G (MD x MD) then u (MD)

// touched atom u of walker w: its Jacobian rows j_d (slots of one CV summed)
// and its terms m^-1 j_d . j_e and m^-1 j_d . q added to acc
__device__ __forceinline__ void abf_atom_terms(const AbfArgs &a, int32_t w, int u, double (&acc)[NA])
{
    const WalkerTabs &t = a.tabs;
    const int64_t jb = (int64_t)w * a.nslots, ab = t.atom_off[w];
    double jv[MD][3];
#pragma unroll
    for (int d = 0; d < MD; ++d) jv[d][0] = jv[d][1] = jv[d][2] = 0.0;
    for (int q = t.inv_ptr[u]; q < t.inv_ptr[u + 1]; ++q) {
        const int32_t s = t.inv_slot[q];
        const int d = t.slot_cv[s];
        const double *js = a.J + (jb + s) * 3;
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

// What the update reads that does not depend on the sums (AbfPre): xi, its
// bin (row major, first CV slowest), the bin's count and force sums (the
// samples before this step), FUNN's bias, the momentum estimator's previous
// values and the device step counter.  Called by every lane of a workgroup,
// the addresses are uniform, so the loads go through the scalar cache and
// are in flight while the sums are formed.
__device__ __forceinline__ AbfPre abf_prefetch(const AbfArgs &a, int32_t w)
{
    // loops over the largest CV count with run-time guards: every array
    // index is a compile-time constant, so nothing lives in scratch memory
    AbfPre r{};
    const int D = a.D;
    r.k = 0;
    r.inr = true;
#pragma unroll
    for (int d = 0; d < MD; ++d) {
        if (d >= D) continue;
        r.xi[d] = a.xi[(int64_t)w * D + d];
        int64_t i = (int64_t)floor((r.xi[d] - a.lo[d]) / a.delta[d]);
        if (a.periodic[d]) {
            i %= a.nbins[d];
            if (i < 0) i += a.nbins[d];
        } else if (i < 0 || i >= a.nbins[d]) {
            r.inr = false;
        }
        r.k = r.k * a.nbins[d] + i;
    }
    if (r.inr) {
        r.cnt = a.N[(int64_t)w * a.nbins_total + r.k];
#pragma unroll
        for (int d = 0; d < MD; ++d)
            if (d < D) r.F[d] = a.Fsum[((int64_t)w * a.nbins_total + r.k) * D + d];
    }
#pragma unroll
    for (int d = 0; d < MD; ++d)
        if (d < D && a.b_ext) r.bext[d] = a.b_ext[(int64_t)w * D + d];
    if (a.estimator == 1) {
        r.has = a.has_prev[w];
#pragma unroll
        for (int d = 0; d < MD; ++d) {
            if (d >= D) continue;
            r.bprev[d] = a.b_prev[(int64_t)w * D + d];
            r.wpprev[d] = a.Wp_prev[(int64_t)w * D + d];
        }
    }
    if (w == 0 && a.step < 0) r.dstep = *a.dstep;
    return r;
}

// One thread, the reduced G and u and the prefetched values: solve G x = u,
// form theta, and take the bias of xi's bin (zero outside the grid or when x
// or theta is not finite).  A pure function of its inputs, so every
// workgroup that evaluates it gets the same bits.
struct AbfOut {
    double x[MD], theta[MD], b[MD];
    bool sample, finite;
};

__device__ AbfOut abf_solve(const AbfArgs &a, const double (&acc)[NA], const AbfPre &pre)
{
    // every loop runs over MD with a run-time guard (d < D), so that all
    // array indices are compile-time constants (registers, no scratch); the
    // operations on rows and columns below D are those of plain Gaussian
    // elimination with partial pivoting on the D x D system, in its order
    const int D = a.D;
    AbfOut r{};
    double G[MD][MD], rhs[MD];
#pragma unroll
    for (int d = 0; d < MD; ++d) {
#pragma unroll
        for (int e = 0; e < MD; ++e) G[d][e] = (d < D && e < D) ? acc[d * MD + e] : 0.0;
        rhs[d] = d < D ? acc[MD * MD + d] : 0.0;
    }
#pragma unroll
    for (int col = 0; col < MD; ++col) {
        if (col >= D) continue;
        // pivot: the first row r >= col with the largest |G[r][col]|
        int piv = col;
        double best = fabs(G[col][col]);
#pragma unroll
        for (int q = col + 1; q < MD; ++q)
            if (q < D && fabs(G[q][col]) > best) {
                best = fabs(G[q][col]);
                piv = q;
            }
#pragma unroll
        for (int q = col + 1; q < MD; ++q)
            if (q == piv) {
#pragma unroll
                for (int e = 0; e < MD; ++e) {
                    const double tmp = G[col][e];
                    G[col][e] = G[q][e];
                    G[q][e] = tmp;
                }
                const double tmp = rhs[col];
                rhs[col] = rhs[q];
                rhs[q] = tmp;
            }
#pragma unroll
        for (int q = col + 1; q < MD; ++q) {
            if (q >= D) continue;
            const double fct = G[q][col] / G[col][col];
#pragma unroll
            for (int e = col; e < MD; ++e)
                if (e < D) G[q][e] -= fct * G[col][e];
            rhs[q] -= fct * rhs[col];
        }
    }
#pragma unroll
    for (int d = MD - 1; d >= 0; --d) {
        if (d >= D) continue;
        double sd = rhs[d];
#pragma unroll
        for (int e = d + 1; e < MD; ++e)
            if (e < D) sd -= G[d][e] * r.x[e];
        r.x[d] = sd / G[d][d];
    }
    r.sample = true;
    if (a.estimator == 1) r.sample = pre.has != 0;
    r.finite = true;
#pragma unroll
    for (int d = 0; d < MD; ++d) {
        if (d >= D) continue;
        r.theta[d] = a.estimator == 1 ? pre.bprev[d] - (r.x[d] - pre.wpprev[d]) / a.dt : -r.x[d];
        r.finite = r.finite && isfinite(r.theta[d]) && isfinite(r.x[d]);
    }
    if (pre.inr && r.finite) {
        const double den = (double)max((int64_t)pre.cnt, (int64_t)a.n_threshold);
#pragma unroll
        for (int d = 0; d < MD; ++d)
            if (d < D) r.b[d] = a.b_ext ? pre.bext[d] : den > 0.0 ? pre.F[d] / den : 0.0;
    }
    return r;
}

// Once per walker and step: add the sample to the grid, keep the momentum
// estimator's state, write the outputs and advance the step counter.
__device__ void abf_commit(const AbfArgs &a, int32_t w, const AbfPre &pre, const AbfOut &r)
{
    const int D = a.D;
    if (!r.finite) atomicOr(a.flags, kFlagNonFinite);
    if (pre.inr && r.finite && r.sample) {
        a.N[(int64_t)w * a.nbins_total + pre.k] = pre.cnt + 1u;
        double *Fk = a.Fsum + ((int64_t)w * a.nbins_total + pre.k) * D;
#pragma unroll
        for (int d = 0; d < MD; ++d)
            if (d < D) Fk[d] = pre.F[d] + r.theta[d];
    }
#pragma unroll
    for (int d = 0; d < MD; ++d) {
        if (d >= D) continue;
        if (a.estimator == 1) {  // for the next step: this step's W p and bias
            a.Wp_prev[(int64_t)w * D + d] = r.x[d];
            a.b_prev[(int64_t)w * D + d] = r.b[d];
        }
        if (a.dV_out) a.dV_out[(int64_t)w * D + d] = -r.b[d];
        if (a.xi_out) a.xi_out[(int64_t)w * D + d] = pre.xi[d];
    }
    if (a.estimator == 1) a.has_prev[w] = 1;
    if (a.V_out) a.V_out[w] = 0.0;
    if (w == 0) *a.dstep = a.step >= 0 ? a.step + 1 : pre.dstep + 1;
}

__global__ void __launch_bounds__(kBlock) k_abf(AbfArgs a)
{
    __shared__ double lds[NA * (kBlock / 64)];
    __shared__ double s_coef[kMaxCv];
    const int32_t w = blockIdx.x;
    const AbfPre pre = abf_prefetch(a, w);
    double acc[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = 0.0;
    for (int u = threadIdx.x; u < a.tabs.U; u += blockDim.x) abf_atom_terms(a, w, u, acc);
    block_sum0<NA>(acc, lds);
    if (threadIdx.x == 0) {
        const AbfOut r = abf_solve(a, acc, pre);
        abf_commit(a, w, pre, r);
#pragma unroll
        for (int d = 0; d < MD; ++d)
            if (d < a.D) s_coef[d] = r.b[d];
    }
    __syncthreads();
    gather_forces(a.tabs, a.J + (int64_t)w * a.nslots * 3, w, s_coef, a.F);
}

// Walkers with many touched atoms, in two launches: (1) one lane per touched
// atom, the terms reduced per workgroup (fixed tree) into a record per
// (walker, block), and the first workgroup's first lane keeps the walker's
// AbfPre in the workspace; (2) per (walker, block of touched atoms): the
// first wavefront sums the walker's records in a fixed order and its first
// lane solves from them and the kept AbfPre -- every workgroup the same bits
// -- the first workgroup alone commits the sample, and every workgroup
// gathers the forces of its atoms.  The grid is read in (1) and written in
// (2) by one lane, so no workgroup reads it while it changes.
// The coordination numbers' values of walker w from their block records:
// lane-strided sums, a fixed butterfly, times the scale (the value kernel's
// order, so the same bits); run by one whole wavefront, lane 0 writes.
__device__ void fold_cn_values(const AbfArgs &a, int32_t w)
{
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < a.ncn_fold && k < kMaxBiasDim; ++k) {
        const double *p = a.cn_vpart + (int64_t)w * a.vblk_per_walker + a.cn_vblk0[k];
        double v = 0.0;
        for (int b = lane; b < a.cn_nblk[k]; b += 64) v += p[b];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) a.xi_ws[(int64_t)w * a.D + a.cn_d[k]] = v * a.cn_scale[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_abf_part(AbfArgs a)
{
    __shared__ double lds[NA * (kBlock / 64)];
    const int32_t w = blockIdx.y;
    const int u = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < 64) {  // lane 0 reads the values it wrote
        if (a.ncn_fold > 0) fold_cn_values(a, w);
        if (threadIdx.x == 0) a.pre[w] = abf_prefetch(a, w);
    }
    double acc[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = 0.0;
    if (u < a.tabs.U) abf_atom_terms(a, w, u, acc);
    block_sum0<NA>(acc, lds);
    if (threadIdx.x == 0) {
        double *r = a.part + ((int64_t)w * a.nblk + blockIdx.x) * NA;
#pragma unroll
        for (int j = 0; j < NA; ++j) r[j] = acc[j];
    }
}

__global__ void __launch_bounds__(kBlock) k_abf_finish(AbfArgs a)
{
    __shared__ double s_coef[kMaxCv];
    const int32_t w = blockIdx.y;
    // this lane's atom: its rows and force requested before the solve
    const int u = blockIdx.x * kBlock + threadIdx.x;
    const double *Jw = a.J + (int64_t)w * a.nslots * 3;
    AtomRows<double> rows;
    if (u < a.tabs.U) atom_rows(a.tabs, Jw, w, a.F, u, rows);
    if (threadIdx.x < 64) {  // the first wavefront
        const AbfPre pre = a.pre[w];
        double acc[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) acc[j] = 0.0;
        for (int b = threadIdx.x; b < a.nblk; b += 64) {
            const double *r = a.part + ((int64_t)w * a.nblk + b) * NA;
#pragma unroll
            for (int j = 0; j < NA; ++j) acc[j] += r[j];
        }
#pragma unroll
        for (int j = 0; j < NA; ++j)
            for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
        if (threadIdx.x == 0) {
            const AbfOut r = abf_solve(a, acc, pre);
            if (blockIdx.x == 0) abf_commit(a, w, pre, r);
#pragma unroll
            for (int d = 0; d < MD; ++d)
                if (d < a.D) s_coef[d] = r.b[d];
        }
    }
    __syncthreads();
    if (u < a.tabs.U) atom_add(a.tabs, Jw, s_coef, a.F, rows);
}

}  // namespace

hipError_t launch_abf(const AbfArgs &a, hipStream_t s)
{
    if (a.nblk == 0) {
        hipLaunchKernelGGL(k_abf, dim3(a.tabs.W), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_abf_part, dim3((unsigned)a.nblk, (unsigned)a.tabs.W), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_abf_finish, dim3((unsigned)a.nblk, (unsigned)a.tabs.W), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace sx
