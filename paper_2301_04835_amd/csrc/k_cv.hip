// Collective-variable kernels: values xi and the sparse Jacobian dxi/dx
// (PySAGES obtains the Jacobian by automatic differentiation of the CV
// function, Sec. 2 and Sec. 2.2; here each CV has its analytic gradient).
//
//  * dihedral angle: one lane per (walker, dihedral), FP64 arithmetic;
//  * radius of gyration: one workgroup per (walker, CV), two passes in FP64;
//  * coordination number, all pairs: member blocks x side (A or B) x
//    (walker, CV).  L lanes own one member of their side and gather
//    over the other group staged in LDS, so every sum has exactly one writer
//    (no atomics); a one-wavefront kernel sums the CV value's per-block
//    records in a fixed order (bitwise deterministic).
//
// All three run in one launch (k_cv_values), each workgroup in one role, so
// the kinds overlap on the device instead of following one another.
#include "dev_cv.h"

#include <type_traits>

namespace sx {
namespace {

// Jacobian slot store: float for the hill-sum paths, double for ABF, whose
// Gram matrix and J.F are formed from the rows as computed
__device__ __forceinline__ void st_slot(float *J, int64_t slot, double3 g)
{
    J[slot * 3 + 0] = (float)g.x;
    J[slot * 3 + 1] = (float)g.y;
    J[slot * 3 + 2] = (float)g.z;
}
__device__ __forceinline__ void st_slot(double *J, int64_t slot, double3 g)
{
    J[slot * 3 + 0] = g.x;
    J[slot * 3 + 1] = g.y;
    J[slot * 3 + 2] = g.z;
}

// ------------------------------------------------------------------ dihedral
// One lane per (walker, dihedral CV), FP64 (see dihedral_fp64); block bx of
// the dihedral range.
template <typename JT>
__device__ __forceinline__ void dihedral_block(const CvSet &cs, const WalkerTabs &t, const PosView &pos, double *xi,
                                               JT *J, int32_t ndih, int64_t bx)
{
    int64_t gid = bx * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)t.W * ndih) return;
    int32_t w = (int32_t)(gid / ndih), j = (int32_t)(gid % ndih);
    int c = 0, seen = 0;
    for (; c < cs.ncv; ++c)
        if (cs.cv[c].kind == CV_DIHEDRAL && seen++ == j) break;
    const CvDesc cv = cs.cv[c];
    double3 g[4];
    const double phi = J ? dihedral_at<true>(cv, pos, t.atom_off[w], g) : dihedral_at<false>(cv, pos, t.atom_off[w], g);
    xi[(int64_t)w * cs.D + cv.d] = phi;
    if (J) {
        const int64_t sb = (int64_t)w * cs.nslots + cv.slot0;
        for (int q = 0; q < 4; ++q) st_slot(J, sb + q, g[q]);
    }
}

// ----------------------------------------------------- block reductions (FP64)
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *lds /* N * kBlock/64 */)
{
    // fixed reduction tree: wave butterfly, then the waves in index order
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[wv * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < N; ++k) {
            double s = lds[k];
            for (int q = 1; q < nw; ++q) s += lds[q * N + k];
            lds[k] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = lds[k];
    __syncthreads();
}

// ------------------------------------------------------- radius of gyration
// Rg = sqrt((1/n) sum |r_i - c|^2), c = (1/n) sum r_i; dRg/dr_i = (r_i - c)/(n Rg).
// One workgroup per (walker w, gyration CV j); lds: 4 * kBlock / 64 doubles.
template <typename JT>
__device__ __forceinline__ void gyration_block(const CvSet &cs, const WalkerTabs &t, const PosView &pos, double *xi,
                                               JT *J, int32_t w, int j, double *lds)
{
    int c = 0, seen = 0;
    for (; c < cs.ncv; ++c)
        if (cs.cv[c].kind == CV_GYRATION && seen++ == j) break;
    const CvDesc cv = cs.cv[c];
    const int64_t base = t.atom_off[w];
    const int n = cv.na;
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double3 r = ld_pos(pos, base + t.slot_atom[cv.slot0 + i]);
        s[0] += r.x;
        s[1] += r.y;
        s[2] += r.z;
    }
    block_sum<3>(s, lds);
    const double3 cen = make_double3(s[0] / n, s[1] / n, s[2] / n);
    double q[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double3 d = d3sub(ld_pos(pos, base + t.slot_atom[cv.slot0 + i]), cen);
        q[0] += d3dot(d, d);
    }
    block_sum<1>(q, lds);
    const double rg = sqrt(q[0] / n);
    if (threadIdx.x == 0) xi[(int64_t)w * cs.D + cv.d] = rg;
    if (J) {
        const double inv = 1.0 / ((double)n * rg);
        const int64_t sb = (int64_t)w * cs.nslots + cv.slot0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double3 d = d3sub(ld_pos(pos, base + t.slot_atom[cv.slot0 + i]), cen);
            st_slot(J, sb + i, d3scale(d, inv));
        }
    }
}

// ---------------------------------------------- coordination number, all pairs
struct Partner {  // a partner atom staged in LDS
    double x, y, z;
    int32_t idx, pad;
};
constexpr int kCnStage = 1024;  // partners staged per round (32 KB)

template <typename T>
__device__ __forceinline__ double3 ld_d3(const PosView &p, int64_t i)
{
    const T *q = static_cast<const T *>(p.ptr) + i * p.sa;
    return make_double3((double)q[0], (double)q[p.sk], (double)q[2 * p.sk]);
}

// minimum-image component in FP64, rounded once to float (or kept in FP64)
__device__ __forceinline__ float min_img(double d, double L, double iL) { return (float)fma(-L, rint(d * iL), d); }
__device__ __forceinline__ double min_img_d(double d, double L, double iL) { return fma(-L, rint(d * iL), d); }

// The hard cut decided from the positions as given, in FP64, one operation
// at a time and without contraction: d = a - b, d -= L rint(d / L),
// r = sqrt((dx^2 + dy^2) + dz^2), inside unless r >= rcut (the plain
// definition, so that a pair at the cut's edge falls on the same side as
// under it).  Called only for pairs whose working r^2 lies within a relative
// band of rcut^2 wider than its rounding error.
__device__ __attribute__((noinline)) bool cut_inside_exact(double ax, double ay, double az, double bx, double by,
                                                          double bz, double L0, double L1, double L2, double rcut)
{
#pragma clang fp contract(off)
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    dx = dx - L0 * rint(dx / L0);
    dy = dy - L1 * rint(dy / L1);
    dz = dz - L2 * rint(dz / L2);
    return !(sqrt(dx * dx + dy * dy + dz * dz) >= rcut);
}

// grid: x = block of kBlock / L members of one side, y = side (0: A gathers
// over B, 1: B gathers over A), z = walker * ncoord + k (k-th coordination
// CV); L = cv.lanes lanes per member.  The other side's members are staged
// in LDS kCnStage at a time; lane l of a member takes partners l, l + L,
// ... of each round.  The pair difference and its minimum image are taken in
// FP64 (exact for float inputs up to the final rounding), the switching
// function in FP32, its sums in FP32 over each eight of a lane's partners and
// in FP64 beyond (for a Jacobian kept in FP64, JT = double, every pair term
// is FP64); a pair whose r^2 lies within 1e-5 (FP64 terms: 1e-12) of the
// hard cut's, relative, is re-decided by cut_inside_exact.  The member's
// lanes combine in a fixed butterfly and the first writes the Jacobian slot.  On the A side the members' switch sums are
// reduced per workgroup (fixed tree) into one value record per block, which
// k_coord_value sums in order.
template <typename T, typename JT>
__device__ __forceinline__ void coord_block(const CvSet &cs, const WalkerTabs &t, const PosView &pos, double *vpart,
                                            JT *J, int32_t ncoord, int bx, int side, int z, Partner *oth,
                                            double *lds)
{
    const int32_t w = z / ncoord, k = z % ncoord;
    int c = 0, seen = 0;
    for (; c < cs.ncv; ++c)
        if (cs.cv[c].kind == CV_COORD && seen++ == k) break;
    const CvDesc cv = cs.cv[c];
    const int nmine = side ? cv.nb : cv.na, noth = side ? cv.na : cv.nb;
    const int mine0 = cv.slot0 + (side ? cv.na : 0), oth0 = cv.slot0 + (side ? 0 : cv.na);
    const int L = cv.lanes, per = kBlock / L;
    if (bx * per >= nmine) return;  // whole workgroup idle: uniform exit
    const int64_t base = t.atom_off[w];
    const double Lb[3] = {cs.box[0], cs.box[1], cs.box[2]};
    const double iL[3] = {cs.inv_box[0], cs.inv_box[1], cs.inv_box[2]};
    const int i = bx * per + threadIdx.x / L, l = threadIdx.x % L;
    const bool live = i < nmine;
    const int32_t me = live ? t.slot_atom[mine0 + i] : -1;
    const double3 ri = live ? ld_d3<T>(pos, base + me) : make_double3(0.0, 0.0, 0.0);
    double S = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j0 = 0; j0 < noth; j0 += kCnStage) {
        const int jn = min(kCnStage, noth - j0);
        __syncthreads();  // the previous round is consumed
        for (int j = threadIdx.x; j < jn; j += blockDim.x) {
            const int32_t a = t.slot_atom[oth0 + j0 + j];
            const double3 r = ld_d3<T>(pos, base + a);
            oth[j] = Partner{r.x, r.y, r.z, a, 0};
        }
        __syncthreads();
        if (!live) continue;
        // the loops below without any cut test when the CV has no hard cut
        auto pairs = [&](auto has_cut) {
            constexpr bool CUT = decltype(has_cut)::value;
            if (std::is_same<JT, double>::value) {  // FP64 pair terms: ABF's Gram matrix and J.F
                for (int j = l; j < jn; j += L) {
                    const Partner o = oth[j];
                    const double dx = min_img_d(ri.x - o.x, Lb[0], iL[0]);
                    const double dy = min_img_d(ri.y - o.y, Lb[1], iL[1]);
                    const double dz = min_img_d(ri.z - o.z, Lb[2], iL[2]);
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    bool use = o.idx != me;
                    if (CUT) {
                        const double rc2 = cv.rcut * cv.rcut;
                        if (fabs(r2 - rc2) <= 1e-12 * rc2)  // rare: the edge of the cut
                            use = use && cut_inside_exact(ri.x, ri.y, ri.z, o.x, o.y, o.z, Lb[0], Lb[1], Lb[2], cv.rcut);
                        else
                            use = use && r2 < rc2;
                    }
                    double sv, f;
                    switch_fn(r2, cv, sv, f);
                    S += use ? sv : 0.0;
                    f = use ? f : 0.0;
                    gx = fma(f, dx, gx);
                    gy = fma(f, dy, gy);
                    gz = fma(f, dz, gz);
                }
                return;
            }
            for (int j = l; j < jn; j += 8 * L) {
                float s8 = 0.f, x8 = 0.f, y8 = 0.f, z8 = 0.f;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int jj = j + q * L;
                    if (jj >= jn) break;
                    const Partner o = oth[jj];
                    const float dx = min_img(ri.x - o.x, Lb[0], iL[0]);
                    const float dy = min_img(ri.y - o.y, Lb[1], iL[1]);
                    const float dz = min_img(ri.z - o.z, Lb[2], iL[2]);
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    bool use = o.idx != me;
                    if (CUT) {
                        if (fabsf(r2 - cv.rcut2) <= 1e-5f * cv.rcut2)  // rare: the edge of the cut
                            use = use && cut_inside_exact(ri.x, ri.y, ri.z, o.x, o.y, o.z, Lb[0], Lb[1], Lb[2], cv.rcut);
                        else
                            use = use && r2 < cv.rcut2;
                    }
                    float sv, f;
                    switch_fn(r2, cv, sv, f);
                    sv = use ? sv : 0.f;
                    f = use ? f : 0.f;
                    s8 += sv;
                    x8 = fmaf(f, dx, x8);
                    y8 = fmaf(f, dy, y8);
                    z8 = fmaf(f, dz, z8);
                }
                S += s8;
                gx += x8;
                gy += y8;
                gz += z8;
            }
        };
        if (cv.rcut > 0.0)
            pairs(std::true_type{});
        else
            pairs(std::false_type{});
    }
    for (int o = 1; o < L; o <<= 1) {  // within the member's lanes (aligned groups of a wavefront)
        S += __shfl_xor(S, o, 64);
        gx += __shfl_xor(gx, o, 64);
        gy += __shfl_xor(gy, o, 64);
        gz += __shfl_xor(gz, o, 64);
    }
    if (J && live && l == 0)
        st_slot(J, (int64_t)w * cs.nslots + mine0 + i, make_double3(gx * cv.scale, gy * cv.scale, gz * cv.scale));
    if (side == 0) {  // uniform per workgroup
        double v[1] = {live && l == 0 ? S : 0.0};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) vpart[(int64_t)w * cs.vblk_per_walker + cv.vblk0 + bx] = v[0];
    }
}

// All CV values and Jacobians in one launch (a 1-D grid): first the pair
// blocks of the all-pairs coordination numbers (x = member block of one
// side, then side, then walker * ncoord + k), then one workgroup per
// (walker, gyration CV), then the dihedral lanes.  Each workgroup takes one
// role, so its barriers are uniform.
struct CvGrid {
    int32_t ncn, nrg, ndih, cn_x;  // cn_x: member blocks per (side, walker, CV)
    int64_t cn_blocks, rg_blocks;
};

template <typename T, bool CN, typename JT>
__global__ void __launch_bounds__(kBlock) k_cv_values(CvSet cs, WalkerTabs t, PosView pos, double *xi, JT *J,
                                                       double *vpart, CvGrid g)
{
    __shared__ Partner oth[CN ? kCnStage : 1];
    __shared__ double lds[4 * (kBlock / 64)];
    int64_t b = blockIdx.x;
    if (CN && b < g.cn_blocks) {
        const int bx = (int)(b % g.cn_x), side = (int)((b / g.cn_x) % 2), z = (int)(b / (2 * (int64_t)g.cn_x));
        coord_block<T, JT>(cs, t, pos, vpart, J, g.ncn, bx, side, z, oth, lds);
        return;
    }
    b -= g.cn_blocks;
    if (b < g.rg_blocks) {
        gyration_block(cs, t, pos, xi, J, (int32_t)(b / g.nrg), (int)(b % g.nrg), lds);
        return;
    }
    dihedral_block(cs, t, pos, xi, J, g.ndih, b - g.rg_blocks);
}

// one wavefront per (walker, coordination CV): the value records of its A
// side's blocks in a fixed order (lane-strided, then a butterfly), times the
// CV's scale.
__global__ void __launch_bounds__(64) k_coord_value(CvSet cs, const double *vpart, double *xi, int32_t ncoord)
{
    const int32_t w = blockIdx.x / ncoord, k = blockIdx.x % ncoord;
    int c = 0, seen = 0;
    for (; c < cs.ncv; ++c)
        if (cs.cv[c].kind == CV_COORD && seen++ == k) break;
    const CvDesc cv = cs.cv[c];
    const int per = kBlock / cv.lanes, nblk = (cv.na + per - 1) / per;
    const double *p = vpart + (int64_t)w * cs.vblk_per_walker + cv.vblk0;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) v += p[b];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) xi[(int64_t)w * cs.D + cv.d] = v * (double)cv.scale;
}

template <typename JT>
hipError_t launch_cv_t(const CvSet &cs, const WalkerTabs &t, PosView pos, double *xi, JT *J, double *cn_vpart,
                       hipStream_t s, bool cn_values)
{
    CvGrid g{};
    for (int c = 0; c < cs.ncv; ++c) {
        const CvDesc &d = cs.cv[c];
        if (d.kind == CV_DIHEDRAL) ++g.ndih;
        if (d.kind == CV_GYRATION) ++g.nrg;
        if (d.kind == CV_COORD) {
            ++g.ncn;
            const int per = kBlock / d.lanes;
            g.cn_x = max(g.cn_x, (max(d.na, d.nb) + per - 1) / per);
        }
    }
    g.cn_blocks = (int64_t)g.cn_x * 2 * t.W * g.ncn;
    g.rg_blocks = (int64_t)t.W * g.nrg;
    const int64_t dih_blocks = ((int64_t)t.W * g.ndih + kBlock - 1) / kBlock;
    const int64_t blocks = g.cn_blocks + g.rg_blocks + dih_blocks;
    if (blocks == 0) return hipSuccess;
    if (g.ncn) {
        if (pos.f64)
            hipLaunchKernelGGL((k_cv_values<double, true, JT>), dim3((unsigned)blocks), dim3(kBlock), 0, s, cs, t, pos,
                               xi, J, cn_vpart, g);
        else
            hipLaunchKernelGGL((k_cv_values<float, true, JT>), dim3((unsigned)blocks), dim3(kBlock), 0, s, cs, t, pos,
                               xi, J, cn_vpart, g);
    } else {
        hipLaunchKernelGGL((k_cv_values<float, false, JT>), dim3((unsigned)blocks), dim3(kBlock), 0, s, cs, t, pos, xi,
                           J, cn_vpart, g);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g.ncn || !cn_values) return e;
    hipLaunchKernelGGL(k_coord_value, dim3((unsigned)t.W * g.ncn), dim3(64), 0, s, cs, cn_vpart, xi, g.ncn);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cv(const CvSet &cs, const WalkerTabs &t, PosView pos, double *xi, float *J, double *J64,
                     double *cn_vpart, hipStream_t s, bool cn_values)
{
    if (J64) return launch_cv_t<double>(cs, t, pos, xi, J64, cn_vpart, s, cn_values);
    return launch_cv_t<float>(cs, t, pos, xi, J, cn_vpart, s, cn_values);
}

}  // namespace sx
