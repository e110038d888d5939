// Coordination numbers with a hard cutoff through cell lists (the switching
// form s(r) = (1 - (r/r0)^n) / (1 - (r/r0)^m), minimum image in an
// orthorhombic periodic box; CVs of this kind extend the paper's CV set,
// Sec. 2.2).  For groups of tens of thousands of atoms the all-pairs
// evaluation gives way to:
//
//   k_cell_build   one workgroup per (walker, group): the cell of every
//                  member (positions wrapped into the box), LDS counts, an
//                  exclusive scan, and an in-order placement (stable within
//                  a cell), so every later sum runs in a fixed order; each
//                  member is stored as (x, y, z) relative to its cell's
//                  origin (float, ~6e-8 nm) and its atom index.
//   k_cn_cell      one workgroup per (walker, CV, home cell of group A): the
//                  B members of the 27 neighbour cells are staged in LDS
//                  relative to the home cell's origin (a neighbour's offset
//                  is its cell step times the cell edge, periodic wrap
//                  included), groups of 16 lanes take home atoms (four per
//                  wavefront), their lanes take partners, four at a time;
//                  FP32 pair terms, FP64 sums; one partial per home cell.
//   k_cn_cell_fin  per (walker, CV): the home-cell partials in cell order.
//   k_cell_vjp     one workgroup per (walker, group, home cell): for every use
//                  of the group (CV, side, partner group) the partners of each
//                  home atom are recomputed and its gradient accumulated in
//                  FP64; the workgroup alone writes its atoms' forces (no
//                  atomics; needs groups that are identical or disjoint).
//
// Cells have edge >= the cutoff and there are >= 3 per dimension, so the 27
// neighbour cells are distinct and hold exactly the one image of every
// partner within the cutoff.
#include "sx_internal.h"
#include "dev_cv.h"

namespace sx {
namespace {

constexpr int kBuildBlock = 1024;
constexpr int kStageMax = 1024;  // partner atoms staged per round (16 KB of LDS)
constexpr int kHomeMax = 128;    // home atoms per force round

__device__ __forceinline__ int cell_of(double x, double L, double iL, double clen, int nc, double &rel)
{
    const double xw = x - L * floor(x * iL);  // into [0, L)
    int c = (int)(xw / clen);
    c = c < 0 ? 0 : (c >= nc ? nc - 1 : c);
    rel = xw - c * clen;
    return c;
}

template <typename T>
__global__ void __launch_bounds__(kBuildBlock) k_cell_build(CellArgs c, PosView pos)
{
    __shared__ int32_t s_off[kCellMax * kCellMax * kCellMax];
    __shared__ int32_t s_tot[kBuildBlock];
    const int w = blockIdx.x / c.G, g = blockIdx.x % c.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t n = c.goff[g + 1] - c.goff[g];
    const int32_t *ga = c.gatoms + c.goff[g];
    const int64_t aoff = c.atom_off[w];
    int32_t *cid = c.cid + (int64_t)w * c.gtotal + c.goff[g];
    int32_t *cst = c.cstart + ((int64_t)w * c.G + g) * (c.ncell + 1);
    float4 *srt = c.sorted + (int64_t)w * c.gtotal + c.goff[g];
    for (int i = tid; i < c.ncell; i += kBuildBlock) s_off[i] = 0;
    __syncthreads();
    // pass 1: cells and counts
    for (int32_t i = tid; i < n; i += kBuildBlock) {
        const double3 r = ld_pos_t<T>(pos, aoff + ga[i]);
        double rel;
        const int cx = cell_of(r.x, c.L[0], c.inv_L[0], c.clen[0], c.nc[0], rel);
        const int cy = cell_of(r.y, c.L[1], c.inv_L[1], c.clen[1], c.nc[1], rel);
        const int cz = cell_of(r.z, c.L[2], c.inv_L[2], c.clen[2], c.nc[2], rel);
        const int cell = (cx * c.nc[1] + cy) * c.nc[2] + cz;
        cid[i] = cell;
        atomicAdd(&s_off[cell], 1);  // counts only: the placement below is ordered
    }
    __syncthreads();
    // exclusive scan of the counts: 4 cells per thread, then across threads
    int32_t loc[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cc = tid * 4 + q;
        loc[q] = cc < c.ncell ? s_off[cc] : 0;
        sum += loc[q];
    }
    s_tot[tid] = sum;
    __syncthreads();
    for (int o = 1; o < kBuildBlock; o <<= 1) {  // inclusive Hillis-Steele
        const int32_t add = tid >= o ? s_tot[tid - o] : 0;
        __syncthreads();
        s_tot[tid] += add;
        __syncthreads();
    }
    int32_t run = s_tot[tid] - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cc = tid * 4 + q;
        if (cc < c.ncell) {
            s_off[cc] = run;
            cst[cc] = run;
        }
        run += loc[q];
    }
    if (tid == 0) cst[c.ncell] = n;
    __syncthreads();
    // pass 2: placement in member order; within a chunk of 1024 members the
    // rank among same-cell members comes from shuffles inside a wavefront
    // and from the wavefronts taking turns
    for (int32_t base = 0; base < n; base += kBuildBlock) {
        const int32_t i = base + tid;
        const bool valid = i < n;
        const int cell = valid ? cid[i] : -1;
        int rank = 0, cnt = 0;
        for (int k = 0; k < 64; ++k) {
            const int ck = __shfl(cell, k, 64);
            cnt += ck == cell ? 1 : 0;
            rank += (ck == cell && k < lane) ? 1 : 0;
        }
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) {
            const int32_t atom = ga[i];
            const double3 r = ld_pos_t<T>(pos, aoff + atom);
            double rx, ry, rz;
            cell_of(r.x, c.L[0], c.inv_L[0], c.clen[0], c.nc[0], rx);
            cell_of(r.y, c.L[1], c.inv_L[1], c.clen[1], c.nc[1], ry);
            cell_of(r.z, c.L[2], c.inv_L[2], c.clen[2], c.nc[2], rz);
            v = make_float4((float)rx, (float)ry, (float)rz, __int_as_float(atom));
        }
        for (int t = 0; t < kBuildBlock / 64; ++t) {
            __syncthreads();
            if (wave == t && valid) {
                const int dst = s_off[cell] + rank;
                srt[dst] = v;
                if (rank == cnt - 1) s_off[cell] += cnt;  // after every lane of the wave read it
            }
        }
        __syncthreads();
    }
}

// Is the pair within the cut?  Far from its edge the FP32 distance decides.
// Within 1e-5 of it the pair is decided from the positions as given, in
// FP64, one operation at a time and without contraction: d = a - b,
// d -= L rint(d / L), r = sqrt((dx^2 + dy^2) + dz^2), inside unless r >= rcut
// (the plain definition of the minimum-image cut, so that a pair at the
// edge falls on the same side as under that definition).  Out of line: the
// path is rare and keeps its registers out of the pair loop.
__device__ __attribute__((noinline)) bool cut_exact(PosView pos, int64_t aoff, int32_t ai, int32_t aj, double L0,
                                                   double L1, double L2, double rcut)
{
#pragma clang fp contract(off)
    const double3 p = ld_pos(pos, aoff + ai), q = ld_pos(pos, aoff + aj);
    double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    dx = dx - L0 * rint(dx / L0);
    dy = dy - L1 * rint(dy / L1);
    dz = dz - L2 * rint(dz / L2);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    return !(r >= rcut);
}

__device__ __forceinline__ bool within_cut(float r2, const CvDesc &cv, const CellArgs &c, const PosView &pos,
                                           int64_t aoff, int32_t ai, int32_t aj)
{
    if (fabsf(r2 - cv.rcut2) > 1e-5f * cv.rcut2) return r2 < cv.rcut2;
    return cut_exact(pos, aoff, ai, aj, c.L[0], c.L[1], c.L[2], cv.rcut);
}

// switching function: the (6, 12) form as a template choice, else the
// general form of switch_fn
template <bool S612>
__device__ __forceinline__ void sw(float r2, const CvDesc &cv, float &s, float &f)
{
    if (S612) {
        const float ir = cv.inv_r0 * cv.inv_r0;
        const float x2 = r2 * ir, x4 = x2 * x2;
        const float sv = __builtin_amdgcn_rcpf(fmaf(x4, x2, 1.0f));
        s = sv;
        f = -6.0f * x4 * sv * sv * ir;
    } else {
        switch_fn(r2, cv, s, f);
    }
}

// Four partners j0 + kLpa q (q < 4) of home atom `me` at pi, the kLpa lanes
// of a lane group over j0: r^2 in FP32 from cell-relative coordinates, the
// cut decided by within_cut (its exact path behind one wavefront-uniform
// vote).  A wavefront works on 64 / kLpa home atoms at a time.
constexpr int kUnroll = 4;
constexpr int kLpa = 16;             // lanes per home atom
constexpr int kApw = 64 / kLpa;      // home atoms per wavefront
struct PairBatch {
    float dx[kUnroll], dy[kUnroll], dz[kUnroll], r2[kUnroll];
    bool in[kUnroll];
};

__device__ __forceinline__ void pair_batch(const float4 &pi, int32_t me, const float4 *s_p, int j0, int m,
                                           const CvDesc &cv, const CellArgs &c, const PosView &pos, int64_t aoff,
                                           PairBatch &b)
{
    // s_p is padded with far atoms to a multiple of 64 >= m: j0 + kLpa q < 64 ceil(m / 64)
    const bool self = cv.ga == cv.gb;  // uniform: a group paired with itself skips i == j
    const float band = 1e-5f * cv.rcut2;
    bool near = false;
    int32_t him[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
        const float4 pj = s_p[j0 + kLpa * q];
        him[q] = __float_as_int(pj.w);
        b.dx[q] = pi.x - pj.x;
        b.dy[q] = pi.y - pj.y;
        b.dz[q] = pi.z - pj.z;
        b.r2[q] = fmaf(b.dx[q], b.dx[q], fmaf(b.dy[q], b.dy[q], b.dz[q] * b.dz[q]));
        const float t = b.r2[q] - cv.rcut2;
        const bool ok = m > 0 && (!self || him[q] != me);
        b.in[q] = ok && t < 0.f;
        near = near || (ok && fabsf(t) <= band);
    }
    if (__any(near)) {  // rare: a pair at the edge of the cut somewhere in the wavefront
#pragma unroll
        for (int q = 0; q < kUnroll; ++q)
            if (m > 0 && him[q] >= 0 && (!self || him[q] != me) && fabsf(b.r2[q] - cv.rcut2) <= band)
                b.in[q] = cut_exact(pos, aoff, me, him[q], c.L[0], c.L[1], c.L[2], cv.rcut);
    }
}

__device__ __forceinline__ const CvDesc &cell_cv(const CvSet &cs, int k)
{
    int c = 0;
    for (; c < cs.ncv - 1; ++c)
        if (cs.cv[c].kind == CV_COORD_CELL && cs.cv[c].cn == k) break;
    return cs.cv[c];
}

// stage the members of group gp in the 27 cells around `home` into s_p,
// relative to home's origin: entries [r0, r0 + kStageMax) of the
// concatenation in neighbour order; returns how many were staged
__device__ __forceinline__ int stage_partners(const CellArgs &c, int w, int gp, int home, int r0, float4 *s_p,
                                              int32_t *s_seg, float *s_sh)
{
    const int32_t *cst = c.cstart + ((int64_t)w * c.G + gp) * (c.ncell + 1);
    const float4 *srt = c.sorted + (int64_t)w * c.gtotal + c.goff[gp];
    const int hz = home % c.nc[2], hy = (home / c.nc[2]) % c.nc[1], hx = home / (c.nc[1] * c.nc[2]);
    if (threadIdx.x < 27) {
        const int t = threadIdx.x;
        const int ox = t / 9 - 1, oy = (t / 3) % 3 - 1, oz = t % 3 - 1;
        const int nx = (hx + ox + c.nc[0]) % c.nc[0], ny = (hy + oy + c.nc[1]) % c.nc[1], nz = (hz + oz + c.nc[2]) % c.nc[2];
        const int nb = (nx * c.nc[1] + ny) * c.nc[2] + nz;
        s_seg[32 + t] = cst[nb];                   // first member of the neighbour
        s_seg[t + 1] = cst[nb + 1] - cst[nb];      // its count (prefix below)
        s_sh[3 * t] = (float)(ox * c.clen[0]);
        s_sh[3 * t + 1] = (float)(oy * c.clen[1]);
        s_sh[3 * t + 2] = (float)(oz * c.clen[2]);
    }
    if (threadIdx.x == 0) s_seg[0] = 0;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int t = 1; t <= 27; ++t) s_seg[t] += s_seg[t - 1];
    __syncthreads();
    const int total = s_seg[27];
    const int m = min(kStageMax, total - r0);
    // padded to a multiple of 64 with atoms far outside any cut (index -1)
    const int mp = min(kStageMax, (m + 63) & ~63);
    for (int j = threadIdx.x; j < mp; j += blockDim.x) {
        float4 v = make_float4(1e6f, 1e6f, 1e6f, __int_as_float(-1));
        if (j < m) {
            const int e = r0 + j;
            int t = 0;
            while (s_seg[t + 1] <= e) ++t;  // at most 26 steps
            v = srt[s_seg[32 + t] + (e - s_seg[t])];
            v.x += s_sh[3 * t];
            v.y += s_sh[3 * t + 1];
            v.z += s_sh[3 * t + 2];
        }
        s_p[j] = v;
    }
    __syncthreads();
    return m;
}

template <bool S612>
__global__ void __launch_bounds__(kBlock) k_cn_cell(CellArgs c, CvSet cs, PosView pos, int k)
{
    __shared__ float4 s_p[kStageMax];
    __shared__ int32_t s_seg[64];
    __shared__ float s_sh[81];
    __shared__ double s_red[kBlock / 64];
    const int home = blockIdx.x, w = blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const CvDesc cv = cell_cv(cs, k);
    const int32_t *cstA = c.cstart + ((int64_t)w * c.G + cv.ga) * (c.ncell + 1);
    const float4 *sA = c.sorted + (int64_t)w * c.gtotal + c.goff[cv.ga];
    const int a0 = cstA[home], a1 = cstA[home + 1];
    double *out = c.part + ((int64_t)w * c.ncn + k) * c.ncell + home;
    if (a0 == a1) {  // uniform: an empty home cell
        if (threadIdx.x == 0) *out = 0.0;
        return;
    }
    const int64_t aoff = c.atom_off[w];
    float acc[kUnroll] = {0.f, 0.f, 0.f, 0.f};
    for (int r0 = 0;; r0 += kStageMax) {
        const int m = stage_partners(c, w, cv.gb, home, r0, s_p, s_seg, s_sh);
        const int grp = lane / kLpa, gl = lane % kLpa;
        for (int ib = a0 + wave * kApw; ib < a1; ib += (kBlock / 64) * kApw) {
            const int i = ib + grp;  // this lane group's home atom
            const bool live = i < a1;
            const float4 pi = sA[live ? i : a0];
            const int32_t me = __float_as_int(pi.w);
            const int mm = live ? m : 0;
            for (int j0 = gl; j0 < m; j0 += kLpa * kUnroll) {
                PairBatch b;
                pair_batch(pi, me, s_p, j0, mm, cv, c, pos, aoff, b);
#pragma unroll
                for (int q = 0; q < kUnroll; ++q) {
                    float sv, f;
                    sw<S612>(b.r2[q], cv, sv, f);
                    acc[q] += b.in[q] ? sv : 0.f;
                }
            }
        }
        if (r0 + m >= s_seg[27]) break;  // uniform
        __syncthreads();                 // the next round overwrites s_p
    }
    double v = ((double)acc[0] + (double)acc[1]) + ((double)acc[2] + (double)acc[3]);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = s_red[0];
        for (int q = 1; q < kBlock / 64; ++q) t += s_red[q];
        *out = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_cn_cell_fin(CellArgs c, CvSet cs, double *xi)
{
    __shared__ double s_red[kBlock / 64];
    const int k = blockIdx.x, w = blockIdx.y;
    const CvDesc cv = cell_cv(cs, k);
    const double *p = c.part + ((int64_t)w * c.ncn + k) * c.ncell;
    double v = 0.0;
    for (int i = threadIdx.x; i < c.ncell; i += kBlock) v += p[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = s_red[0];
        for (int q = 1; q < kBlock / 64; ++q) t += s_red[q];
        xi[(int64_t)w * cs.D + cv.d] = t * (double)cv.scale;
    }
}

template <bool S612>
__global__ void __launch_bounds__(kBlock) k_cell_vjp(CellArgs c, CvSet cs, PosView pos, const double *coef,
                                                      double sign, ForceView F)
{
    __shared__ float4 s_p[kStageMax];
    __shared__ int32_t s_seg[64];
    __shared__ float s_sh[81];
    __shared__ double s_f[kHomeMax][3];
    const int home = blockIdx.x, g = blockIdx.y, w = blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t *cst = c.cstart + ((int64_t)w * c.G + g) * (c.ncell + 1);
    const float4 *sg = c.sorted + (int64_t)w * c.gtotal + c.goff[g];
    const int a0 = cst[home], a1 = cst[home + 1];
    if (a0 == a1) return;  // uniform
    const int64_t aoff = c.atom_off[w];
    for (int h0 = a0; h0 < a1; h0 += kHomeMax) {
        const int h1 = min(a1, h0 + kHomeMax);
        for (int i = threadIdx.x; i < kHomeMax; i += kBlock) s_f[i][0] = s_f[i][1] = s_f[i][2] = 0.0;
        __syncthreads();
        for (int u = 0; u < c.ninv[g]; ++u) {
            const CvDesc &cv = cs.cv[c.inv_cv[g][u]];
            const double cf = sign * coef[(int64_t)w * cs.D + cv.d] * (double)cv.scale;
            for (int r0 = 0;; r0 += kStageMax) {
                const int m = stage_partners(c, w, c.inv_p[g][u], home, r0, s_p, s_seg, s_sh);
                const int grp = lane / kLpa, gl = lane % kLpa;
                for (int ib = h0 + wave * kApw; ib < h1; ib += (kBlock / 64) * kApw) {
                    const int i = ib + grp;  // this lane group's home atom
                    const bool live = i < h1;
                    const float4 pi = sg[live ? i : h0];
                    const int32_t me = __float_as_int(pi.w);
                    const int mm = live ? m : 0;
                    float gx = 0.f, gy = 0.f, gz = 0.f;
                    for (int j0 = gl; j0 < m; j0 += kLpa * kUnroll) {
                        PairBatch b;
                        pair_batch(pi, me, s_p, j0, mm, cv, c, pos, aoff, b);
#pragma unroll
                        for (int q = 0; q < kUnroll; ++q) {
                            float sv, f;
                            sw<S612>(b.r2[q], cv, sv, f);
                            f = b.in[q] ? f : 0.f;
                            gx = fmaf(f, b.dx[q], gx);
                            gy = fmaf(f, b.dy[q], gy);
                            gz = fmaf(f, b.dz[q], gz);
                        }
                    }
                    // butterfly over the lane group (FP32: error ~ log2(16) ulp of the terms)
                    for (int o = kLpa / 2; o > 0; o >>= 1) {
                        gx += __shfl_xor(gx, o, 64);
                        gy += __shfl_xor(gy, o, 64);
                        gz += __shfl_xor(gz, o, 64);
                    }
                    if (gl == 0 && live) {  // one lane group per home atom: the only writer
                        s_f[i - h0][0] += cf * (double)gx;
                        s_f[i - h0][1] += cf * (double)gy;
                        s_f[i - h0][2] += cf * (double)gz;
                    }
                }
                if (r0 + m >= s_seg[27]) break;  // uniform
                __syncthreads();
            }
            __syncthreads();  // the next use restages s_p and its segments
        }
        for (int i = h0 + (int)threadIdx.x; i < h1; i += kBlock) {
            const int32_t atom = __float_as_int(sg[i].w);
            float *f = F.ptr + (aoff + atom) * F.sa;
            f[0] += (float)s_f[i - h0][0];
            f[F.sk] += (float)s_f[i - h0][1];
            f[2 * F.sk] += (float)s_f[i - h0][2];
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_cell_cv(const CellArgs &c, const CvSet &cs, const PosView &pos, double *xi, hipStream_t s)
{
    if (c.ncn == 0) return hipSuccess;
    if (pos.f64)
        hipLaunchKernelGGL(k_cell_build<double>, dim3(c.W * c.G), dim3(kBuildBlock), 0, s, c, pos);
    else
        hipLaunchKernelGGL(k_cell_build<float>, dim3(c.W * c.G), dim3(kBuildBlock), 0, s, c, pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int d = 0; d < cs.ncv; ++d) {  // one launch per CV: its switching form is a template choice
        const CvDesc &cv = cs.cv[d];
        if (cv.kind != CV_COORD_CELL) continue;
        if (cv.n == 6 && cv.m == 12)
            hipLaunchKernelGGL(k_cn_cell<true>, dim3(c.ncell, 1, c.W), dim3(kBlock), 0, s, c, cs, pos, cv.cn);
        else
            hipLaunchKernelGGL(k_cn_cell<false>, dim3(c.ncell, 1, c.W), dim3(kBlock), 0, s, c, cs, pos, cv.cn);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_cn_cell_fin, dim3(c.ncn, c.W), dim3(kBlock), 0, s, c, cs, xi);
    return hipGetLastError();
}

hipError_t launch_cell_vjp(const CellArgs &c, const CvSet &cs, const PosView &pos, const double *coef, double sign,
                           ForceView out, hipStream_t s)
{
    if (c.ncn == 0) return hipSuccess;
    bool all612 = true;
    for (int d = 0; d < cs.ncv; ++d)
        if (cs.cv[d].kind == CV_COORD_CELL) all612 = all612 && cs.cv[d].n == 6 && cs.cv[d].m == 12;
    if (all612)
        hipLaunchKernelGGL(k_cell_vjp<true>, dim3(c.ncell, c.G, c.W), dim3(kBlock), 0, s, c, cs, pos, coef, sign, out);
    else
        hipLaunchKernelGGL(k_cell_vjp<false>, dim3(c.ncell, c.G, c.W), dim3(kBlock), 0, s, c, cs, pos, coef, sign, out);
    return hipGetLastError();
}

}  // namespace sx
