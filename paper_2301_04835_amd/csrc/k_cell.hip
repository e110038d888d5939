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
//                  origin (float, ~6e-8 nm) and its atom index, and its
//                  sorted position is kept in member order.
//   k_cell_jac     one workgroup per (walker, group, column block of cells
//                  in z): the partner group's members in the cells around
//                  the block are staged in LDS relative to the block's
//                  origin (a cell's offset is its cell step times the cell
//                  edge, periodic wrap included), slice by slice, so each
//                  home cell's neighbours form one contiguous range; eight
//                  lanes own one home atom and walk that range: FP32 pair
//                  terms, the switch sum (the CV value, on the A side) and
//                  the gradient sum_j f(r_ij)(r_i - r_j) of each (CV, side)
//                  use, stored per member (no atomics, fixed order).
//   k_cn_cell_fin  per (walker, CV): the column-block partials in order.
//   k_cell_gather  the vector-Jacobian product from the stored gradients,
//                  one lane per member in member order (groups identical
//                  or disjoint: one writer per atom).

// Cut-length cells (edge >= the cutoff, >= 3 per dimension) are cut into rxy
// sub-cells in x and y and rz in z, so the (2 rxy + 1)^2 (2 rz + 1)
// neighbour sub-cells of a sub-cell are distinct and hold exactly the one
// image of every partner within the cutoff.  The sub-cells shrink the
// partners a home atom visits from 27 cut-length cubes to
// ((2 rxy + 1) / rxy)^2 (2 rz + 1) / rz: 14.1 at rxy = 2, rz = 4 (5.8 cut
// spheres' worth of volume down to 3.4).
#include "sx_internal.h"
#include "dev_cv.h"

namespace sx {
namespace {

constexpr int kBuildBlock = 1024;

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
    __shared__ int32_t s_off[kCellTotal];
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
    // pass 1: cells and counts, four members per thread at a time with their
    // loads issued together (a member past the group's end reads member b
    // instead and is dropped)
    for (int32_t b = tid; b < n; b += 4 * kBuildBlock) {
        double3 r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t i = b + k * kBuildBlock;
            r[k] = ld_pos_t<T>(pos, aoff + ga[i < n ? i : b]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t i = b + k * kBuildBlock;
            if (i >= n) break;
            double rel;
            const int cx = cell_of(r[k].x, c.L[0], c.inv_L[0], c.clen[0], c.nc[0], rel);
            const int cy = cell_of(r[k].y, c.L[1], c.inv_L[1], c.clen[1], c.nc[1], rel);
            const int cz = cell_of(r[k].z, c.L[2], c.inv_L[2], c.clen[2], c.nc[2], rel);
            const int cell = (cx * c.nc[1] + cy) * c.nc[2] + cz;
            cid[i] = cell;
            atomicAdd(&s_off[cell], 1);  // counts only: the placement below is ordered
        }
    }
    __syncthreads();
    // exclusive scan of the counts: kScanPer cells per thread, then across threads
    constexpr int kScanPer = kCellTotal / kBuildBlock;
    int32_t loc[kScanPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int cc = tid * kScanPer + q;
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
    for (int q = 0; q < kScanPer; ++q) {
        const int cc = tid * kScanPer + q;
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
        const int32_t atom = ga[valid ? i : base];  // in flight during the ranking
        const double3 r = ld_pos_t<T>(pos, aoff + atom);
        int rank = 0, cnt = 0;
        for (int k = 0; k < 64; ++k) {
            const int ck = __shfl(cell, k, 64);
            cnt += ck == cell ? 1 : 0;
            rank += (ck == cell && k < lane) ? 1 : 0;
        }
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) {
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
                cid[i] = dst;  // from here on: the member's sorted position
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

__device__ __forceinline__ const CvDesc &cell_cv(const CvSet &cs, int k)
{
    int c = 0;
    for (; c < cs.ncv - 1; ++c)
        if (cs.cv[c].kind == CV_COORD_CELL && cs.cv[c].cn == k) break;
    return cs.cv[c];
}

// Stage the members of group gp in the region of column block (cx, cy, z0):
// the n x n x (czb + 2 rz) sub-cells around it (n = 2 rxy + 1), slice by
// slice (z offset -rz .. czb + rz - 1), each slice in (x, y) order, so that
// the neighbour sub-cells of the block's k-th home sub-cell (z offsets
// -rz .. rz around it) are the contiguous range s_seg[n^2 k] ..
// s_seg[n^2 (k + 2 rz + 1)].  Positions
// relative to the origin of cell (cx, cy, z0), times sc; entries
// [r0, r0 + kColStage) of the region, followed by kStride atoms far outside
// any cut (index -1), so a lane reading four partners kLpa apart from any
// start below the count stays inside.  Returns how many are real.
constexpr int kJacBlock = 256;
constexpr int kLpa = 8;                     // lanes per home atom
constexpr int kApp = kJacBlock / kLpa;      // home atoms per pass
constexpr int kStride = 4 * kLpa;           // partners per lane step
constexpr int kColStage = 1536;             // partner atoms staged per round (24 KB)
constexpr int kRegMax = (2 * kXYReach + 1) * (2 * kXYReach + 1) * (kCzMax + 2 * kZReach);

constexpr int kRegPer = (kRegMax + kJacBlock - 1) / kJacBlock;  // region sub-cells per thread

// i + o wrapped into [0, n) for -n <= i + o < 2n (no division)
__device__ __forceinline__ int wrap_cell(int v, int n)
{
    v += v < 0 ? n : 0;
    return v >= n ? v - n : v;
}

template <int RXY>
__device__ __forceinline__ int stage_column(const CellArgs &c, int w, int gp, int cx, int cy, int z0, int czb, int r0,
                                            float sc, float4 *s_p, int32_t *s_seg, int32_t *s_first, int32_t *s_wsum)
{
    const int32_t *cst = c.cstart + ((int64_t)w * c.G + gp) * (c.ncell + 1);
    const float4 *srt = c.sorted + (int64_t)w * c.gtotal + c.goff[gp];
    constexpr int side = 2 * RXY + 1, nxy = side * side;  // RXY = c.rxy: divisions by constants
    const int nreg = nxy * (czb + 2 * c.rz);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // thread tid owns region sub-cells [tid kRegPer, (tid + 1) kRegPer): their
    // first sorted member to s_first and, until the scan below, their member
    // count to s_seg (one at a time: few registers live)
    int loc = 0;
#pragma unroll 1
    for (int q = 0; q < kRegPer; ++q) {
        const int t = tid * kRegPer + q;
        if (t >= nreg) break;
        const int sl = t / nxy, xy = t % nxy;
        const int ox = xy / side - RXY, oy = xy % side - RXY, oz = sl - c.rz;
        // |ox|, |oy| <= rxy < nc and -rz <= z0 + oz < nc2 + rz with rz <= nc2
        const int nx = wrap_cell(cx + ox, c.nc[0]), ny = wrap_cell(cy + oy, c.nc[1]);
        const int nz = wrap_cell(z0 + oz, c.nc[2]);
        const int nb = (nx * c.nc[1] + ny) * c.nc[2] + nz;
        const int f = cst[nb], n = cst[nb + 1] - f;
        s_first[t] = f;
        s_seg[t] = n;
        loc += n;
    }
    // exclusive scan of the counts over the workgroup: inclusive scan inside
    // each wavefront, then the wavefronts' totals in order
    int x = loc;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    int base = x - loc, total = 0;
#pragma unroll
    for (int wv = 0; wv < kJacBlock / 64; ++wv) {
        const int ws = s_wsum[wv];
        base += wv < wave ? ws : 0;
        total += ws;
    }
#pragma unroll 1
    for (int q = 0; q < kRegPer; ++q) {
        const int t = tid * kRegPer + q;
        if (t >= nreg) break;
        const int n = s_seg[t];  // this thread's own count
        s_seg[t] = base;
        base += n;
    }
    if (tid == 0) s_seg[nreg] = total;
    __syncthreads();
    // the window [r0, r0 + m) of the region, sub-cell by sub-cell: each
    // member shifted by its sub-cell's offset from the block origin
    const int m = min(kColStage, total - r0);
    for (int t = tid; t < nreg; t += blockDim.x) {
        const int sg = s_seg[t];
        const int e0 = max(sg, r0), e1 = min(s_seg[t + 1], r0 + m);
        if (e0 >= e1) continue;
        const int f = s_first[t];
        const int sl = t / nxy, xy = t % nxy;
        const int ox = xy / side - RXY, oy = xy % side - RXY, oz = sl - c.rz;
        const float shx = (float)(ox * c.clen[0]), shy = (float)(oy * c.clen[1]), shz = (float)(oz * c.clen[2]);
        for (int e = e0; e < e1; ++e) {
            float4 v = srt[f + (e - sg)];
            v.x = (v.x + shx) * sc;
            v.y = (v.y + shy) * sc;
            v.z = (v.z + shz) * sc;
            s_p[e - r0] = v;
        }
    }
    for (int j = m + tid; j < m + kStride; j += blockDim.x) s_p[j] = make_float4(1e6f, 1e6f, 1e6f, __int_as_float(-1));
    __syncthreads();
    return m;
}

// One workgroup of 256 threads per (column block, group, walker); kLpa
// lanes per home atom (the members of the block's cells, contiguous in the
// sorted order), kApp home atoms per pass.  For every use (CV, partner
// group) of the group each lane walks every kLpa-th partner of its home
// cell's contiguous range, four at a time, accumulating in FP32 the switch sum (A
// side of the CV: the CV value) and the gradient sum_j f(r_ij) (r_i - r_j);
// the atom's lanes combine in a fixed butterfly and the gradient is stored per
// member and use (the VJP reads it).  A group's own CV counts its self pair
// (r = 0: s = 1 exactly, zero gradient), so the A-side sum drops 1 per atom
// instead of testing every pair.
// Four partners p[0], p[kLpa], p[2 kLpa], p[3 kLpa] of one home atom (o):
// the cut decision, the switch sum and the gradient sum.  In the (6, 12)
// form the coordinates are in units of r0 (x^2 = r^2 / r0^2 directly) and
// the gradient term is x^4 s^2 (r_i - r_j) / r0, the factor -6 / r0 applied
// once per atom; otherwise plain units and f of switch_fn.  TAIL: partners
// at or past pe do not count.  SIDEA: the switch sum is wanted (the A side
// of the CV); on the B side only the gradient is.
//
// The cut enters the (6, 12) switch without a select: t = (r^2 - rc^2) 2^100
// (one fma; scaling by a power of two keeps the rounding of r^2 - rc^2, so
// the decision and its band are those of the unscaled difference), and
// s = 1 / max(1 + x^6, t).  Inside the cut t < 0 and s is the switch; a
// partner decided outside (outside the band) has t > 2^100 * 1e-5 rc^2
// (rc^2 in r0 units: 7e25 at rc = 2.4 r0, above 3e24 for any cut beyond
// r0 / 2), so s < 3e-25 and x^4 s^2 underflows to zero or a denormal: it
// adds nothing measurable to the gradient and less than 3e-25 to the switch
// sum, far below the sum's last bit.  Partners that do not count (tail,
// exact decision outside) get t = +inf, s = 0.
constexpr float kTScale = 0x1p100f;

template <bool S612, bool TAIL, bool SIDEA>
__device__ __forceinline__ void pair4(const float4 *p, const float4 *pe, float3 o, float rc2s, float bandcs,
                                      float rc2, const CvDesc &cv, const CellArgs &c, const PosView &pos,
                                      int64_t aoff, int32_t me, float &sA, float &gx, float &gy, float &gz)
{
    float dx[4], dy[4], dz[4], r2[4], t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 pj = p[q * kLpa];  // < pe + kStride: padded
        dx[q] = o.x - pj.x;
        dy[q] = o.y - pj.y;
        dz[q] = o.z - pj.z;
        r2[q] = fmaf(dx[q], dx[q], fmaf(dy[q], dy[q], dz[q] * dz[q]));
        t[q] = S612 ? fmaf(r2[q], kTScale, -rc2s) : r2[q] - rc2;
        if (TAIL && p + q * kLpa >= pe) t[q] = __builtin_inff();
    }
    const float tmin = fminf(fminf(fabsf(t[0]), fabsf(t[1])), fminf(fabsf(t[2]), fabsf(t[3])));
    if (tmin <= bandcs) {  // rare: the edge of the cut
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (fabsf(t[q]) <= bandcs)
                t[q] = cut_exact(pos, aoff, me, __float_as_int(p[q * kLpa].w), c.L[0], c.L[1], c.L[2], cv.rcut)
                           ? -1.0f
                           : __builtin_inff();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float f;
        if (S612) {
            const float x4 = r2[q] * r2[q];
            // max(1 + x^6, t) on the bit patterns: 1 + x^6 is positive, so
            // the signed-integer order agrees with the float order here
            const float den = __int_as_float(max(__float_as_int(fmaf(x4, r2[q], 1.0f)), __float_as_int(t[q])));
            const float sv = __builtin_amdgcn_rcpf(den);
            if (SIDEA) sA += sv;
            f = x4 * sv * sv;
        } else {
            const bool in = t[q] < 0.f;
            float sv;
            switch_fn(r2[q], cv, sv, f);
            if (SIDEA) sA += in ? sv : 0.f;
            f = in ? f : 0.f;
        }
        gx = fmaf(f, dx[q], gx);
        gy = fmaf(f, dy[q], gy);
        gz = fmaf(f, dz[q], gz);
    }
}

// One home atom's partners [p, pe) of the staged window, every kLpa-th from
// this lane's start, four per step; pe3 = max(pe - 3 kLpa, window start):
// a step starting below pe3 reads only partners below pe.
template <bool S612, bool SIDEA>
__device__ __forceinline__ void home_pairs(const float4 *p, const float4 *pe, const float4 *pe3, float3 o,
                                           float rc2s, float bandcs, float rc2, const CvDesc &cv, const CellArgs &c,
                                           const PosView &pos, int64_t aoff, int32_t me, float &sA, float &gx,
                                           float &gy, float &gz)
{
    for (; p < pe3; p += kStride)
        pair4<S612, false, SIDEA>(p, pe, o, rc2s, bandcs, rc2, cv, c, pos, aoff, me, sA, gx, gy, gz);
    if (p < pe) pair4<S612, true, SIDEA>(p, pe, o, rc2s, bandcs, rc2, cv, c, pos, aoff, me, sA, gx, gy, gz);
}

template <bool S612, int RXY>
__global__ void __launch_bounds__(kJacBlock, 5) k_cell_jac(CellArgs c, CvSet cs, PosView pos)
{
    __shared__ float4 s_p[kColStage + kStride];
    __shared__ int32_t s_seg[kRegMax + 1], s_first[kRegMax], s_wsum[kJacBlock / 64];
    __shared__ double s_red[kJacBlock / 64];
    __shared__ int32_t s_home[kCzMax + 1];  // sorted position of the block's home cells
    const int blk = blockIdx.x, g = blockIdx.y, w = blockIdx.z;
    const int tid = threadIdx.x, sub = tid & (kLpa - 1), wave = tid >> 6;
    const int zb = blk % c.nzb, cy = (blk / c.nzb) % c.nc[1], cx = blk / (c.nzb * c.nc[1]);
    // blocks split the column evenly: nzb blocks of at most kCzMax cells
    const int z0 = zb * c.nc[2] / c.nzb, czb = (zb + 1) * c.nc[2] / c.nzb - z0;
    const int32_t *cst = c.cstart + ((int64_t)w * c.G + g) * (c.ncell + 1);
    const float4 *sg = c.sorted + (int64_t)w * c.gtotal + c.goff[g];
    const int cell0 = (cx * c.nc[1] + cy) * c.nc[2] + z0;
    if (tid <= czb) s_home[tid] = cst[cell0 + tid];
    __syncthreads();
    const int a0 = s_home[0], a1 = s_home[czb];
    const int64_t aoff = c.atom_off[w];
    constexpr int nxy = (2 * RXY + 1) * (2 * RXY + 1);  // RXY = c.rxy
    const int nreg = nxy * (czb + 2 * c.rz), span = nxy * (2 * c.rz + 1);
    for (int u = 0; u < c.ninv[g]; ++u) {
        const CvDesc &cv = cs.cv[c.inv_cv[g][u]];
        const bool sideA = c.inv_side[g][u] == 0;
        const float self1 = cv.ga == cv.gb ? 1.0f : 0.0f;
        float4 *J = c.jac + (int64_t)w * c.jtotal + c.joff[g][u];
        // coordinate scale, squared cut, its band, and the gradient factor
        const float sc = S612 ? cv.inv_r0 : 1.0f;
        const float rc2 = cv.rcut2 * sc * sc, bandc = 1e-5f * rc2, gsc = S612 ? -6.0f * cv.inv_r0 : 1.0f;
        // the cut test's difference and band in the units of pair4's t
        const float rc2s = S612 ? rc2 * kTScale : rc2, bandcs = S612 ? bandc * kTScale : bandc;
        double ssum = 0.0;  // this lane's switch sums (A side), over its home atoms
        for (int r0 = 0;; r0 += kColStage) {
            const int m = stage_column<RXY>(c, w, c.inv_p[g][u], cx, cy, z0, czb, r0, sc, s_p, s_seg, s_first, s_wsum);
            for (int h0 = a0; h0 + (64 / kLpa) * wave < a1; h0 += kApp) {  // uniform per wavefront
                const int i = h0 + tid / kLpa;
                const bool live = i < a1;
                const float4 pi = sg[live ? i : a0];
                int k = 0;  // this atom's home cell within the block: the last k with s_home[k] <= i
                for (int hi = czb - 1; k < hi;) {
                    const int mid = (k + hi + 1) >> 1;
                    if (s_home[mid] <= i) k = mid; else hi = mid - 1;
                }
                // this atom's partners in the staged window
                const int b0 = max(0, s_seg[nxy * k] - r0), b1 = live ? min(m, s_seg[nxy * k + span] - r0) : 0;
                // home atoms are stored relative to their own cell: the k-th
                // cell of the block sits k cell edges above the block origin
                const float3 o = make_float3(pi.x * sc, pi.y * sc, (pi.z + (float)(k * c.clen[2])) * sc);
                const int32_t me = __float_as_int(pi.w);
                float sA = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
                const float4 *const p0 = s_p + (b0 + sub), *const pe = s_p + b1;
                const float4 *const pe3 = s_p + max(b1 - 3 * kLpa, 0);
                if (sideA)
                    home_pairs<S612, true>(p0, pe, pe3, o, rc2s, bandcs, rc2, cv, c, pos, aoff, me, sA, gx, gy, gz);
                else
                    home_pairs<S612, false>(p0, pe, pe3, o, rc2s, bandcs, rc2, cv, c, pos, aoff, me, sA, gx, gy, gz);
#pragma unroll
                for (int o = 1; o < kLpa; o <<= 1) {
                    sA += __shfl_xor(sA, o, 64);
                    gx += __shfl_xor(gx, o, 64);
                    gy += __shfl_xor(gy, o, 64);
                    gz += __shfl_xor(gz, o, 64);
                }
                if (sub == 0 && live) {
                    float4 gv = make_float4(gx * gsc, gy * gsc, gz * gsc, 0.f);
                    if (r0 > 0) {  // later windows add to the earlier ones (same thread)
                        const float4 pv = J[i];
                        gv.x += pv.x;
                        gv.y += pv.y;
                        gv.z += pv.z;
                    }
                    J[i] = gv;
                    if (sideA) ssum += (double)sA - (r0 == 0 ? (double)self1 : 0.0);
                }
            }
            const bool last = r0 + m >= s_seg[nreg];  // uniform
            __syncthreads();  // the next window or use restages
            if (last) break;
        }
        if (sideA) {  // the CV's partial over this block: fixed butterfly, then waves in order
            for (int o = 32; o > 0; o >>= 1) ssum += __shfl_xor(ssum, o, 64);
            if ((tid & 63) == 0) s_red[wave] = ssum;
            __syncthreads();
            if (tid == 0) {
                double t = s_red[0];
                for (int q = 1; q < kJacBlock / 64; ++q) t += s_red[q];
                c.part[((int64_t)w * c.ncn + cv.cn) * c.nblk + blk] = t;
            }
        }
    }
}

// per (walker, CV): the column-block partials of its A side in block order
__global__ void __launch_bounds__(kBlock) k_cn_cell_fin(CellArgs c, CvSet cs, double *xi)
{
    __shared__ double s_red[kBlock / 64];
    const int k = blockIdx.x, w = blockIdx.y;
    const CvDesc cv = cell_cv(cs, k);
    const double *p = c.part + ((int64_t)w * c.ncn + k) * c.nblk;
    double v = 0.0;
    for (int i = threadIdx.x; i < c.nblk; i += kBlock) v += p[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = s_red[0];
        for (int q = 1; q < kBlock / 64; ++q) t += s_red[q];
        xi[(int64_t)w * cs.D + cv.d] = t * (double)cv.scale;
    }
}

// VJP from the stored gradients: one lane per member of each group in
// member order, out += sign sum over the group's uses of coef[cv] scale_cv J,
// J read at the member's sorted position (left in cid by the build); the
// groups are identical or disjoint, so every atom has one writer.  Members
// listed in atom order make the force updates contiguous; the gradient
// reads land anywhere in the walker's records, so all blocks of one walker
// run on one XCD (blocks are dealt to the 8 XCDs in turn): block b serves
// walker 8 (k / nch) + b % 8, chunk k % nch, k = b / 8, and those records
// pass through one L2.
__global__ void __launch_bounds__(kBlock) k_cell_gather(CellArgs c, CvSet cs, const double *coef, double sign,
                                                         ForceView F, int32_t nch)
{
    const int k = blockIdx.x / 8;
    const int w = (k / nch) * 8 + (int)(blockIdx.x % 8);
    const int64_t e = (int64_t)(k % nch) * blockDim.x + threadIdx.x;
    if (w >= c.W || e >= c.gtotal) return;
    int g = 0;
    while (g + 1 < c.G && e >= c.goff[g + 1]) ++g;
    const int32_t atom = c.gatoms[e];
    const int32_t sp = c.cid[(int64_t)w * c.gtotal + e];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int u = 0; u < c.ninv[g]; ++u) {
        const CvDesc &cv = cs.cv[c.inv_cv[g][u]];
        const double cf = sign * coef[(int64_t)w * cs.D + cv.d] * (double)cv.scale;
        const float4 j = c.jac[(int64_t)w * c.jtotal + c.joff[g][u] + sp];
        fx += cf * (double)j.x;
        fy += cf * (double)j.y;
        fz += cf * (double)j.z;
    }
    float *f = F.ptr + (c.atom_off[w] + atom) * F.sa;
    f[0] += (float)fx;
    f[F.sk] += (float)fy;
    f[2 * F.sk] += (float)fz;
}

}  // namespace

hipError_t launch_cell_cv(const CellArgs &c, const CvSet &cs, const PosView &pos, double *xi, hipStream_t s, int which)
{
    if (c.ncn == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (which & 1) {
        if (pos.f64)
            hipLaunchKernelGGL(k_cell_build<double>, dim3(c.W * c.G), dim3(kBuildBlock), 0, s, c, pos);
        else
            hipLaunchKernelGGL(k_cell_build<float>, dim3(c.W * c.G), dim3(kBuildBlock), 0, s, c, pos);
        e = hipGetLastError();
        if (e != hipSuccess || !(which & 2)) return e;
    }
    bool all612 = true;
    for (int d = 0; d < cs.ncv; ++d)
        if (cs.cv[d].kind == CV_COORD_CELL) all612 = all612 && cs.cv[d].n == 6 && cs.cv[d].m == 12;
    const dim3 grid(c.nblk, c.G, c.W);
    if (c.rxy != 1 && c.rxy != 2) return hipErrorInvalidValue;
    if (all612 && c.rxy == 2)
        hipLaunchKernelGGL((k_cell_jac<true, 2>), grid, dim3(kJacBlock), 0, s, c, cs, pos);
    else if (all612)
        hipLaunchKernelGGL((k_cell_jac<true, 1>), grid, dim3(kJacBlock), 0, s, c, cs, pos);
    else if (c.rxy == 2)
        hipLaunchKernelGGL((k_cell_jac<false, 2>), grid, dim3(kJacBlock), 0, s, c, cs, pos);
    else
        hipLaunchKernelGGL((k_cell_jac<false, 1>), grid, dim3(kJacBlock), 0, s, c, cs, pos);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cn_cell_fin, dim3(c.ncn, c.W), dim3(kBlock), 0, s, c, cs, xi);
    return hipGetLastError();
}

hipError_t launch_cell_vjp(const CellArgs &c, const CvSet &cs, const PosView &, const double *coef, double sign,
                           ForceView out, hipStream_t s)
{
    if (c.ncn == 0) return hipSuccess;
    const int32_t nch = (int32_t)((c.gtotal + kBlock - 1) / kBlock);
    const int64_t nb = (int64_t)nch * ((c.W + 7) / 8) * 8;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cell_gather, dim3((unsigned)nb), dim3(kBlock), 0, s, c, cs, coef, sign, out, nch);
    return hipGetLastError();
}

}  // namespace sx
