// Device helpers shared by the CV kernels and the fused hill-sum kernels:
// strided position loads and the dihedral angle with its gradient.
#pragma once

#include "sx_internal.h"

namespace sx {

template <typename T>
__device__ __forceinline__ double3 ld_pos_t(const PosView &p, int64_t i)
{
    const T *q = static_cast<const T *>(p.ptr) + i * p.sa;
    return make_double3((double)q[0], (double)q[p.sk], (double)q[2 * p.sk]);
}

__device__ __forceinline__ double3 ld_pos(const PosView &p, int64_t i)
{
    if (p.f64) {
        const double *q = static_cast<const double *>(p.ptr) + i * p.sa;
        return make_double3(q[0], q[p.sk], q[2 * p.sk]);
    }
    const float *q = static_cast<const float *>(p.ptr) + i * p.sa;
    return make_double3((double)q[0], (double)q[p.sk], (double)q[2 * p.sk]);
}

__device__ __forceinline__ double3 d3sub(double3 a, double3 b) { return make_double3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ double d3dot(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double3 d3cross(double3 a, double3 b)
{
    return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double3 d3scale(double3 a, double s) { return make_double3(a.x * s, a.y * s, a.z * s); }

// Dihedral of r0..r3 in the IUPAC sign convention, range (-pi, pi].
// With F = r0 - r1, G = r1 - r2, H = r3 - r2, A = F x G, B = H x G:
//   phi = atan2(-|G| F.B, A.B)
//   dphi/dr0 = -|G|/|A|^2 A,   dphi/dr3 = |G|/|B|^2 B,
//   dphi/dr1 = (|G|/|A|^2 + F.G/(|A|^2 |G|)) A - H.G/(|B|^2 |G|) B,
//   dphi/dr2 = -(|G|/|B|^2 - H.G/(|B|^2 |G|)) B - F.G/(|A|^2 |G|) A
// (Blondel & Karplus 1996).  FP64 throughout.
template <bool GRAD>
__device__ __forceinline__ double dihedral_fp64(const double3 (&r)[4], double3 (&g)[4])
{
    const double3 F = d3sub(r[0], r[1]), G = d3sub(r[1], r[2]), H = d3sub(r[3], r[2]);
    const double3 A = d3cross(F, G), B = d3cross(H, G);
    const double lg = sqrt(d3dot(G, G));
    const double phi = atan2(-lg * d3dot(F, B), d3dot(A, B));
    if (GRAD) {
        const double ia = 1.0 / d3dot(A, A), ib = 1.0 / d3dot(B, B), ig = 1.0 / lg;
        const double fg = d3dot(F, G) * ia * ig, hg = d3dot(H, G) * ib * ig;
        g[0] = d3scale(A, -lg * ia);
        g[3] = d3scale(B, lg * ib);
        g[1] = d3sub(d3scale(A, lg * ia + fg), d3scale(B, hg));
        g[2] = d3sub(d3scale(B, hg - lg * ib), d3scale(A, fg));
    }
    return phi;
}

// Dihedral CV `cv` of the walker whose first atom is aoff; T is the
// position type, so the twelve coordinate loads are straight-line code.
template <typename T, bool GRAD>
__device__ __forceinline__ double dihedral_at_t(const CvDesc &cv, const PosView &pos, int64_t aoff, double3 (&g)[4])
{
    double3 r[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) r[s] = ld_pos_t<T>(pos, aoff + cv.atom[s]);
    return dihedral_fp64<GRAD>(r, g);
}

template <bool GRAD>
__device__ __forceinline__ double dihedral_at(const CvDesc &cv, const PosView &pos, int64_t aoff, double3 (&g)[4])
{
    return pos.f64 ? dihedral_at_t<double, GRAD>(cv, pos, aoff, g) : dihedral_at_t<float, GRAD>(cv, pos, aoff, g);
}

// Rational switch s = (1 - x^n)/(1 - x^m), x = r/r0, and f = (1/r) ds/dr.
// (6, 12): s = 1/(1 + x^6) and f = -6 x^4 s^2 / r0^2, both from r^2 alone.
// Other (n, m): s = P_n(x)/P_m(x) with P_k(x) = 1 + x + ... + x^(k-1), the
// same rational function with the factor (1 - x) cancelled, which stays
// exact around x = 1 where the plain quotient loses all its digits.
__device__ __forceinline__ void switch_fn(float r2, const CvDesc &c, float &s, float &f)
{
    if (c.n == 6 && c.m == 12) {
        float x2 = r2 * (c.inv_r0 * c.inv_r0);
        float x4 = x2 * x2;
        float sv = __builtin_amdgcn_rcpf(1.0f + x4 * x2);
        s = sv;
        f = -6.0f * x4 * sv * sv * (c.inv_r0 * c.inv_r0);
        return;
    }
    float r = sqrtf(r2), x = r * c.inv_r0;
    float pn = 0.f, dpn = 0.f, pm = 0.f, dpm = 0.f;
    for (int i = c.n - 1; i >= 0; --i) {  // Horner: P and P'
        dpn = fmaf(dpn, x, pn);
        pn = fmaf(pn, x, 1.0f);
    }
    for (int i = c.m - 1; i >= 0; --i) {
        dpm = fmaf(dpm, x, pm);
        pm = fmaf(pm, x, 1.0f);
    }
    float ipm = __builtin_amdgcn_rcpf(pm);
    s = pn * ipm;
    float dsdx = (dpn * pm - pn * dpm) * ipm * ipm;
    f = r > 0.f ? dsdx * c.inv_r0 / r : 0.f;
}

// The same switch in FP64 (IEEE division and square root), for the pair
// terms of a Jacobian kept in FP64.
__device__ __forceinline__ void switch_fn(double r2, const CvDesc &c, double &s, double &f)
{
    const double ir = c.inv_r0d;
    if (c.n == 6 && c.m == 12) {
        const double x2 = r2 * (ir * ir), x4 = x2 * x2;
        const double sv = 1.0 / (1.0 + x4 * x2);
        s = sv;
        f = -6.0 * x4 * sv * sv * (ir * ir);
        return;
    }
    const double r = sqrt(r2), x = r * ir;
    double pn = 0.0, dpn = 0.0, pm = 0.0, dpm = 0.0;
    for (int i = c.n - 1; i >= 0; --i) {
        dpn = fma(dpn, x, pn);
        pn = fma(pn, x, 1.0);
    }
    for (int i = c.m - 1; i >= 0; --i) {
        dpm = fma(dpm, x, pm);
        pm = fma(pm, x, 1.0);
    }
    s = pn / pm;
    const double dsdx = (dpn * pm - pn * dpm) / (pm * pm);
    f = r > 0.0 ? dsdx * ir / r : 0.0;
}

}  // namespace sx
