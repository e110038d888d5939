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

}  // namespace sx
