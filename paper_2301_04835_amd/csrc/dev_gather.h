// Atomic-free gather of a bias force onto one walker's atoms (chain rule,
// Sec. 2: the bias force is added to the engine's forces):
//   F_i += sum over the Jacobian slots s of atom i of coef[cv(s)] * J_s
// Each walker's atoms are disjoint from every other walker's, and one lane
// owns one atom, so no two lanes write the same force entry.
#pragma once
#include "sx_internal.h"

namespace sx {

// touched atom u of walker w; Jw: the walker's slots (s x 3; JT float, or
// double on the ABF path)
template <typename JT>
__device__ __forceinline__ void gather_atom(const WalkerTabs &t, const JT *Jw, int32_t w, const double *coef,
                                            const ForceView &F, int u)
{
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int q = t.inv_ptr[u]; q < t.inv_ptr[u + 1]; ++q) {
        const int32_t s = t.inv_slot[q];
        const double cf = coef[t.slot_cv[s]];
        const JT *js = Jw + (int64_t)s * 3;
        fx += cf * (double)js[0];
        fy += cf * (double)js[1];
        fz += cf * (double)js[2];
    }
    float *f = F.ptr + (t.atom_off[w] + t.touched[u]) * F.sa;
    f[0] += (float)fx;
    f[F.sk] += (float)fy;
    f[2 * F.sk] += (float)fz;
}

// Force gather from the table in kernel-argument form (SmallTabs): lane
// u < U owns touched atom u of a walker whose atoms start at aoff and whose
// Jacobian slots start at Jw.  small_rows requests the atom's current force,
// the table row (the whole row: unused entries are zero, i.e. slot 0 of CV
// 0, which exists) and every Jacobian row it names, and waits for none of
// them; entries q >= nent are skipped where they are used.
struct SmallGather {
    float f0, f1, f2;
    float *dst;
};

__device__ __forceinline__ void small_rows(const SmallTabs &st, const float *Jw, const ForceView &F, int64_t aoff,
                                           int u, SmallGather &sg, int &nent, int32_t (&cvq)[kSmallPer],
                                           float (&jr)[kSmallPer][3])
{
    nent = st.nent[u];
    sg.dst = F.ptr + (aoff + st.touched[u]) * F.sa;
    sg.f0 = sg.dst[0];
    sg.f1 = sg.dst[F.sk];
    sg.f2 = sg.dst[2 * F.sk];
    int32_t e[kSmallPer];
#pragma unroll
    for (int q = 0; q < kSmallPer; ++q) e[q] = st.ent[u][q];
#pragma unroll
    for (int q = 0; q < kSmallPer; ++q) {
        const int32_t slot = e[q] & 0xFFFFF;
        cvq[q] = e[q] >> 20;
        jr[q][0] = Jw[slot * 3 + 0];
        jr[q][1] = Jw[slot * 3 + 1];
        jr[q][2] = Jw[slot * 3 + 2];
    }
}

// gather_atom in two halves, for kernels that know the coefficients only
// late: atom_rows requests touched atom u's first kAtomRows entries (their
// CVs and Jacobian rows) and its current force before the coefficients
// exist; atom_add then sums in the same order and arithmetic as gather_atom
// (entries past kAtomRows are read there, as gather_atom reads them).
constexpr int kAtomRows = 4;
template <typename JT>
struct AtomRows {
    int32_t q0, q1;
    int32_t cv[kAtomRows];
    JT j[kAtomRows][3];
    float f0, f1, f2;
    float *dst;
};

template <typename JT>
__device__ __forceinline__ void atom_rows(const WalkerTabs &t, const JT *Jw, int32_t w, const ForceView &F, int u,
                                          AtomRows<JT> &r)
{
    r.q0 = t.inv_ptr[u];
    r.q1 = t.inv_ptr[u + 1];  // > q0: a touched atom has a slot
#pragma unroll
    for (int k = 0; k < kAtomRows; ++k) {
        const int32_t s = t.inv_slot[min(r.q0 + k, r.q1 - 1)];
        r.cv[k] = t.slot_cv[s];
        r.j[k][0] = Jw[(int64_t)s * 3];
        r.j[k][1] = Jw[(int64_t)s * 3 + 1];
        r.j[k][2] = Jw[(int64_t)s * 3 + 2];
    }
    r.dst = F.ptr + (t.atom_off[w] + t.touched[u]) * F.sa;
    r.f0 = r.dst[0];
    r.f1 = r.dst[F.sk];
    r.f2 = r.dst[2 * F.sk];
}

template <typename JT>
__device__ __forceinline__ void atom_add(const WalkerTabs &t, const JT *Jw, const double *coef, const ForceView &F,
                                         const AtomRows<JT> &r)
{
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int k = 0; k < kAtomRows; ++k) {
        const bool use = r.q0 + k < r.q1;
        const double cf = coef[r.cv[k]];
        fx += use ? cf * (double)r.j[k][0] : 0.0;
        fy += use ? cf * (double)r.j[k][1] : 0.0;
        fz += use ? cf * (double)r.j[k][2] : 0.0;
    }
    for (int q = r.q0 + kAtomRows; q < r.q1; ++q) {
        const int32_t s = t.inv_slot[q];
        const double cf = coef[t.slot_cv[s]];
        const JT *js = Jw + (int64_t)s * 3;
        fx += cf * (double)js[0];
        fy += cf * (double)js[1];
        fz += cf * (double)js[2];
    }
    r.dst[0] = r.f0 + (float)fx;
    r.dst[F.sk] = r.f1 + (float)fy;
    r.dst[2 * F.sk] = r.f2 + (float)fz;
}

// the whole walker, lanes of the workgroup striding over its touched atoms
template <typename JT>
__device__ __forceinline__ void gather_forces(const WalkerTabs &t, const JT *Jw, int32_t w, const double *coef,
                                              const ForceView &F)
{
    for (int u = threadIdx.x; u < t.U; u += blockDim.x) gather_atom(t, Jw, w, coef, F, u);
}

}  // namespace sx
