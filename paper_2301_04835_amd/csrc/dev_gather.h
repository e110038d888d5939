// Atomic-free gather of a bias force onto one walker's atoms (chain rule,
// Sec. 2: the bias force is added to the engine's forces):
//   F_i += sum over the Jacobian slots s of atom i of coef[cv(s)] * J_s
// Each walker's atoms are disjoint from every other walker's, and one lane
// owns one atom, so no two lanes write the same force entry.
#pragma once
#include "sx_internal.h"

namespace sx {

// touched atom u of walker w; Jw: the walker's slots (s x 3 floats)
__device__ __forceinline__ void gather_atom(const WalkerTabs &t, const float *Jw, int32_t w, const double *coef,
                                            const ForceView &F, int u)
{
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int q = t.inv_ptr[u]; q < t.inv_ptr[u + 1]; ++q) {
        const int32_t s = t.inv_slot[q];
        const double cf = coef[t.slot_cv[s]];
        const float *js = Jw + (int64_t)s * 3;
        fx += cf * (double)js[0];
        fy += cf * (double)js[1];
        fz += cf * (double)js[2];
    }
    float *f = F.ptr + (t.atom_off[w] + t.touched[u]) * F.sa;
    f[0] += (float)fx;
    f[F.sk] += (float)fy;
    f[2 * F.sk] += (float)fz;
}

// the whole walker, lanes of the workgroup striding over its touched atoms
__device__ __forceinline__ void gather_forces(const WalkerTabs &t, const float *Jw, int32_t w, const double *coef,
                                              const ForceView &F)
{
    for (int u = threadIdx.x; u < t.U; u += blockDim.x) gather_atom(t, Jw, w, coef, F, u);
}

}  // namespace sx
