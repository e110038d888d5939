// Bias surrogate: a small tanh network of the CVs fitted to the hill sum.
// The paper's neural-network methods (ANN, Sec. 2.1.7; FUNN, Sec. 2.1.8)
// bias with such networks; here the network stands in for the exact hill
// sum of Sec. 2.1.5 on a frozen bias, with the exact sum as fallback.
//
//   features f(xi): (sin xi_d, cos xi_d) periodic, (u_d, u_d^2) otherwise
//   z1 = W1 f + b1, a1 = tanh z1, z2 = W2 a1 + b2, a2 = tanh z2, y = w3.a2 + b3
//   dy/dxi_d: one forward tangent per CV through the same layers
//
// Kernels
//   k_mlp_fwd   (matrix cores): one wavefront per 16 samples.  Layer 1 and
//               its tangents are VALU (F <= 6 inputs); a1 and the tangents
//               da1_d enter v_mfma_f32_16x16x32_bf16 as bf16 pairs
//               (hi = bf16(x), lo = bf16(x - hi): about 16 significant bits)
//               against W2 in bf16, FP32 accumulation, so 2 (1 + D) products
//               share every W2 fragment.  y and dy/dxi are reduced across
//               the 16 output lanes of each sample with shuffles.
//   k_mlp_bwd   (training): reverse mode over the forward and its tangents
//               for a Sobolev loss on (V, dV/dxi); 16 samples per workgroup
//               (8 at H = 128) in LDS; the two H x H products (back through
//               W2, and the W2 gradient) on the matrix cores with bf16-pair
//               operands, the rest on VALU; per-workgroup gradients.
//   k_mlp_adam  sums the workgroup gradients in order (FP64) and applies
//               Adam (Kingma & Ba 2015) to the FP32 master weights, then
//               refreshes their bf16 copies.
#include "sx_internal.h"
#include "dev_cv.h"
#include "dev_gather.h"

namespace sx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSamplesPerWave = 16;

// parameter offsets (FP32 master and bf16 copies share the layout)
struct POff {
    int W1, b1, W2, b2, w3, b3, P;
};
__host__ __device__ constexpr POff poff(int H, int F)
{
    return POff{0, H * F, H * F + H, H * F + H + H * H, H * F + 2 * H + H * H, H * F + 3 * H + H * H,
                H * F + 3 * H + H * H + 1};
}

__device__ __forceinline__ float bf(const uint16_t *p, int i) { return (float)reinterpret_cast<const __bf16 *>(p)[i]; }

// tanh x = sign(x) (1 - 2 / (exp(2|x|) + 1)) with v_exp_f32 and v_rcp_f32:
// absolute error a few 1e-8, no overflow (exp -> inf gives 1)
__device__ __forceinline__ float tanh_fast(float x)
{
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * fabsf(x));  // 2 log2(e) |x|
    const float t = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
    return copysignf(t, x);
}

// features and their CV tangents for one sample
template <int D>
__device__ __forceinline__ void featurize(const MlpArgs &a, const double *xi, float (&f)[2 * D],
                                          float (&u)[D][2 * D])
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int q = 0; q < 2 * D; ++q) u[d][q] = 0.f;
        const double x = xi[d];
        if (a.periodic[d]) {
            double s, c;
            sincos(x, &s, &c);
            f[2 * d] = (float)s;
            f[2 * d + 1] = (float)c;
            u[d][2 * d] = (float)c;
            u[d][2 * d + 1] = (float)-s;
        } else {
            const double z = (x - a.mu[d]) * a.inv_s[d];
            f[2 * d] = (float)z;
            f[2 * d + 1] = (float)(z * z);
            u[d][2 * d] = (float)a.inv_s[d];
            u[d][2 * d + 1] = (float)(2.0 * z * a.inv_s[d]);
        }
    }
}

// ------------------------------------------------------------------ forward
// n samples xi[n][D] (FP64).  Outputs (each may be null): V[n], dV[n][D]
// (FP64); for training, the per-sample a2[n][H], dz2[D][n][H], y[n],
// dy[n][D] (FP32).  Inference with a certification mask: mask != null marks
// samples whose cell is not certified (flag[i] = 1).
// certification flag of one sample: 1 if its cell of the cert_n^D grid is
// not certified (or lies outside the grid)
template <int D>
__device__ __forceinline__ uint8_t fallback_flag(const MlpArgs &a, const double *x)
{
    int64_t cell = 0;
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        int64_t i = (int64_t)floor((x[d] - a.cert_lo[d]) * a.cert_inv_h[d]);
        if (a.periodic[d]) {
            i %= a.cert_n;
            if (i < 0) i += a.cert_n;
        } else if (i < 0 || i >= a.cert_n) {
            inside = false;
        }
        cell = cell * a.cert_n + (inside ? i : 0);
    }
    return (inside && a.mask[cell]) ? 0 : 1;
}

// A surrogate step's CVs (every CV a dihedral): dihedral d of sample si,
// its four positions requested by dihedral_atoms at the start of the
// kernel, the angle and its gradient formed in FP64 by step_dihedral, which
// stores xi and the Jacobian slots.
template <typename T, int D>
__device__ __forceinline__ void dihedral_atoms(const MlpStep &st, int64_t si, int d, double3 (&r)[4])
{
    const int64_t aoff = st.tabs.atom_off[si];
    int32_t at[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) at[q] = st.cs.cv[0].atom[q];
#pragma unroll
    for (int dd = 1; dd < D; ++dd)
#pragma unroll
        for (int q = 0; q < 4; ++q) at[q] = d == dd ? st.cs.cv[dd].atom[q] : at[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = ld_pos_t<T>(st.pos, aoff + at[q]);
}

template <int D>
__device__ __forceinline__ double step_dihedral(const MlpStep &st, int64_t si, int d, const double3 (&r)[4])
{
    int32_t slot0 = st.cs.cv[0].slot0;
#pragma unroll
    for (int dd = 1; dd < D; ++dd) slot0 = d == dd ? st.cs.cv[dd].slot0 : slot0;
    double3 g[4];
    const double x = dihedral_fp64<true>(r, g);
    st.xi_ws[si * D + d] = x;
    float *js = st.J + (si * st.nslots + slot0) * 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        js[3 * q] = (float)g[q].x;
        js[3 * q + 1] = (float)g[q].y;
        js[3 * q + 2] = (float)g[q].z;
    }
    return x;
}

template <int H, int D, bool CVF>
__global__ void __launch_bounds__(kBlock) k_mlp_fwd(MlpArgs a, const double *xi, int64_t n, double *V, double *dV,
                                                     float *t_a2, float *t_dz2, float *t_y, float *t_dy,
                                                     uint8_t *flag, MlpStep st, int32_t step_on)
{
    constexpr int F = 2 * D;
    constexpr int KB = H / 32;  // 32-wide K blocks of the H x H product
    constexpr int NT = H / 16;  // 16-wide output tiles
    constexpr POff o = poff(H, F);
    static_assert(D <= 4, "a surrogate step gives each dihedral one of the four row groups");
    __shared__ double s_coef[kSamplesPerWave][D];  // surrogate step: -dV/dxi per sample
    __shared__ uint8_t s_fb[kSamplesPerWave];
    const int lane = threadIdx.x & 63;
    const int64_t s0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * kSamplesPerWave;
    // whole wavefront idle; its workgroup is this wavefront alone whenever the
    // one barrier below is used
    if (s0 >= n) return;
    const int row = lane & 15, kg = lane >> 4;
    const int64_t si = s0 + row;  // this lane's sample in the A operand
    const bool live = si < n;
    // a surrogate step: the lanes of row group kg < D evaluate dihedral kg
    // of their walker; its positions are requested first, then every weight
    // this lane will use (layer 1, the layer-2 fragments, b2, w3 and b3),
    // which arrive during the angles
    const bool cv_lane = CVF && live && kg < D;
    double3 rr[4];
    if (cv_lane) {
        if (st.pos.f64)
            dihedral_atoms<double, D>(st, si, kg, rr);
        else
            dihedral_atoms<float, D>(st, si, kg, rr);
    }
    float w1p[CVF ? KB : 1][8][F], b1p[CVF ? KB : 1][8], b2p[CVF ? NT : 1], w3p[CVF ? NT : 1], b3p = 0.f;
    bf16x8 w2p[CVF ? NT : 1][CVF ? KB : 1];
    if (CVF) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            b2p[nt] = bf(a.Pb, o.b2 + nt * 16 + row);
            w3p[nt] = bf(a.Pb, o.w3 + nt * 16 + row);
        }
        b3p = bf(a.Pb, o.b3);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = kb * 32 + kg * 8 + t;
                b1p[kb][t] = bf(a.Pb, o.b1 + k);
#pragma unroll
                for (int q = 0; q < F; ++q) w1p[kb][t][q] = bf(a.Pb, o.W1 + k * F + q);
            }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                w2p[nt][kb] = *reinterpret_cast<const bf16x8 *>(a.Pb + o.W2 + (nt * 16 + row) * H + kb * 32 + kg * 8);
    }
    double x[D];
    if (CVF) {
        // lane (kg, row) with kg < D forms dihedral kg of sample `row` (FP64)
        // and stores it and its Jacobian slots; shuffles hand every lane its
        // sample's D angles
        const double xd = cv_lane ? step_dihedral<D>(st, si, kg, rr) : 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = __shfl(xd, d * 16 + row, 64);
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = live ? xi[si * D + d] : 0.0;
    }
    float f[F], u[D][F];
    featurize<D>(a, x, f, u);
    // the certification flag of this lane's sample, requested here so that
    // the mask read overlaps the network
    int fb_row = 0;
    if (flag && live) fb_row = fallback_flag<D>(a, x);
    // layer 1 for this lane's 8 K entries of every K block (+ tangents),
    // each split into bf16 hi and lo parts
    bf16x8 av[KB], al[KB], tv[D][KB], tl[D][KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = kb * 32 + kg * 8 + t;
            float z = CVF ? b1p[CVF ? kb : 0][t] : bf(a.Pb, o.b1 + k);
            float dz[D];
#pragma unroll
            for (int d = 0; d < D; ++d) dz[d] = 0.f;
#pragma unroll
            for (int q = 0; q < F; ++q) {
                const float w = CVF ? w1p[CVF ? kb : 0][t][q] : bf(a.Pb, o.W1 + k * F + q);
                z = fmaf(w, f[q], z);
#pragma unroll
                for (int d = 0; d < D; ++d) dz[d] = fmaf(w, u[d][q], dz[d]);
            }
            const float a1 = tanh_fast(z);
            const __bf16 h = (__bf16)a1;
            av[kb][t] = h;
            al[kb][t] = (__bf16)(a1 - (float)h);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float da = (1.f - a1 * a1) * dz[d];
                const __bf16 dh = (__bf16)da;
                tv[d][kb][t] = dh;
                tl[d][kb][t] = (__bf16)(da - (float)dh);
            }
        }
    // layer 2 on the matrix cores, one 16-wide output tile at a time
    float yp[4] = {0.f, 0.f, 0.f, 0.f}, dyp[D][4];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int r = 0; r < 4; ++r) dyp[d][r] = 0.f;
    const int64_t crow0 = s0 + kg * 4;  // samples of this lane's accumulator rows
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int j = nt * 16 + row;  // output unit of this lane's accumulator column
        f32x4 acc = {0.f, 0.f, 0.f, 0.f}, tacc[D];
#pragma unroll
        for (int d = 0; d < D; ++d) tacc[d] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            // B operand: W2^T[k][j] = W2[j][k], 8 consecutive k of row j
            const bf16x8 bv = CVF ? w2p[CVF ? nt : 0][CVF ? kb : 0]
                                  : *reinterpret_cast<const bf16x8 *>(a.Pb + o.W2 + j * H + kb * 32 + kg * 8);  // 16 B aligned
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kb], bv, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[kb], bv, acc, 0, 0, 0);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                tacc[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tv[d][kb], bv, tacc[d], 0, 0, 0);
                tacc[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl[d][kb], bv, tacc[d], 0, 0, 0);
            }
        }
        const float b2 = CVF ? b2p[CVF ? nt : 0] : bf(a.Pb, o.b2 + j);
        const float w3 = CVF ? w3p[CVF ? nt : 0] : bf(a.Pb, o.w3 + j);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float a2 = tanh_fast(acc[r] + b2);
            const float g = 1.f - a2 * a2;
            yp[r] = fmaf(w3, a2, yp[r]);
            const int64_t sr = crow0 + r;
            if (t_a2 && sr < n) t_a2[sr * H + j] = a2;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                dyp[d][r] = fmaf(w3, g * tacc[d][r], dyp[d][r]);
                if (t_dz2 && sr < n) t_dz2[((int64_t)d * a.nmax + sr) * H + j] = tacc[d][r];
            }
        }
    }
    // reduce over the 16 output lanes of each row group (fixed butterfly)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        for (int m = 1; m < 16; m <<= 1) {
            yp[r] += __shfl_xor(yp[r], m, 64);
#pragma unroll
            for (int d = 0; d < D; ++d) dyp[d][r] += __shfl_xor(dyp[d][r], m, 64);
        }
    }
    // CVs of this lane's four output samples (rows kg*4 + r), for the
    // certification lookup and the outputs
    double xo[4][D];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int d = 0; d < D; ++d) xo[r][d] = __shfl(x[d], kg * 4 + r, 64);
    int fbo[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) fbo[r] = __shfl(fb_row, kg * 4 + r, 64);
    if (row == 0) {
        const float b3 = CVF ? b3p : bf(a.Pb, o.b3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t sr = crow0 + r;
            if (sr >= n) continue;
            const float y = yp[r] + b3;
            const double Vs = a.out_shift + a.out_scale * (double)y;
            double dvs[D], xs[D];
            bool finite = isfinite(Vs);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                dvs[d] = a.out_scale * (double)dyp[d][r];
                finite = finite && isfinite(dvs[d]);
            }
            if (V) V[sr] = Vs;
            if (t_y) t_y[sr] = y;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (dV) dV[sr * D + d] = dvs[d];
                if (t_dy) t_dy[sr * D + d] = dyp[d][r];
            }
            if (!flag) continue;
#pragma unroll
            for (int d = 0; d < D; ++d) xs[d] = xo[r][d];
            const uint8_t fb = (uint8_t)fbo[r];
            flag[sr] = fb;
            if (!step_on) continue;
            // a surrogate step: outputs (the fallback overwrites its walkers'
            // V and dV later) and the force of the walkers served here
            if (st.V_out) st.V_out[sr] = Vs;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (st.dV_out) st.dV_out[sr * D + d] = dvs[d];
                if (st.xi_out) st.xi_out[sr * D + d] = xs[d];
            }
            if (!fb && !finite && st.flags) atomicOr(st.flags, kFlagNonFinite);
            s_fb[kg * 4 + r] = fb;
#pragma unroll
            for (int d = 0; d < D; ++d) s_coef[kg * 4 + r][d] = -dvs[d];
        }
    }
    // force gather of the walkers served here: (sample, touched atom) pairs
    // over all 64 lanes.  A surrogate step launches one wavefront per
    // workgroup, so this barrier only orders the wavefront's own LDS traffic.
    if (!step_on || !st.do_forces) return;
    __syncthreads();
    const int U = st.tabs.U;
    for (int pi = lane; pi < kSamplesPerWave * U; pi += 64) {
        const int sl = pi / U, u = pi % U;
        const int64_t sr = s0 + sl;
        if (sr >= n || s_fb[sl]) continue;
        gather_atom(st.tabs, st.J + sr * st.nslots * 3, (int32_t)sr, s_coef[sl], st.F, u);
    }
}

// ------------------------------------------------------------------ reverse
// S samples per workgroup.  Sobolev loss
//   L = (1/B) sum_b [alpha (y_b - V_b)^2 + beta sum_d (dy_bd - G_bd)^2]
// Gradient of the forward above: activations rounded (bf16 hi + lo) where
// the forward rounds them, the rounding itself passed straight through,
// weights at their bf16 values, FP32 arithmetic.
// Every parameter-gradient entry has one owning lane (no atomics); the
// workgroup writes its partial gradient (and loss) to gpart[blockIdx][.].
// the value the forward feeds to the matrix cores: bf16 hi + bf16 lo
__device__ __forceinline__ float round_bf2(float x)
{
    const float h = (float)(__bf16)x;
    return h + (float)(__bf16)(x - h);
}

template <int H>
__host__ __device__ constexpr int bwd_samples()
{
    return H >= 128 ? 8 : 16;
}

// the bf16 pair (hi, lo) of eight consecutive FP32 values, the form in
// which an FP32 operand enters the bf16 matrix product
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const __bf16 h = (__bf16)v[t];
        hi[t] = h;
        lo[t] = (__bf16)(v[t] - (float)h);
    }
}

// The reverse pass: per workgroup S samples, their value row and D tangent
// rows stacked (row c S + sl: c = 0 the value, c = d + 1 tangent d; rows
// padded with zeros to a multiple of 32).  The two H x H products run on
// the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), every
// FP32 operand entering as a bf16 pair:
//   a1b rows  = z2b rows . W2        (M = rows, K = H, N = H; W2 exact bf16,
//                                     staged transposed in LDS)
//   dL/dW2    = z2b rows^T . act rows (M = H, K = rows, N = H; act = the
//                                     forward's bf16-pair activations a1r,
//                                     da1r_d; hi.hi + hi.lo + lo.hi)
// the rest (features, tanh derivatives, the small layers, the loss) on the
// vector units in FP32.  Every gradient entry has one owning lane (no
// atomics); the workgroup's partial gradient and loss go to gpart[blockIdx].
template <int H, int D>
__global__ void __launch_bounds__(kBlock) k_mlp_bwd(MlpArgs a, const double *xi, const double *Vl, const double *Gl,
                                                     int64_t n, float inv_b, float alpha, float beta,
                                                     const float *t_a2, const float *t_dz2, const float *t_y,
                                                     const float *t_dy, float *gpart)
{
    constexpr int F = 2 * D;
    constexpr int S = bwd_samples<H>();
    constexpr int R = (1 + D) * S;          // stacked rows
    constexpr int MP = (R + 31) / 32 * 32;  // rows padded to the product depth
    constexpr int HP = H + 4;               // LDS row stride (floats): strided column reads spread over banks
    constexpr int HT = H + 8;               // row stride of the transposed W2 (bf16)
    constexpr POff o = poff(H, F);
    __shared__ float s_f[S][F], s_u[S][D][F];
    __shared__ float s_yb[S], s_dyb[S][D];
    __shared__ float s_zx[MP][HP];  // z2b, dz2b_d
    __shared__ float s_ac[MP][HP];  // a1r, da1r_d (the forward's matrix-core inputs)
    __shared__ float s_x[MP][HP];   // a2, da2_d (phase 1); a1b, da1b_d (phase 2b); z1b, dz1b_d (phase 2c)
    __shared__ __bf16 s_w2t[H][HT];  // s_w2t[k][j] = W2[j][k]
    __shared__ float s_loss[kBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * S;
    float *gp = gpart + (int64_t)blockIdx.x * (o.P + 1);
    // phase 0: features and the loss adjoints of y and dy; W2 staged
    // transposed; padding rows zeroed
    float lossp = 0.f;
    if (tid < S) {
        const int64_t s = b0 + tid;
        const bool live = s < n;
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = live ? xi[s * D + d] : 0.0;
        float f[F], u[D][F];
        featurize<D>(a, x, f, u);
#pragma unroll
        for (int q = 0; q < F; ++q) {
            s_f[tid][q] = f[q];
#pragma unroll
            for (int d = 0; d < D; ++d) s_u[tid][d][q] = u[d][q];
        }
        // targets in network units: (V - out_shift) / out_scale, G / out_scale
        const double inv_sc = 1.0 / a.out_scale;
        const float r0 = live ? t_y[s] - (float)((Vl[s] - a.out_shift) * inv_sc) : 0.f;
        s_yb[tid] = 2.f * alpha * r0 * inv_b;
        lossp += alpha * r0 * r0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float r1 = live ? t_dy[s * D + d] - (float)(Gl[s * D + d] * inv_sc) : 0.f;
            s_dyb[tid][d] = 2.f * beta * r1 * inv_b;
            lossp += beta * r1 * r1;
        }
    }
    for (int e = tid; e < H * H; e += kBlock) {
        const int j = e / H, k = e % H;
        s_w2t[k][j] = reinterpret_cast<const __bf16 *>(a.Pb)[o.W2 + e];
    }
    for (int e = tid; e < (MP - R) * H; e += kBlock) {
        const int m = R + e / H, k = e % H;
        s_zx[m][k] = 0.f;
        s_ac[m][k] = 0.f;
    }
    __syncthreads();
    // phase 1 (sample sl, output unit j): y = w3.a2 + b3, dy_d = w3.da2_d,
    // da2_d = (1 - a2^2) dz2_d  ->  adjoints of z2 and of the tangents dz2_d
    for (int idx = tid; idx < S * H; idx += kBlock) {
        const int sl = idx / H, j = idx % H;
        const int64_t s = b0 + sl;
        const bool live = s < n;
        const float a2 = live ? t_a2[s * H + j] : 0.f;
        const float g2 = 1.f - a2 * a2;
        const float w3 = bf(a.Pb, o.w3 + j);
        float a2b = s_yb[sl] * w3;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float dz2 = live ? t_dz2[((int64_t)d * a.nmax + s) * H + j] : 0.f;
            const float da2b = s_dyb[sl][d] * w3;
            a2b += da2b * (-2.f * a2 * dz2);
            s_zx[(d + 1) * S + sl][j] = da2b * g2;
            s_x[(d + 1) * S + sl][j] = g2 * dz2;  // da2_d
        }
        s_zx[sl][j] = a2b * g2;
        s_x[sl][j] = a2;
    }
    __syncthreads();
    // phase 1b: b2, w3, b3 gradients (lane j owns unit j)
    for (int j = tid; j < H; j += kBlock) {
        float gb2 = 0.f, gw3 = 0.f;
        for (int sl = 0; sl < S; ++sl) {
            gb2 += s_zx[sl][j];
            gw3 += s_yb[sl] * s_x[sl][j];
#pragma unroll
            for (int d = 0; d < D; ++d) gw3 += s_dyb[sl][d] * s_x[(d + 1) * S + sl][j];
        }
        gp[o.b2 + j] = gb2;
        gp[o.w3 + j] = gw3;
    }
    if (tid == 0) {
        float gb3 = 0.f;
        for (int sl = 0; sl < S; ++sl) gb3 += s_yb[sl];
        gp[o.b3] = gb3;
    }
    // phase 2a (sample sl, input unit k): layer 1 recomputed, the forward's
    // matrix-core inputs a1r and da1r_d kept
    for (int idx = tid; idx < S * H; idx += kBlock) {
        const int sl = idx / H, k = idx % H;
        float z = bf(a.Pb, o.b1 + k), dz1[D];
#pragma unroll
        for (int d = 0; d < D; ++d) dz1[d] = 0.f;
#pragma unroll
        for (int q = 0; q < F; ++q) {
            const float w = bf(a.Pb, o.W1 + k * F + q);
            z = fmaf(w, s_f[sl][q], z);
#pragma unroll
            for (int d = 0; d < D; ++d) dz1[d] = fmaf(w, s_u[sl][d][q], dz1[d]);
        }
        const float a1 = tanh_fast(z), g1 = 1.f - a1 * a1;
        s_ac[sl][k] = round_bf2(a1);
#pragma unroll
        for (int d = 0; d < D; ++d) s_ac[(d + 1) * S + sl][k] = round_bf2(g1 * dz1[d]);
    }
    __syncthreads();  // phase 1b has read s_x; s_zx and s_w2t complete
    // phase 2b (matrix cores): s_x rows = s_zx rows . W2, 16 x 16 tiles dealt
    // to the four wavefronts
    {
        const int r16 = lane & 15, kg = lane >> 4;
        for (int t = wave; t < (MP / 16) * (H / 16); t += kBlock / 64) {
            const int mt = t / (H / 16), nt = t % (H / 16);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < H / 32; ++kb) {
                const int j0 = kb * 32 + kg * 8;
                float v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = s_zx[mt * 16 + r16][j0 + q];
                bf16x8 hi, lo;
                split8(v, hi, lo);
                const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(&s_w2t[nt * 16 + r16][j0]);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, bw, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, bw, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) s_x[mt * 16 + kg * 4 + i][nt * 16 + r16] = acc[i];
        }
    }
    __syncthreads();
    // phase 2c (sample sl, input unit k): through tanh of layer 1:
    // a1b = a1b' + sum_d da1b_d (-2 a1 dz1_d), z1b = a1b g1, dz1b_d = da1b_d g1
    for (int idx = tid; idx < S * H; idx += kBlock) {
        const int sl = idx / H, k = idx % H;
        float z = bf(a.Pb, o.b1 + k), dz1[D];
#pragma unroll
        for (int d = 0; d < D; ++d) dz1[d] = 0.f;
#pragma unroll
        for (int q = 0; q < F; ++q) {
            const float w = bf(a.Pb, o.W1 + k * F + q);
            z = fmaf(w, s_f[sl][q], z);
#pragma unroll
            for (int d = 0; d < D; ++d) dz1[d] = fmaf(w, s_u[sl][d][q], dz1[d]);
        }
        const float a1 = tanh_fast(z), g1 = 1.f - a1 * a1;
        float a1b = s_x[sl][k];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float da1b = s_x[(d + 1) * S + sl][k];
            a1b += da1b * (-2.f * a1 * dz1[d]);
            s_x[(d + 1) * S + sl][k] = da1b * g1;
        }
        s_x[sl][k] = a1b * g1;
    }
    // phase 3a (matrix cores): dL/dW2[j][k] = sum over rows m of
    // s_zx[m][j] s_ac[m][k]; 16 x 16 tiles of (j, k) dealt to the wavefronts
    {
        const int r16 = lane & 15, kg = lane >> 4;
        for (int t = wave; t < (H / 16) * (H / 16); t += kBlock / 64) {
            const int jt = t / (H / 16), kt = t % (H / 16);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < MP / 32; ++kb) {
                const int m0 = kb * 32 + kg * 8;
                float va[8], vb[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    va[q] = s_zx[m0 + q][jt * 16 + r16];
                    vb[q] = s_ac[m0 + q][kt * 16 + r16];
                }
                bf16x8 ah, al, bh, bl;
                split8(va, ah, al);
                split8(vb, bh, bl);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) gp[o.W2 + (jt * 16 + kg * 4 + i) * H + kt * 16 + r16] = acc[i];
        }
    }
    __syncthreads();  // phase 2c's z1b, dz1b complete
    // phase 3b: W1 and b1 gradients (lane-owned)
    for (int e = tid; e < H * (F + 1); e += kBlock) {
        const int k = e / (F + 1), q = e % (F + 1);
        float g = 0.f;
        for (int sl = 0; sl < S; ++sl) {
            if (q == F) {
                g += s_x[sl][k];
            } else {
                g = fmaf(s_x[sl][k], s_f[sl][q], g);
#pragma unroll
                for (int d = 0; d < D; ++d) g = fmaf(s_x[(d + 1) * S + sl][k], s_u[sl][d][q], g);
            }
        }
        if (q == F)
            gp[o.b1 + k] = g;
        else
            gp[o.W1 + k * F + q] = g;
    }
    // loss partial (fixed reduction order)
    for (int m = 32; m > 0; m >>= 1) lossp += __shfl_xor(lossp, m, 64);
    if ((tid & 63) == 0) s_loss[tid >> 6] = lossp;
    __syncthreads();
    if (tid == 0) {
        float l = 0.f;
        for (int w = 0; w < kBlock / 64; ++w) l += s_loss[w];
        gp[o.P] = l;
    }
}

// stage 1 of the gradient sum: lane p of slice y sums the workgroup
// partials [y * per, (y + 1) * per) of parameter p (index P: the loss) in
// order, in FP64
__global__ void __launch_bounds__(kBlock) k_mlp_reduce(const float *gpart, int32_t nblk, int32_t P, int32_t per,
                                                        double *red)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const int b0 = blockIdx.y * per, b1 = min(nblk, b0 + per);
    double g = 0.0;
    for (int b = b0; b < b1; ++b) g += (double)gpart[(int64_t)b * (P + 1) + p];
    red[(int64_t)blockIdx.y * (P + 1) + p] = g;
}

// stage 2, one lane per parameter: the slices in order, Adam on the FP32
// master value, refresh of its bf16 copy; lane P writes the loss sum.
__global__ void __launch_bounds__(kBlock) k_mlp_adam(MlpArgs a, const double *red, int32_t ns, int32_t P, int64_t t,
                                                      float lr, double *loss_out, int32_t update, double *gsum)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    double g = 0.0;
    for (int y = 0; y < ns; ++y) g += red[(int64_t)y * (P + 1) + p];
    if (gsum) gsum[p] = g;
    if (p == P) {
        if (loss_out) *loss_out = g;  // sum of per-sample losses
        return;
    }
    if (!update) return;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double m = b1 * a.m[p] + (1.0 - b1) * g;
    const double v = b2 * a.v[p] + (1.0 - b2) * g * g;
    a.m[p] = (float)m;
    a.v[p] = (float)v;
    const double mh = m / (1.0 - pow(b1, (double)t)), vh = v / (1.0 - pow(b2, (double)t));
    const float w = (float)((double)a.P32[p] - (double)lr * mh / (sqrt(vh) + eps));
    a.P32[p] = w;
    reinterpret_cast<__bf16 *>(a.Pw)[p] = (__bf16)w;
}

// bf16 copies of the FP32 master weights
__global__ void k_mlp_round(MlpArgs a, int32_t P)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) reinterpret_cast<__bf16 *>(a.Pw)[p] = (__bf16)a.P32[p];
}

template <int H, int D>
hipError_t mlp_fwd_hd(const MlpArgs &a, const double *xi, int64_t n, double *V, double *dV, float *t_a2, float *t_dz2,
                      float *t_y, float *t_dy, uint8_t *flag, hipStream_t s, const MlpStep *step)
{
    // one wavefront per 16 samples; single-wavefront workgroups spread a
    // small batch over as many CUs as it has wavefronts
    const int64_t waves = (n + kSamplesPerWave - 1) / kSamplesPerWave;
    const int per = (waves >= 4096 && !step) ? kBlock / 64 : 1;  // a step: one wavefront per workgroup
    const unsigned blocks = (unsigned)((waves + per - 1) / per);
    if (blocks == 0) return hipSuccess;
    MlpStep st{};
    if (step) st = *step;
    if (step && step->fuse_cv)
        hipLaunchKernelGGL((k_mlp_fwd<H, D, true>), dim3(blocks), dim3(64 * per), 0, s, a, xi, n, V, dV, t_a2, t_dz2,
                           t_y, t_dy, flag, st, 1);
    else
        hipLaunchKernelGGL((k_mlp_fwd<H, D, false>), dim3(blocks), dim3(64 * per), 0, s, a, xi, n, V, dV, t_a2, t_dz2,
                           t_y, t_dy, flag, st, step ? 1 : 0);
    return hipGetLastError();
}

template <int H, int D>
hipError_t mlp_bwd_hd(const MlpArgs &a, const double *xi, const double *Vl, const double *Gl, int64_t n, float inv_b,
                      float alpha, float beta, const float *t_a2, const float *t_dz2, const float *t_y,
                      const float *t_dy, float *gpart, int32_t &nblk, hipStream_t s)
{
    constexpr int S = bwd_samples<H>();
    nblk = (int32_t)((n + S - 1) / S);
    hipLaunchKernelGGL((k_mlp_bwd<H, D>), dim3(nblk), dim3(kBlock), 0, s, a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2,
                       t_dz2, t_y, t_dy, gpart);
    return hipGetLastError();
}

}  // namespace

int32_t mlp_param_count(int32_t H, int32_t D) { return poff(H, 2 * D).P; }
int32_t mlp_bwd_blocks(int32_t H, int64_t n) { return (int32_t)((n + (H >= 128 ? 8 : 16) - 1) / (H >= 128 ? 8 : 16)); }

#define SX_MLP_DISPATCH(FN, ...)                                                   \
    switch (a.H * 10 + a.D) {                                                      \
    case 641: return FN<64, 1>(__VA_ARGS__);                                       \
    case 642: return FN<64, 2>(__VA_ARGS__);                                       \
    case 643: return FN<64, 3>(__VA_ARGS__);                                       \
    case 1281: return FN<128, 1>(__VA_ARGS__);                                     \
    case 1282: return FN<128, 2>(__VA_ARGS__);                                     \
    case 1283: return FN<128, 3>(__VA_ARGS__);                                     \
    default: return hipErrorInvalidValue;                                          \
    }

hipError_t launch_mlp_fwd(const MlpArgs &a, const double *xi, int64_t n, double *V, double *dV, float *t_a2,
                          float *t_dz2, float *t_y, float *t_dy, uint8_t *flag, hipStream_t s, const MlpStep *step)
{
    SX_MLP_DISPATCH(mlp_fwd_hd, a, xi, n, V, dV, t_a2, t_dz2, t_y, t_dy, flag, s, step)
}

static hipError_t reduce_and_adam(const MlpArgs &a, const float *gpart, int32_t nblk, double *red, float lr, int64_t t,
                                  double *loss_out, int32_t update, double *gsum, hipStream_t s)
{
    const int P = mlp_param_count(a.H, a.D);
    const int ns = nblk < kMlpRedSlices ? nblk : kMlpRedSlices;
    const int per = (nblk + ns - 1) / ns;
    const unsigned gx = (unsigned)((P + 1 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(gx, ns), dim3(kBlock), 0, s, gpart, nblk, P, per, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_adam, dim3(gx), dim3(kBlock), 0, s, a, (const double *)red, ns, P, t, lr, loss_out, update,
                       gsum);
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(const MlpArgs &a, const double *xi, const double *Vl, const double *Gl, int64_t n,
                                 float alpha, float beta, float lr, int64_t t, float *t_a2, float *t_dz2, float *t_y,
                                 float *t_dy, float *gpart, double *red, double *loss_out, hipStream_t s)
{
    hipError_t e = launch_mlp_fwd(a, xi, n, nullptr, nullptr, t_a2, t_dz2, t_y, t_dy, nullptr, s);
    if (e != hipSuccess) return e;
    int32_t nblk = 0;
    const float inv_b = 1.f / (float)n;
    switch (a.H * 10 + a.D) {
    case 641: e = mlp_bwd_hd<64, 1>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    case 642: e = mlp_bwd_hd<64, 2>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    case 643: e = mlp_bwd_hd<64, 3>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    case 1281: e = mlp_bwd_hd<128, 1>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    case 1282: e = mlp_bwd_hd<128, 2>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    case 1283: e = mlp_bwd_hd<128, 3>(a, xi, Vl, Gl, n, inv_b, alpha, beta, t_a2, t_dz2, t_y, t_dy, gpart, nblk, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (lr > 0.f) return reduce_and_adam(a, gpart, nblk, red, lr, t, loss_out, 1, nullptr, s);
    return hipSuccess;  // gradient only: launch_mlp_grad_sum reads gpart
}

hipError_t launch_mlp_grad_sum(const MlpArgs &a, const float *gpart, int64_t n, double *red, double *gsum,
                               hipStream_t s)
{
    return reduce_and_adam(a, gpart, mlp_bwd_blocks(a.H, n), red, 0.f, 1, nullptr, 0, gsum, s);
}

// ------------------------------------------------------- certification mask
template <int D>
__global__ void __launch_bounds__(kBlock) k_cert_mask(MlpArgs a, const double *dVhat, const double *dV, double h0,
                                                       double h1, double h2, double tol, uint8_t *mask)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = a.cert_n;
    int64_t ncell = 1, ci[D], npts[D];
#pragma unroll
    for (int d = 0; d < D; ++d) ncell *= n;
    if (cell >= ncell) return;
    int64_t r = cell;
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {  // row-major, last CV fastest
        ci[d] = r % n;
        r /= n;
        npts[d] = a.periodic[d] ? n : n + 1;
    }
    const double h[3] = {h0, h1, h2};
    double e[1 << D][D];
    double emax = 0.0;
#pragma unroll
    for (int c = 0; c < (1 << D); ++c) {
        int64_t pt = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int64_t i = ci[d] + ((c >> (D - 1 - d)) & 1);
            if (i >= npts[d]) i -= npts[d];  // periodic wrap (i == n)
            pt = pt * npts[d] + i;
        }
        double s2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            e[c][d] = dVhat[pt * D + d] - dV[pt * D + d];
            s2 += e[c][d] * e[c][d];
        }
        emax = fmax(emax, sqrt(s2));
    }
    // largest change of the error vector per unit length along cell edges
    double L = 0.0;
#pragma unroll
    for (int c = 0; c < (1 << D); ++c)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int bit = 1 << (D - 1 - d);
            if (c & bit) continue;
            double s2 = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const double df = e[c | bit][q] - e[c][q];
                s2 += df * df;
            }
            L = fmax(L, sqrt(s2) / h[d]);
        }
    double diag2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) diag2 += h[d] * h[d];
    const double bound = emax + 2.0 * L * 0.5 * sqrt(diag2);
    mask[cell] = (isfinite(bound) && bound <= tol) ? 1 : 0;
}

hipError_t launch_cert_mask(const MlpArgs &a, const double *dVhat, const double *dV, const double *h, double tol,
                            uint8_t *mask, hipStream_t s)
{
    int64_t ncell = 1;
    for (int d = 0; d < a.D; ++d) ncell *= a.cert_n;
    const unsigned blocks = (unsigned)((ncell + kBlock - 1) / kBlock);
    const double h1 = a.D > 1 ? h[1] : 1.0, h2 = a.D > 2 ? h[2] : 1.0;
    switch (a.D) {
    case 1: hipLaunchKernelGGL(k_cert_mask<1>, dim3(blocks), dim3(kBlock), 0, s, a, dVhat, dV, h[0], h1, h2, tol, mask); break;
    case 2: hipLaunchKernelGGL(k_cert_mask<2>, dim3(blocks), dim3(kBlock), 0, s, a, dVhat, dV, h[0], h1, h2, tol, mask); break;
    case 3: hipLaunchKernelGGL(k_cert_mask<3>, dim3(blocks), dim3(kBlock), 0, s, a, dVhat, dV, h[0], h1, h2, tol, mask); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


hipError_t launch_mlp_round(const MlpArgs &a, hipStream_t s)
{
    const int P = mlp_param_count(a.H, a.D);
    hipLaunchKernelGGL(k_mlp_round, dim3((P + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a, P);
    return hipGetLastError();
}

}  // namespace sx
