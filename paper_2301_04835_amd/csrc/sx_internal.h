// Internal definitions shared by the host side of libsampx and its HIP
// kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sx {

constexpr int kMaxCv = 8;        // CVs per context
constexpr int kMaxBiasDim = 3;   // CVs a bias (hills / ABF grid) may span
constexpr int kBlock = 256;      // threads per workgroup of the main kernels
constexpr int kHillsPerLoad = 4; // float4 per lane
constexpr int kTileUnit = kBlock * kHillsPerLoad;  // 1024 hills: smallest tile
constexpr int kMaxTileUnits = 8;                   // largest tile: 8192 hills

// CV_COORD_CELL: a coordination number with a hard cut evaluated through
// cell lists (no Jacobian slots; its forces come from the VJP kernel).
enum CvKind : int32_t { CV_DIHEDRAL = 0, CV_GYRATION = 1, CV_COORD = 2, CV_COORD_CELL = 3 };

// Device-side flags (bit = sx_status value).
constexpr uint32_t kFlagCapacity = 1u << 3;
constexpr uint32_t kFlagNonFinite = 1u << 4;

// Strided view of a position-like array: element (i, k) of atom i,
// component k sits at ptr[i * sa + k * sk].
struct PosView {
    const void *ptr;
    int32_t f64;  // 1: double, 0: float
    int64_t sa, sk;
};
struct ForceView {
    float *ptr;
    int64_t sa, sk;
};

// One CV as the kernels see it.  Member atoms (walker-relative) live in the
// slot table: slot_atom[slot0 .. slot0 + nslot).
struct CvDesc {
    int32_t kind;
    int32_t d;      // index in xi
    int32_t slot0;  // first Jacobian slot
    int32_t na, nb; // coordination: group sizes (A slots first, then B); others: na = members
    int32_t n, m;   // switching exponents
    float r0, inv_r0;
    float rcut2;    // <= 0: no cut
    float scale;    // 1 or 1/na
    int32_t lanes;  // coordination all-pairs: lanes per member (a power of two <= 64)
    int32_t vblk0;  // coordination all-pairs: first value record of this CV (per walker)
    int32_t atom[4];  // dihedral: its four atoms (walker-relative)
    int32_t ga, gb;   // cell-list coordination: the two atom groups
    int32_t cn;       // cell-list coordination: index among those CVs
    double rcut;      // the cut (FP64), for decisions at its edge
    double inv_r0d;   // 1 / r0 in FP64 (the FP64 pair terms of ABF's Jacobian)
};

struct CvSet {
    int32_t ncv, D;
    CvDesc cv[kMaxCv];
    double box[3], inv_box[3];  // 0: open
    int32_t nslots;
    int64_t vblk_per_walker;   // coordination value records per walker (one per A-side member block)
};

// Common walker tables.
struct WalkerTabs {
    int32_t W;
    const int64_t *atom_off;   // W + 1
    const int32_t *slot_atom;  // nslots
    const int32_t *slot_cv;    // nslots
    const int32_t *touched;    // U walker-relative atoms touched by any CV
    const int32_t *inv_ptr;    // U + 1
    const int32_t *inv_slot;   // nslots: slots of touched atom u
    int32_t U;
};

// Packed per-tile record, one 32-byte load: walker, first hill of the tile,
// last float4 start inside the walker's capacity, hill base / 4, the
// walker's first atom.
struct __align__(16) TileRec {
    int32_t w, h0, klast, hb4;
    int32_t aoff_lo, aoff_hi;  // first atom of the walker (64-bit, split)
    int32_t pad[2];
};
// Packed per-walker record for the finalize kernel.
struct __align__(16) WalkerRec {
    int32_t t0, nt, cap, hb4;
    int64_t aoff;
    int32_t pad[2];
};

// The walker-relative force-gather table when it is small enough to travel
// in the kernel arguments: touched atom u, its slots ent[u][0..nent[u]).
constexpr int kSmallU = 32, kSmallPer = 8;
struct SmallTabs {
    int32_t on, U;
    int32_t touched[kSmallU];
    int32_t nent[kSmallU];
    int32_t ent[kSmallU][kSmallPer];  // slot | cv << 20
};

// Hill-sum launch (private hill lists).
struct HillArgs {
    // hill storage (SoA): centres c[d][...] and heights h[...]
    float *c[kMaxBiasDim];
    float *h;
    int32_t *count;            // per walker
    const TileRec *tiles;
    const WalkerRec *wrec;
    int32_t ntiles, tile_units;
    double *partial;           // ntiles x 4
    // constants
    int32_t D;
    double period[kMaxBiasDim], inv_period[kMaxBiasDim];  // 0: not periodic
    float a2[kMaxBiasDim];     // log2(e) / (2 sigma^2)
    double inv_sig2[kMaxBiasDim];
    // inputs / outputs
    const double *xi;          // W x D
    double *V_ws, *dV_ws;      // W, W x D
    double *xi_out, *V_out, *dV_out;  // may be null
    double *xi_save;           // fused CVs: where kernel B keeps xi (workspace)
    int32_t count_step;        // kernel A sets the device step counter
    int32_t fuse;              // every CV is a dihedral: xi and J computed in the hill kernels
    // deposition
    int32_t deposit;           // 0: never, 1: by stride, 2: always
    int64_t step;              // < 0: device counter
    int32_t stride;
    double height, inv_kdT;    // inv_kdT == 0: constant height
    int64_t *dstep;            // next step number
    uint32_t *flags;
    // forces
    int32_t do_forces;
    float *J;                  // W x nslots x 3 (fused dihedrals: written by kernel A)
    int32_t nslots;
    WalkerTabs tabs;
    SmallTabs small;
    ForceView F;
};

// What an ABF update reads before the step's sums are known (per walker):
// xi, its bin k (inr: inside the grid), the bin's count and force sums, the
// FUNN bias, the momentum estimator's previous bias and W p and whether there
// was a previous step, and the device step counter (when the step is not
// given).
struct AbfPre {
    double xi[kMaxBiasDim], F[kMaxBiasDim], bext[kMaxBiasDim], bprev[kMaxBiasDim], wpprev[kMaxBiasDim];
    int64_t k, dstep;
    uint32_t cnt;
    int32_t has;
    bool inr;
};

struct AbfArgs {
    int32_t D;
    const double *xi;     // W x D
    const double *J;      // W x nslots x 3 (FP64 rows: the Gram matrix and J.F see them as computed)
    int32_t nslots;
    WalkerTabs tabs;
    PosView Fsys;         // system forces (float)
    ForceView F;          // biased forces (+=)
    uint32_t *N;          // W x nbins
    double *Fsum;         // W x nbins x D
    int64_t nbins_total;
    double lo[kMaxBiasDim], delta[kMaxBiasDim];
    int32_t nbins[kMaxBiasDim], periodic[kMaxBiasDim];
    int32_t n_threshold;
    double *xi_out, *V_out, *dV_out;
    uint32_t *flags;
    int64_t step;
    int64_t *dstep;
    // estimator 0: theta from the projected system force (unit masses; Fsys
    // holds the system forces); 1: from the time derivative of the CV-space
    // momentum (Fsys holds the momenta; inverse masses per atom, step dt, and
    // per walker the previous step's W p, bias and whether there was one)
    int32_t estimator;
    double dt;
    const double *inv_mass;   // total atoms
    double *Wp_prev, *b_prev; // W x D
    int32_t *has_prev;        // W
    // FUNN: the bias is this W x D gradient of a network fitted to the mean
    // forces (null: the grid's Fsum / max(N, N_thr))
    const double *b_ext;
    // nblk > 0: the two-launch form for walkers with many touched atoms,
    // with W x nblk records of (D_max^2 + D_max) doubles in part and one
    // AbfPre per walker in pre (workspace)
    int32_t nblk;
    double *part;
    AbfPre *pre;
    // two-launch form without FUNN: the all-pairs coordination numbers'
    // values are summed here from their block records (cn_vpart, as the CV
    // kernel left them) by the first wavefront of the first workgroup, in
    // the order of the value kernel it replaces, and written to xi_ws before
    // the bin is taken: cn_d the CV index, cn_vblk0 its first record,
    // cn_nblk its records, cn_scale its scale
    int32_t ncn_fold;
    int32_t cn_d[kMaxBiasDim], cn_vblk0[kMaxBiasDim], cn_nblk[kMaxBiasDim];
    double cn_scale[kMaxBiasDim];
    const double *cn_vpart;
    int64_t vblk_per_walker;
    double *xi_ws;
};
constexpr int kAbfSplitU = 2 * kBlock;  // touched atoms above which ABF takes the two-launch form

// Hill sum over one shared list at nq query points.
// Metadynamics bias kept on a grid: V and dV/dxi of each hill list at the
// nodes (row-major, first CV slowest; a periodic CV has n bins = n nodes and
// wraps, a non-periodic one n + 1 nodes up to hi), read back by multilinear
// interpolation.  One grid per hill list.
struct GridArgs {
    int32_t D, L, shared;                 // CVs, hill lists (grids), one list for all walkers
    int32_t nbins[kMaxBiasDim], n[kMaxBiasDim], per[kMaxBiasDim];  // bins, nodes, periodic
    double lo[kMaxBiasDim], delta[kMaxBiasDim];
    double period[kMaxBiasDim], inv_sig2[kMaxBiasDim];
    int64_t N;                            // nodes per grid
    double *V, *G;                        // L x N, L x D x N
    int32_t *pend;                        // L: hills appended by the step, not yet on the grid
    // hill lists: list l starts at wrec[l].hb4 * 4, holds wrec[l].cap
    float *c[kMaxBiasDim];
    float *h;
    int32_t *count;
    const WalkerRec *wrec;
    // step
    const double *xi;                     // W x D
    double *V_ws, *dV_ws, *xi_out, *V_out, *dV_out;  // outputs may be null
    int32_t deposit, count_step, stride;
    int32_t count_in_step;  // set by the launcher: the step kernel advances the counter (no add kernel follows)
    int64_t step;
    double height, inv_kdT;
    int64_t *dstep;
    uint32_t *flags;
    int32_t do_forces, nslots;
    const float *J;
    WalkerTabs tabs;
    ForceView F;
    SmallTabs small;  // the gather table in kernel-argument form (on = 0: the walker tables)
    // fuse_cv: every CV a dihedral, evaluated by the one-wavefront step
    // itself from the positions (values into xi_ws, gradients into J_ws)
    int32_t fuse_cv;
    CvSet cs;
    PosView pos;
    double *xi_ws;
    float *J_ws;
};

// Harmonic bias k/2 (xi - xi0_w)^2 per walker (umbrella windows) and the
// windows' running sums for umbrella integration.
struct HarmonicArgs {
    int32_t D, accumulate;
    double period[kMaxBiasDim];           // 0: not periodic
    double k[kMaxBiasDim];
    const double *xi0;                    // W x D window centres
    const double *xi;                     // W x D
    double *V_ws, *dV_ws, *xi_out, *V_out, *dV_out;  // outputs may be null
    int64_t *n;                           // W samples
    double *s1, *s2;                      // W x D sums of D, W x D x D sums of D D^T
    int64_t *dstep;
    int32_t count_step;
    int64_t step;
    uint32_t *flags;
    int32_t do_forces, nslots;
    const float *J;
    WalkerTabs tabs;
    ForceView F;
    // fuse_cv: every CV a dihedral, evaluated by the kernel itself from the
    // positions (values into xi_ws, gradients into J_ws, which J then reads)
    int32_t fuse_cv;
    CvSet cs;
    PosView pos;
    double *xi_ws;
    float *J_ws;
};

struct SharedArgs {
    int32_t D;
    float *c[kMaxBiasDim];
    float *h;
    int32_t *count;
    int64_t cap;
    double period[kMaxBiasDim], inv_period[kMaxBiasDim];
    float a2[kMaxBiasDim];
    double inv_sig2[kMaxBiasDim];
    const double *xi;  // nq x D
    int64_t nq;        // queries (walkers, or evaluation points)
    // fallback mode (fb != null): nq = W and only walkers w with fb[w] = 1
    // are summed; walker w's records sit at query index w
    const uint8_t *fb;
    double *partial;   // nchunk x nq x 4
    int32_t chunk, nchunk;
    double *V_ws, *dV_ws, *xi_out, *V_out, *dV_out;  // may be null
    int32_t deposit, count_step, stride;
    int64_t step;
    double height, inv_kdT;
    int64_t *dstep;
    uint32_t *flags;
    // forces of the queried walkers (the finalize gathers them): do_forces
    int32_t do_forces, nslots;
    const float *J;
    WalkerTabs tabs;
    ForceView F;
    SmallTabs small;  // the gather table in kernel-argument form (on = 0: the walker tables)
};

// What a surrogate step adds to the network's forward pass: per-walker
// outputs, finiteness flag, and the force gather of the walkers the network
// serves (the others are overwritten and gathered by the exact fallback).
struct MlpStep {
    double *xi_out, *V_out, *dV_out;  // may be null
    uint32_t *flags;
    int32_t do_forces, nslots;
    float *J;
    WalkerTabs tabs;
    ForceView F;
    // every CV a dihedral: the kernel evaluates them from the positions
    // (values into xi_ws, gradients into J) instead of reading xi
    int32_t fuse_cv;
    CvSet cs;
    PosView pos;
    double *xi_ws;
};

// Cell lists of coordination-number groups (orthorhombic periodic box):
// cut-length cells (edge >= the cutoff, 3 to 16 per dimension), each cut into
// rxy sub-cells in x and y and rz = 4, 2 or 1 in z (the largest that keep
// the total within kCellTotal, rz reduced first), so partners within the cut
// lie within rxy sub-cells in x and y and rz in z.  rxy = 1: with rxy = 2 a
// home atom visits 1.44x fewer candidates, but each column block stages
// 25/9 as many partners per home atom over 25/9 as many sub-cells, and the
// pair pass of the 512-walker workload took 21.2 ms (column blocks of 40
// sub-cells) or 25.1 ms (20) instead of 13.0.
constexpr int kCellMax = 16;   // cut-length cells per dimension
constexpr int kCellTotal = 16384;
constexpr int kXYReach = 1;    // largest rxy
constexpr int kZReach = 4;     // largest rz
constexpr int kCzMax = 24;     // home sub-cells (in z) of one column block
constexpr int kMaxGroups = 8;  // distinct groups of the cell-list CVs
constexpr int kMaxInv = 8;     // (CV, side) uses of one group
struct CellArgs {
    int32_t W, G, ncn;                 // walkers, distinct groups, cell-list CVs
    int32_t nc[3], ncell;              // cells per dimension, total
    int32_t rxy, rz;                   // reach in x and y, and in z, in sub-cells
    double L[3], inv_L[3], clen[3];    // box edges, cell edges
    const int64_t *atom_off;           // W + 1
    const int32_t *gatoms;             // walker-relative atoms of all groups, group after group
    int32_t goff[kMaxGroups + 1];      // group g: gatoms[goff[g] .. goff[g + 1])
    int64_t gtotal;                    // goff[G]
    int32_t *cid;                      // W x gtotal: cell of each group member, then its sorted position
    int32_t *cstart;                   // W x G x (ncell + 1): members of cell c
    float4 *sorted;                    // W x gtotal: (x, y, z) relative to the cell origin, atom
    double *part;                      // W x ncn x nblk: coordination partial sums per column block
    float4 *jac;                       // W x jtotal: per (group, use) gradient of each member, sorted order
    int64_t jtotal;                    // sum over groups of members x uses
    int64_t joff[kMaxGroups][kMaxInv]; // first entry of (group, use) within a walker's jac
    int32_t nzb, nblk;                 // column blocks: nzb per column (even split), nblk in all
    // uses of each group: the CV (index into CvSet::cv) and its partner group
    int32_t ninv[kMaxGroups];
    int32_t inv_cv[kMaxGroups][kMaxInv], inv_p[kMaxGroups][kMaxInv];  // CV index in the set, partner group
    int32_t inv_side[kMaxGroups][kMaxInv];                              // 0: the group is the CV's A side
};

// Surrogate network (bf16 copies as raw 16-bit words in host code).
struct MlpArgs {
    int32_t D, H;
    int32_t periodic[kMaxBiasDim];
    double mu[kMaxBiasDim], inv_s[kMaxBiasDim];  // standardisation of non-periodic CVs
    const uint16_t *Pb;  // bf16 parameters (read)
    uint16_t *Pw;        // the same, written by the optimiser
    float *P32, *m, *v;  // FP32 master parameters, Adam moments
    int64_t nmax;        // row stride of the training tangents
    double out_scale, out_shift;  // V = out_shift + out_scale * y (FP32 network output y)
    double cert_lo[kMaxBiasDim], cert_inv_h[kMaxBiasDim];
    int32_t cert_n;
    const uint8_t *mask;  // certified cells (1) of the cert_n^D grid
};

// ---------------------------------------------------------------- launchers
// Each returns the hipError_t of its launch.
// Jacobian rows into J (float) or, when J64 is given, into J64 (double; the
// ABF path); J may be null when only the values are wanted
// cn_values false: the all-pairs coordination numbers stop at their block
// records in cn_part (a later kernel sums them)
hipError_t launch_cv(const CvSet &cs, const WalkerTabs &t, PosView pos, double *xi, float *J, double *J64,
                     double *cn_part, hipStream_t s, bool cn_values = true);
// which: 1 = tiles (kernel A), 2 = finalize (kernel B), 3 = both
hipError_t launch_hill_private(const HillArgs &a, const CvSet &cs, const PosView &pos, int32_t grid, hipStream_t s,
                               int which = 3);
hipError_t launch_abf(const AbfArgs &a, hipStream_t s);
// grid bias: a step (read-back, outputs, deposit, forces, then the step's
// hills onto the grids); rebuilding grids l0 .. l0 + nl - 1 from their whole
// lists; read-back at n points of grid l
hipError_t launch_harmonic(const HarmonicArgs &a, hipStream_t s);
hipError_t launch_grid_step(const GridArgs &g, hipStream_t s);
// x[i] *= a for i < n (device FP64)
hipError_t launch_scale_f64(double *x, int64_t n, double a, hipStream_t s);
hipError_t launch_grid_rebuild(const GridArgs &g, int32_t l0, int32_t nl, hipStream_t s);
hipError_t launch_grid_eval(const GridArgs &g, int32_t l, const double *xi, int64_t n, double *V, double *dV,
                            hipStream_t s);
// chunking of a shared-list sum over nq queries: chunk (hills) and count
// chunking of a shared-list sum: about `target` workgroups, chunks of whole
// 256-hill stages (nchunk <= ceil(cap / 256))
constexpr int32_t kSharedTarget = 2048;
void shared_split(int64_t cap, int64_t nq, int32_t &chunk, int32_t &nchunk, int32_t target = kSharedTarget);
hipError_t launch_hill_shared(const SharedArgs &a, hipStream_t s);
// cell lists (which & 1), then every cell-list coordination number's value
// into xi and the gradients of its members (which & 2)
hipError_t launch_cell_cv(const CellArgs &c, const CvSet &cs, const PosView &pos, double *xi, hipStream_t s,
                          int which = 3);
// out += sign * sum_d coef[w][d] dxi_d/dr for the cell-list coordination
// numbers (pair recompute, one writer per atom); needs the cell lists of the
// same positions (launch_cell_cv first)
hipError_t launch_cell_vjp(const CellArgs &c, const CvSet &cs, const PosView &pos, const double *coef, double sign,
                           ForceView out, hipStream_t s);
int32_t mlp_param_count(int32_t H, int32_t D);
int32_t mlp_bwd_blocks(int32_t H, int64_t n);
hipError_t launch_mlp_fwd(const MlpArgs &a, const double *xi, int64_t n, double *V, double *dV, float *t_a2,
                          float *t_dz2, float *t_y, float *t_dy, uint8_t *flag, hipStream_t s,
                          const MlpStep *step = nullptr);
// one optimisation step over n samples: forward, reverse, Adam (lr > 0) or
// only the loss (lr <= 0, gradients left in gpart)
hipError_t launch_mlp_train_step(const MlpArgs &a, const double *xi, const double *Vl, const double *Gl, int64_t n,
                                 float alpha, float beta, float lr, int64_t t, float *t_a2, float *t_dz2, float *t_y,
                                 float *t_dy, float *gpart, double *red, double *loss_out, hipStream_t s);
hipError_t launch_mlp_round(const MlpArgs &a, hipStream_t s);
// ordered FP64 sum of the per-workgroup gradients of the last reverse pass
// over n samples into gsum[0..P) and the loss sum into gsum[P]; red:
// kMlpRedSlices x (P + 1) doubles of scratch
constexpr int kMlpRedSlices = 16;
hipError_t launch_mlp_grad_sum(const MlpArgs &a, const float *gpart, int64_t n, double *red, double *gsum,
                               hipStream_t s);
// certification: one lane per cell of the cert_n^D grid; dVhat and dV
// [M][D] hold the network's and the exact gradient at the M grid corners
// (row-major, the first CV slowest; periodic CVs: cert_n corners per CV,
// others cert_n + 1); a cell is certified when the largest corner error
// plus twice its corner-estimated Lipschitz growth over the half diagonal
// stays within tol
hipError_t launch_cert_mask(const MlpArgs &a, const double *dVhat, const double *dV, const double *h, double tol,
                            uint8_t *mask, hipStream_t s);
hipError_t launch_gather(const WalkerTabs &t, const float *J, int32_t nslots, int32_t D, const double *coef,
                         double coef_sign, ForceView out, hipStream_t s);
hipError_t launch_copy_xi(const double *src, double *dst, int64_t n, hipStream_t s);
hipError_t launch_zero_bytes(void *p, int64_t nbytes, hipStream_t s);

// The fixed device scratch of the no-allocation entry point: its size, the
// once-per-device look-up of its address (with that device made current for
// the call), and that address (null before the look-up).
size_t noalloc_scratch_bytes();
hipError_t noalloc_setup(int device);
double *noalloc_scratch(int device);

}  // namespace sx
