/*
 * sampx — biasing-force path of CV-based enhanced sampling on one MI355X.
 *
 * C ABI of libsampx.so.  The operations follow Sec. 2 of
 * "PySAGES: flexible, advanced sampling methods accelerated with GPUs"
 * (arXiv 2301.04835):
 *   - a sampling method is split into an initialize step that allocates its
 *     state and an update step that reads the simulation and updates that
 *     state (Sec. 2.1, SamplingMethod.build -> initialize / update);
 *   - the simulation's particle buffers are read in place, without copies
 *     (Sec. 2, Snapshot and DLPack);
 *   - the biasing forces are ADDED to the engine's net forces (Sec. 2, the
 *     force-like callback inserted into the integrator);
 *   - methods: metadynamics and well-tempered metadynamics (Sec. 2.1.5), the
 *     adaptive biasing force (Sec. 2.1.4), multiple walkers / replicas
 *     (Sec. 2, parallel runs; Sec. 3.2 performance);
 *   - collective variables: DihedralAngle, RadiusofGyration (Sec. 2.2) and a
 *     rational-switching coordination number.
 *
 * Conventions shared by every call
 *   Units: nm, rad, kJ/mol, K.
 *   Pointers named dev_* or documented "device" are HIP device pointers; all
 *   other pointers are host pointers.  Device pointers are borrowed: the
 *   library never frees them and never keeps them past the call, except the
 *   state and workspace buffers handed to sx_bind, which the caller must keep
 *   alive (and unmoved) until sx_destroy or the next sx_bind.
 *   Device work is enqueued on the context's stream and is stream-ordered;
 *   no hot-path call (sx_step, sx_eval_cv, sx_cv_vjp, sx_hillsum,
 *   sx_graph_launch) synchronises the host or allocates device memory.
 *   Calls marked "host copy, synchronous" block until their copy is done.
 *   Errors: every call returns an sx_status; SX_OK is 0.  On error nothing
 *   has been enqueued and sx_last_error() describes the cause.  No C++
 *   exception crosses the ABI.  A context is not thread-safe.
 *
 * Walkers.  A context advances W walkers (replicas) with the same CV
 * definitions.  Walker w's atoms are rows [atom_off[w], atom_off[w+1]) of the
 * position buffer; CV atom indices are relative to that first row.
 *
 * Position / force layouts (sx_layout): SX_AOS3 x0 y0 z0 x1 ...; SX_AOS4
 * x0 y0 z0 w0 x1 ... (the fourth component is ignored and never written);
 * SX_SOA x0 x1 ... xN-1 y0 ... z0 ... (N = atom_off[W]).  Forces always use
 * the layout of the positions and are float32.
 */
#ifndef SAMPX_H
#define SAMPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sx_ctx sx_ctx;

typedef enum sx_status {
    SX_OK = 0,
    SX_EINVAL = 1,     /* bad argument: index, sigma <= 0, n == m, lo >= hi, ... */
    SX_ENOMEM = 2,     /* a bound buffer is smaller than the size query said */
    SX_ECAPACITY = 3,  /* a hill deposition found its walker's list full */
    SX_ENONFINITE = 4, /* a CV value or bias came out NaN/Inf */
    SX_EDEVICE = 5,    /* a HIP runtime call failed */
    SX_ESTATE = 6      /* call out of order (e.g. step before bind) */
} sx_status;

typedef enum sx_dtype { SX_F32 = 0, SX_F64 = 1 } sx_dtype;
typedef enum sx_layout { SX_AOS3 = 0, SX_AOS4 = 1, SX_SOA = 2 } sx_layout;

/* Passing this as `step` to sx_step uses the device-held step counter. */
#define SX_STEP_DEVICE (-1)

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL:
 * the null stream).  The context owns only host memory until sx_bind. */
sx_status sx_create(sx_ctx **out, int device, void *stream);
/* Destroy a context (and its captured graph, if any).  NULL is ignored. */
void sx_destroy(sx_ctx *ctx);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *sx_last_error(const sx_ctx *ctx);
/* Static text for a status code. */
const char *sx_status_string(int status);
/* Change the stream later work is enqueued on (hipStream_t). */
sx_status sx_set_stream(sx_ctx *ctx, void *stream);

/* ------------------------------------------------- collective variables */
/* Each call appends one CV; its index d (0-based, in call order) is the
 * position of its value in every xi vector.  Host arrays are copied.
 * Allowed only before sx_bind. */

/* DihedralAngle of atoms idx[0..3] (Sec. 2.2, FourPointCV): with
 * b1 = r1-r0, b2 = r2-r1, b3 = r3-r2, n1 = b1 x b2, n2 = b2 x b3,
 * phi = atan2(|b2| b1.n2, n1.n2) in (-pi, pi]; periodic with period 2 pi.
 * Positions are used as given (molecules unwrapped).  EINVAL: negative index
 * or repeated atom. */
sx_status sx_add_cv_dihedral(sx_ctx *ctx, const int32_t idx[4]);

/* RadiusofGyration of atoms idx[0..n) (Sec. 2.2): unweighted,
 * Rg = sqrt((1/n) sum |r_i - rbar|^2); not periodic; positions as given.
 * EINVAL: n < 2, negative or repeated index. */
sx_status sx_add_cv_gyration(sx_ctx *ctx, const int32_t *idx, int32_t n);

/* Coordination number between groups a[0..na) and b[0..nb):
 * CN = sum_{i in a} sum_{j in b, j != i} s(r_ij), s(r) = (1-(r/r0)^n)/(1-(r/r0)^m),
 * minimum image in the box of sx_set_box.  rcut > 0 drops pairs at r >= rcut
 * and evaluates the sum with cell lists (then the box must be set and
 * every box edge must be >= 3 rcut); rcut <= 0 visits all pairs.
 * normalize != 0 divides by na.  Not periodic as a CV.  EINVAL: r0 <= 0,
 * n < 1, m <= n, empty group, negative index. */
sx_status sx_add_cv_coordination(sx_ctx *ctx, const int32_t *a, int32_t na, const int32_t *b, int32_t nb,
                                 double r0, int32_t n, int32_t m, double rcut, int32_t normalize);

/* Orthorhombic box edges L[3] (nm) for minimum images; 0 = open in that
 * direction.  Default: open.  Before sx_bind. */
sx_status sx_set_box(sx_ctx *ctx, const double L[3]);
/* Coordination numbers with a hard cut (rcut > 0) in a periodic box at
 * least 3 rcut wide can be evaluated through cell lists (in x and y cells of
 * edge >= the largest such cut, 3 to 16 per dimension; in z such cells cut
 * into 4, 2 or 1 sub-cells, at most 4096 cells in all): each step sorts the
 * groups' members into cells (stable, so every sum has a fixed order), sums
 * pairs over the neighbour cells in one pass that also keeps each member's
 * gradient per (CV, side), and computes forces as a vector-Jacobian product
 * from those gradients (the per-pair Jacobian is never stored, so it is
 * absent from sx_eval_cv's jac_out and sx_jac_slots).  mode: -1 never; 0
 * (default) when |A| |B| >= 2^22; 1 whenever the box allows.  The groups of
 * all such CVs must be identical or disjoint (mode 1: SX_EINVAL otherwise;
 * mode 0 then keeps the all-pairs kernels); at most 8 distinct groups, each
 * used by at most 8 (CV, side) pairs.  Not with ABF (which needs J itself).
 * Before sx_bind. */
sx_status sx_set_cell_lists(sx_ctx *ctx, int32_t mode);
/* Number of CVs the bound plan evaluates through cell lists. */
int32_t sx_cell_list_cvs(const sx_ctx *ctx);

/* Number of CVs defined so far (D). */
int32_t sx_num_cvs(const sx_ctx *ctx);

/* ---------------------------------------------------------------- walkers */
/* W walkers; atom_off[0..W] (host) gives each walker's rows in the position
 * buffer (non-decreasing, atom_off[0] may be > 0).  hill_capacity[0..W)
 * (host, may be NULL) bounds each walker's private hill list (NULL: the
 * capacity of sx_metad_config for all).  shared_hills != 0 makes all walkers
 * read and append to ONE hill list of capacity hill_capacity[0] (or the
 * sx_metad_config capacity); deposits of one step are appended in walker
 * order.  Default: one walker, atom_off = {0, max CV index + 1}. */
sx_status sx_set_walkers(sx_ctx *ctx, int32_t n_walkers, const int64_t *atom_off, const int64_t *hill_capacity,
                         int32_t shared_hills);

/* ---------------------------------------------------------------- methods */
/* Metadynamics (Sec. 2.1.5).  Bias V(xi) = sum_k h_k exp(-sum_d D_kd^2/(2 sigma_d^2)),
 * D_kd = xi_d - s_kd taken to the minimum image for periodic CVs.  Every
 * `stride` steps (step % stride == 0, step 0 included) one hill per walker is
 * deposited at s = xi(x_t) after the step's forces are computed, with height
 * w exp(-V_t(s)/(k_B dT)) (well-tempered, Barducci et al. 2008), dT =
 * (bias_factor - 1) T.  The well-tempered variant is on iff
 * 1 < bias_factor < inf; bias_factor <= 0 or inf gives plain metadynamics
 * (constant height w).  sigma: host array of D widths (rad or CV units).
 * capacity: default hill capacity per walker.  EINVAL: sigma <= 0, w <= 0,
 * 0 < bias_factor <= 1, T <= 0 with well-tempering, stride < 0,
 * capacity < 1, D > 3.  Before sx_bind; needs the CVs defined. */
sx_status sx_metad_config(sx_ctx *ctx, const double *sigma, double w, double temperature, double bias_factor,
                          int32_t stride, int64_t capacity);
/* Same with the well-tempering temperature dT given directly (dT <= 0 or
 * inf: plain metadynamics), as in the butane example of the appendix. */
sx_status sx_metad_config_dT(sx_ctx *ctx, const double *sigma, double w, double delta_T, int32_t stride,
                             int64_t capacity);

/* FUNN (Sec. 2.1.8, force-biasing using neural networks): the context's
 * network (sx_surrogate_config, which on an ABF context sets up FUNN's
 * network; its features and output scale as for the surrogate) is fitted by
 * Adam, gradient term only (alpha 0, beta 1), to `walker`'s ABF mean
 * forces Fsum / N at the centres of the visited bins (bin order; the
 * batches cycle through them), `steps` steps of `batch` with a cosine decay
 * from lr to lr_final.  n_samples (host, may be NULL): visited bins used.
 * loss_out as sx_surrogate_fit.  Synchronous.  ESTATE: not ABF, no
 * parameters, no visited bin; EINVAL: more visited bins than max_samples. */
sx_status sx_funn_fit(sx_ctx *ctx, int32_t walker, int32_t batch, int32_t steps, double lr, double lr_final,
                      int64_t *n_samples, double *loss_out);
/* on != 0: every ABF step biases with the network's gradient at xi (one
 * network for all walkers; inside the grid's range) instead of
 * Fsum / max(N, N_thr); samples keep accumulating into the grid, so the
 * network can be refitted as the run advances.  ESTATE: not ABF or no
 * parameters. */
sx_status sx_funn_enable(sx_ctx *ctx, int32_t on);

/* ABF with the momentum-derivative estimator (Darve et al. 2008, the
 * algorithm the ABF of Sec. 2.1.4 follows) instead of the projected system
 * force.  masses: n_atoms (all walkers' atoms, > 0; host, copied); dt: the
 * time between consecutive sx_step calls.  sx_step's sys_forces argument
 * then carries the atoms' momenta p (float32, the layout of pos), and per
 * walker
 *   W p   = (J M^-1 J^T)^-1 J M^-1 p          (CV-space momentum)
 *   theta = b_prev - (W p - (W p)_prev) / dt   (estimate of dA/dxi)
 * with b_prev the bias of the previous step; the walker's first step adds
 * no sample.  The previous W p and bias live in the state.  masses NULL and
 * n_atoms 0: back to the projected force.  sx_bind fails with EINVAL
 * unless ABF is configured and n_atoms equals the walkers' total.  Before
 * sx_bind. */
sx_status sx_abf_momentum(sx_ctx *ctx, double dt, const double *masses, int64_t n_atoms);

/* Free energy from a metadynamics bias (Sec. 2.1.5) at n points xi
 * (device, n x D): F = -V (plain) or, well-tempered, F = -(T + dT)/dT V with
 * V the exact hill sum of `walker`'s list (0 for a shared list) and T the
 * simulation temperature (ignored for plain metadynamics).  F_out (device,
 * n); not shifted.  Stream-ordered.  ESTATE: no metadynamics. */
sx_status sx_fes_metad(sx_ctx *ctx, int32_t walker, const double *xi, int64_t n, double temperature, double *F_out);
/* The same free energy on an analysis grid, shifted to min 0 (Sec. 2.1.5):
 * per CV d the nodes lo[d] + i (hi[d] - lo[d]) / nbins[d], i < nbins[d] for
 * a periodic CV (the range wraps), i <= nbins[d] otherwise; row-major, the
 * first CV slowest.  nodes (host, D; may be NULL) receives the node count
 * per CV.  F_host NULL: only that size query.  Otherwise F_host (host,
 * n_nodes = the product of the node counts) receives F - min F.  lo, hi,
 * nbins: host, D.  Allocates temporary device memory for the nodes and
 * synchronises the stream (an analysis call, not part of a step).  EINVAL:
 * lo >= hi, nbins < 1, n_nodes not the node count. */
sx_status sx_fes_metad_grid(sx_ctx *ctx, int32_t walker, const double *lo, const double *hi, const int32_t *nbins,
                            double temperature, int32_t *nodes, double *F_host, int64_t n_nodes);
/* Free energy A from `walker`'s ABF grid (Sec. 2.1.4) at the bin centres:
 * the mean forces g = Fsum / N of the visited bins integrated by least
 * squares over pairs of neighbouring visited bins along each CV,
 * ((A_j - A_i)/delta - (g_i + g_j)/2)^2 summed (periodic CVs wrap; the
 * trapezoidal rule in 1-D), solved by conjugate gradients in FP64 on the
 * host; shifted to min 0 over the visited bins, NaN at unvisited ones.
 * A: host, nbins_total.  Assumes the visited bins are connected.
 * Synchronous.  ESTATE: no ABF. */
sx_status sx_abf_fes(sx_ctx *ctx, int32_t walker, double *A);

/* Harmonic biasing (Sec. 2.1.1) with one window per walker, the sampling
 * of umbrella sampling / umbrella integration (Sec. 2.1.2).  k: D spring
 * constants (> 0; kJ/mol per CV unit squared); centers: n_walkers x D
 * window centres xi0_w (host, copied).  Each sx_step adds
 *   V_w = sum_d k_d D_d^2 / 2,   D = xi_w - xi0_w (minimum image for a
 *   periodic CV),   forces += -sum_d k_d D_d dxi_d/dx
 * and adds the sample to the walker's window sums (count, sum D,
 * sum D D^T; FP64, in the state).  n_walkers must equal the walker count at
 * sx_bind (EINVAL there otherwise).  EINVAL: k <= 0, non-finite centre,
 * D > 3.  Before sx_bind.  Exclusive with metadynamics and ABF. */
sx_status sx_harmonic_config(sx_ctx *ctx, const double *k, const double *centers, int32_t n_walkers);
/* Clear the window sums (e.g. after equilibration).  Stream-ordered. */
sx_status sx_umbrella_reset(sx_ctx *ctx);
/* Per window: samples n (W), mean xi0 + <D> (W x D) and covariance
 * <D D^T> - <D><D>^T (W x D x D); host outputs, each may be NULL.
 * Synchronous. */
sx_status sx_umbrella_stats(sx_ctx *ctx, int64_t *n, double *mean, double *cov);
/* Umbrella integration over the windows in walker order (the path): the
 * mean force on window w, k (xi0_w - <xi>_w) (minimum image), estimates
 * dA/dxi at the window mean; A along the path of means by the trapezoidal
 * rule, A_0 = 0, A_{w+1} = A_w + (g_w + g_{w+1}) . (m_{w+1} - m_w) / 2.
 * mean_force (W x D) and A (W): host, may be NULL (not both).  ESTATE: a
 * window without samples.  Synchronous. */
sx_status sx_umbrella_integrate(sx_ctx *ctx, double *mean_force, double *A);

/* Keep the metadynamics bias on a grid (Sec. 2.1.5: the bias may be stored
 * on a pre-defined grid, trading accuracy for speed).  Per CV d: nbins[d]
 * (>= 2) intervals of [lo_d, hi_d]; a periodic CV (dihedral) needs
 * hi - lo = 2 pi and has nbins[d] nodes lo + i delta that wrap, a
 * non-periodic one nbins[d] + 1 nodes up to hi.  Each hill list (one per
 * walker, or the shared one) has a grid of FP64 node values: the list's
 * bias V and its gradient dV/dxi at every node (the exact Gaussian sum,
 * kept current as hills are appended and rebuilt by sx_hills_set).  A step
 * then reads V and dV/dxi at xi by multilinear interpolation over the 2^D
 * nodes of xi's cell (each interpolated on its own: the force uses the
 * interpolated gradient), instead of summing the hills; outside a
 * non-periodic range the bias is zero and nothing is deposited (a walker of
 * a shared list keeps its slot with a zero-height hill).  Well-tempered
 * heights use the grid's V.  Grids live in the state (so export/import
 * carry them).  sx_hillsum and sx_bias_eval still sum the hills exactly.
 * All three arguments NULL: no grid.  Before sx_bind; sx_bind fails with
 * EINVAL unless metadynamics is configured.  EINVAL: lo >= hi, nbins < 2,
 * a periodic range other than 2 pi, D > 3, more than 2^28 nodes. */
sx_status sx_metad_grid(sx_ctx *ctx, const double *lo, const double *hi, const int32_t *nbins);
/* Nodes per grid of the bound state (0 without a grid). */
int64_t sx_grid_nodes(const sx_ctx *ctx);
/* The grid read-back at n points xi (device, n x D, FP64) of the grid of
 * `walker`'s hill list (0 for a shared list): V_out (device, n) and, if
 * not NULL, dVdxi_out (device, n x D).  Stream-ordered.  ESTATE: no grid. */
sx_status sx_grid_eval(sx_ctx *ctx, int32_t walker, const double *xi, int64_t n, double *V_out, double *dVdxi_out);
/* Copy the node values of `walker`'s grid to the host: V (n_nodes) and, if
 * not NULL, dVdxi (D x n_nodes, CV-major), nodes row-major (first CV
 * slowest).  n_nodes must equal sx_grid_nodes.  Synchronous. */
sx_status sx_grid_get(sx_ctx *ctx, int32_t walker, double *V, double *dVdxi, int64_t n_nodes);

/* Adaptive biasing force (Sec. 2.1.4; Darve et al. 2008).  A grid of
 * nbins[d] bins on [lo_d, hi_d) per CV (row-major, first CV slowest).  At
 * every step, with J = dxi/dx and the system force F passed to sx_step:
 *   theta = -(J J^T)^{-1} J F          (estimate of dA/dxi, unit masses)
 *   b     = Fsum[k] / max(N[k], n_threshold)    (samples before this step)
 *   N[k] += 1, Fsum[k] += theta
 *   forces += sum_d b_d J_d
 * Periodic CVs (dihedrals) wrap the bin index and need hi - lo = 2 pi; a
 * non-periodic CV outside [lo, hi) drops the sample and gets no bias.  Each
 * walker has its own grid.  EINVAL: lo >= hi, nbins < 1, n_threshold < 0,
 * D > 3.  Before sx_bind.  Exclusive with metadynamics. */
sx_status sx_abf_config(sx_ctx *ctx, const double *lo, const double *hi, const int32_t *nbins,
                        int32_t n_threshold);

/* ------------------------------------------------------- memory binding */
/* Bytes of the persistent state (hills, counts, ABF grid, step counter,
 * surrogate weights) and of the workspace (per-step scratch plus index
 * tables).  Valid once CVs, walkers and the method are set. */
size_t sx_state_bytes(const sx_ctx *ctx);
size_t sx_workspace_bytes(const sx_ctx *ctx);
/* Bind caller-owned device buffers (256-byte aligned) of at least the
 * queried sizes.  Zeroes the state (no hills, empty grid, step counter 0),
 * uploads the index tables and synchronises the stream.  ENOMEM: a buffer
 * is too small; EINVAL: misaligned or NULL. */
sx_status sx_bind(sx_ctx *ctx, void *dev_state, size_t state_bytes, void *dev_ws, size_t ws_bytes);

/* ------------------------------------------------------------- hot path */
/* One biasing update (the method's update step) for all walkers:
 *   xi = CVs(pos); bias and dV/dxi (metadynamics: hill sum; ABF: grid);
 *   forces += -sum_d dV/dxi_d dxi_d/dx; then hill deposition / grid update.
 * pos: device, dtype/layout as given.  step >= 0: the step number used for
 * the deposition stride (and the device counter is set to step + 1);
 * SX_STEP_DEVICE: use and advance the device-held counter.
 * Outputs (device, may be NULL): xi_out[W][D], V_out[W] (metadynamics bias;
 * ABF: 0), dVdxi_out[W][D] (ABF: -b, the derivative of the bias potential).
 * forces: device float32, same layout as pos, ADDED to.  sys_forces: device
 * float32 system forces, same layout (ABF only; NULL otherwise).
 * Capacity overflow and non-finite values are flagged on the device and
 * reported by sx_check. */
sx_status sx_step(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, int64_t step, double *xi_out,
                  double *V_out, double *dVdxi_out, float *forces, const float *sys_forces);

/* Synchronise the stream and report device-side flags raised since the last
 * sx_check (ECAPACITY, ENONFINITE), then clear them. */
sx_status sx_check(sx_ctx *ctx);

/* ------------------------------------------------------------ pieces */
/* CV values xi_out[W][D] (device) and, if jac_out != NULL, the sparse
 * Jacobian jac_out[W][n_slots][3] (device float32): slot s holds
 * d xi_{cv(s)} / d r_{atom(s)} for one member atom of one CV (see
 * sx_jac_layout).  The PySAGES counterpart is the JAX gradient of the CVs. */
sx_status sx_eval_cv(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, double *xi_out, float *jac_out);
/* Number of Jacobian slots per walker (valid after sx_bind). */
int64_t sx_jac_slots(const sx_ctx *ctx);
/* Host copy of the slot layout: atom index (walker-relative) and CV index of
 * each slot; arrays of sx_jac_slots entries. */
sx_status sx_jac_layout(const sx_ctx *ctx, int32_t *atom, int32_t *cv);
/* Vector-Jacobian product (the backward of the CV map):
 *   pos_bar += sum_d xi_bar[w][d] d xi_d / d r   for every atom of every walker.
 * The Jacobian is recomputed from pos (gather form, no atomics).  xi_bar:
 * device double [W][D]; pos_bar: device float32 in the layout of pos. */
sx_status sx_cv_vjp(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, const double *xi_bar,
                    float *pos_bar);
/* Metadynamics bias at given CV values: V_out[W], dVdxi_out[W][D] from
 * xi[W][D] (all device).  No deposition, no forces. */
sx_status sx_hillsum(sx_ctx *ctx, const double *xi, double *V_out, double *dVdxi_out);
/* Deposit one hill per walker at xi[W][D] (device) now, whatever the step,
 * with the well-tempered height from the current bias at xi.  With a shared
 * list the W hills are appended in walker order, all or none. */
sx_status sx_deposit(sx_ctx *ctx, const double *xi);
/* Metadynamics bias of one hill list at n arbitrary points: xi[n][D] ->
 * V_out[n], dVdxi_out[n][D] (device; outputs may be NULL).  walker selects
 * the private list (ignored with a shared list).  Same arithmetic as the
 * step's sum; evaluated in batches of 65536 points.  Used for surrogate
 * training labels and certification. */
sx_status sx_bias_eval(sx_ctx *ctx, int32_t walker, const double *xi, int64_t n, double *V_out, double *dVdxi_out);
/* sx_bias_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same kernels and results, with their partial sums in a fixed 16 MiB array
 * inside the library (one per GPU, held until the process ends; its address
 * is looked up in sx_create) instead of the bound workspace.  Allocates
 * nothing and calls no allocating routine.  The caller passes xi, V_out and
 * dVdxi_out (device) as for sx_bias_eval.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (two streams, two contexts) race.
 * ENOMEM when a batch's partial sums would exceed the array (not reached by
 * the 65536-point batches: at most 8 chunks x 65536 points x 32 B). */
sx_status sx_bias_eval_noalloc(sx_ctx *ctx, int32_t walker, const double *xi, int64_t n, double *V_out,
                               double *dVdxi_out);

/* ------------------------------------------------------------ state I/O */
/* Host copies, synchronous.  Walker -1 (or any walker) addresses the shared
 * list when hills are shared.  centers: K x D row-major float32. */
sx_status sx_hills_set(sx_ctx *ctx, int32_t walker, const float *centers, const float *heights, int64_t K);
sx_status sx_hills_get(sx_ctx *ctx, int32_t walker, float *centers, float *heights, int64_t max_K, int64_t *K);
/* ABF grid of walker w: N[nbins_total] counts and Fsum[nbins_total][D]. */
sx_status sx_abf_grid_get(sx_ctx *ctx, int32_t walker, uint32_t *N, double *Fsum);
/* Device step counter (the next step number SX_STEP_DEVICE will use). */
sx_status sx_get_step(sx_ctx *ctx, int64_t *step);
/* Checkpoint: the whole state buffer with a header that identifies the
 * configuration; import refuses a checkpoint of another configuration. */
size_t sx_checkpoint_bytes(const sx_ctx *ctx);
sx_status sx_state_export(sx_ctx *ctx, void *host, size_t bytes);
sx_status sx_state_import(sx_ctx *ctx, const void *host, size_t bytes);

/* ------------------------------------------------- graphs and tuning */
/* Capture n_steps consecutive sx_step calls (device step counter) with the
 * given buffers into one HIP graph owned by the context; sx_graph_launch
 * replays it on the context's stream.  Buffers must stay valid while the
 * graph exists.  A new capture replaces the previous graph. */
sx_status sx_graph_capture(sx_ctx *ctx, int32_t n_steps, const void *pos, int32_t dtype, int32_t layout,
                           double *xi_out, double *V_out, double *dVdxi_out, float *forces,
                           const float *sys_forces);
sx_status sx_graph_launch(sx_ctx *ctx);
/* Launch parameters of the hill-sum kernel: hills per tile (1024, 2048,
 * 4096 or 8192) and persistent grid size (0: one workgroup per
 * tile).  Changing the tile rebuilds the tile table (host, synchronous).
 * With a shared hill list `grid` is instead the number of workgroups the
 * step's shared sum aims at (chunks x query blocks; 0: 2048) and the tile
 * is unused.  A change releases a captured graph (sx_graph_launch then
 * returns SX_ESTATE until the next sx_graph_capture); so does sx_autotune. */
sx_status sx_set_tuning(sx_ctx *ctx, int32_t tile_hills, int32_t grid);
sx_status sx_get_tuning(const sx_ctx *ctx, int32_t *tile_hills, int32_t *grid);
/* Time candidate tilings of the step's hill-sum kernels on the bound state
 * and keep the fastest.  pos (device, may be NULL): positions in the form
 * sx_step receives them, so that the CVs the hill kernels evaluate
 * themselves (all-dihedral sets) are timed as in the step; with NULL the
 * CV values of the last step are used.  Nothing is deposited and no force
 * is written.  cache_path (may be NULL): a JSON file of earlier choices
 * keyed by the problem shape; read first, updated after a search.  Each
 * candidate runs as a captured graph of 20 launches of the step's hill
 * kernels (the tile kernel and the finalize, or the one kernel of a step
 * whose hills are one tile), timed with hipEvents (best of three replays);
 * synchronous. */
sx_status sx_autotune(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, const char *cache_path);

/* ------------------------------------------------- bias surrogate */
/* A small tanh network of the CVs that stands in for the metadynamics bias
 * of hill list 0 (the shared list, or the one walker's list) once the bias
 * is frozen: the network precedent is the paper's ANN and FUNN methods
 * (Sec. 2.1.7, 2.1.8) applied to the hill-sum bias of Sec. 2.1.5.
 *   features f: (sin xi_d, cos xi_d) periodic CV; (u, u^2) otherwise with
 *               u = (xi_d - mu_d) / s_d (sx_surrogate_norm)
 *   y = w3 . tanh(W2 tanh(W1 f + b1) + b2) + b3,  V = shift + scale * y
 * W2 runs on the matrix cores in bf16 with FP32 accumulation; every weight
 * is used at its bf16 value (FP32 master copies are trained).  dV/dxi is
 * the network's exact derivative (forward tangents).  Certified cells of a
 * cert_n^D grid use the network; the others fall back to the exact sum.
 *
 * Declare before sx_bind (it sizes state and workspace).  hidden: 64 or
 * 128 (0 removes the network); max_samples: training points per call;
 * max_batch: samples per optimiser step; cert_n: grid cells per CV;
 * tol_force: the largest |dVhat/dxi - dV/dxi| (2-norm over the CVs,
 * kJ/mol/rad) a certified cell may show.  Needs sx_metad_config, 1-3 CVs. */
sx_status sx_surrogate_config(sx_ctx *ctx, int32_t hidden, int64_t max_samples, int32_t max_batch, int32_t cert_n,
                              double tol_force);
/* Standardisation of non-periodic CVs (host arrays of D; s > 0). */
sx_status sx_surrogate_norm(sx_ctx *ctx, const double *mu, const double *s);
/* Number of parameters P = H(2D) + H + H^2 + H + H + 1, stored in the order
 * W1[H][2D], b1[H], W2[H][H], b2[H], w3[H], b3 (0 without a network). */
int64_t sx_surrogate_param_count(const sx_ctx *ctx);
/* FP32 parameters from / to host memory (count == P).  Setting them resets
 * the optimiser and drops the certification; synchronous. */
sx_status sx_surrogate_params_set(sx_ctx *ctx, const float *params, int64_t count);
sx_status sx_surrogate_params_get(sx_ctx *ctx, float *params, int64_t count);
/* Output affine V = shift + scale * y (scale != 0); sx_surrogate_train sets
 * it from the mean and spread of its targets. */
sx_status sx_surrogate_output(sx_ctx *ctx, double scale, double shift);
sx_status sx_surrogate_output_get(const sx_ctx *ctx, double *scale, double *shift);
/* Network at n points: xi[n][D] -> V_out[n], dVdxi_out[n][D] (device, FP64;
 * outputs may be NULL).  fallback (device uint8[n], may be NULL; needs a
 * certification): 1 where the point's cell is not certified. */
sx_status sx_surrogate_eval(sx_ctx *ctx, const double *xi, int64_t n, double *V_out, double *dVdxi_out,
                            uint8_t *fallback);
/* Sobolev loss of the network over n <= max_batch samples (device xi[n][D],
 * V[n], G[n][D], physical units; the output affine maps them to network
 * units) and its gradient with respect to every parameter:
 *   L = (1/n) sum_i [alpha (y_i - V'_i)^2 + beta sum_d (dy_i/dxi_d - G'_id)^2]
 * with V' = (V - shift)/scale, G' = G/scale.  grad_host: host double[P]
 * (FP64 sum of FP32 per-workgroup partials), loss_host: host double.
 * Synchronous.  Used to check the reverse kernels. */
sx_status sx_surrogate_loss_grad(sx_ctx *ctx, const double *xi, const double *V, const double *G, int64_t n,
                                 double alpha, double beta, double *grad_host, double *loss_host);
/* `steps` Adam steps (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8)
 * on the Sobolev loss above, over consecutive batches of `batch` samples of
 * the n device samples (cyclic; give the samples in random order), with the
 * learning rate decaying from lr to lr_final on a cosine.  loss_out (host,
 * may be NULL): mean loss of the last batch.  Synchronous at the end. */
sx_status sx_surrogate_fit(sx_ctx *ctx, const double *xi, const double *V, const double *G, int64_t n, int32_t batch,
                           int32_t steps, double lr, double lr_final, double alpha, double beta, double *loss_out);
/* Fit to the exact bias: evaluates V and dV/dxi of hill list 0 at the n
 * device points xi[n][D] (n <= max_samples), sets the output affine to their
 * mean and standard deviation, and runs sx_surrogate_fit with alpha = 1 and
 * beta = 1 / (mean gradient variance in network units).  Synchronous. */
sx_status sx_surrogate_train(sx_ctx *ctx, const double *xi, int64_t n, int32_t batch, int32_t steps, double lr,
                             double lr_final, double *loss_out);
/* Certify cells of a cert_n^D grid over [-pi, pi) for periodic CVs and
 * [lo_d, hi_d] (host arrays; may be NULL if every CV is periodic) otherwise:
 * the exact and the network gradient are evaluated at every grid corner; a
 * cell is certified when the largest corner error plus twice the largest
 * corner-to-corner change of the error per unit length times the half
 * diagonal is at most tol_force.  certified_fraction (host, may be NULL).
 * The certification describes the current hill list and network: setting
 * hills or parameters, depositing, training or an exact step that may
 * deposit drops it.  Synchronous. */
sx_status sx_surrogate_certify(sx_ctx *ctx, const double *lo, const double *hi, double *certified_fraction);
/* Change the certification tolerance (kJ/mol per CV unit, > 0); drops the
 * certification. */
sx_status sx_surrogate_tolerance(sx_ctx *ctx, double tol_force);
/* Switch the surrogate into sx_step (needs parameters and a certification;
 * a shared hill list or one walker).  While on, the step evaluates the
 * network for every walker, the exact sum of the shared list for the
 * walkers whose cell is not certified, and deposits nothing (the network
 * stands for a frozen bias). */
sx_status sx_surrogate_enable(sx_ctx *ctx, int32_t on);
/* Walkers that took the exact fallback in the last surrogate step (host
 * int32; synchronous). */
sx_status sx_surrogate_fallback_count(sx_ctx *ctx, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif /* SAMPX_H */
