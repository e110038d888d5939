/*
 * sampx measurement library (libsampx_measure.so): kernel-level timing of
 * the biasing-force path and plain bandwidth probes, for benchmarks and
 * profiles.  Not part of the biasing-path boundary (include/sampx.h);
 * nothing here is needed to run a sampling method.
 *
 * The three sxm_* entry points are kernel-level enqueue primitives that
 * libsampx.so itself exports for this library; the sx_time_* and sx_probe_*
 * calls live in libsampx_measure.so, which links libsampx.so.
 * Conventions (device pointers, layouts, status codes) as in sampx.h.
 */
#ifndef SAMPX_MEASURE_H
#define SAMPX_MEASURE_H

#include "sampx.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------- hooks in libsampx.so */
/* The context's stream (hipStream_t). */
void *sxm_stream(const sx_ctx *ctx);
/* Enqueue one kernel of the private-list hill sum on `stream` (hipStream_t)
 * with the step's configuration (CVs from pos as sx_step evaluates them,
 * tiling as tuned), depositing nothing and leaving the step counter alone:
 * which = 0 prepares (CVs when the tile kernel does not evaluate them, then
 * one tile-kernel launch, so the finalize finds xi and the Jacobian),
 * 1 the tile kernel, 2 the finalize kernel (adds the bias force to forces,
 * device, layout of pos, when not NULL).  ESTATE without private hill lists
 * summed by tiles. */
sx_status sxm_enqueue_hill(sx_ctx *ctx, void *stream, const void *pos, int32_t dtype, int32_t layout, float *forces,
                           int32_t which);
/* The cell-list coordination-number kernels on `stream`: which = 0 sort
 * and pair pass, 1 the cell sort, 2 the pair pass (CV values and the
 * members' gradients, with its finalize), 3 the vector-Jacobian gather
 * adding -dV/dxi (of the last step) times those gradients to forces
 * (device, layout of pos; required).  ESTATE without such CVs. */
sx_status sxm_enqueue_cell(sx_ctx *ctx, void *stream, const void *pos, int32_t dtype, int32_t layout, float *forces,
                           int32_t which);

/* ---------------------------------- libsampx_measure.so: timing, probes */
/* Average duration of the step's two hill-sum kernels: `reps` launches of
 * the tile kernel captured in one HIP graph, then `reps` of the finalize
 * kernel in another, each graph replayed twice to warm up, then five
 * times between hipEvents on the context's stream (the stream the kernels
 * run on); the median replay per launch, so the figure includes the
 * graph's gap between consecutive launches.  Nothing is
 * deposited and the step counter is untouched; if forces is not NULL the
 * bias force is added to it `reps` times per replay (seven replays).
 * Synchronous.
 * ms_tiles / ms_finalize: host, milliseconds per launch. */
sx_status sx_time_hill(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                       float *ms_tiles, float *ms_finalize);
/* The pair of them as a step runs them: `reps` (tile kernel, finalize
 * kernel) pairs in one graph, ms per pair; and ms per launch of a graph of
 * `reps` launches of a one-workgroup kernel that does nothing (what a
 * launch in a graph costs by itself).  Synchronous. */
sx_status sx_time_hill_step(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                            float *ms_pair, float *ms_noop);
/* The same for the cell-list kernels: the cell sort, the pair pass (with
 * its finalize) and the vector-Jacobian gather into forces (may be NULL:
 * not timed, ms_vjp = 0).  Synchronous; ms per launch. */
sx_status sx_time_cell(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                       float *ms_sort, float *ms_pairs, float *ms_vjp);

/* Plain streaming read of `bytes` (multiple of 16) from device memory src
 * with `grid` workgroups; each workgroup writes one float to sink[grid]
 * (device).  nontemporal != 0: non-temporal loads (the hill kernels' kind).
 * Enqueued on `stream` (hipStream_t).  Calibrates the traffic counters and
 * measures the achievable read rate. */
sx_status sx_probe_read(const void *src, size_t bytes, float *sink, int32_t grid, int32_t nontemporal, void *stream);
/* One launch of a one-workgroup kernel that does nothing, on `stream`. */
sx_status sx_probe_noop(void *stream);
/* Plain copy of `bytes` (multiple of 16) from src to dst (device, not
 * overlapping) with `grid` workgroups, enqueued on `stream`. */
sx_status sx_probe_copy(void *dst, const void *src, size_t bytes, int32_t grid, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SAMPX_MEASURE_H */
