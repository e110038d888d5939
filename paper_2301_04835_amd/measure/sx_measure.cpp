// Kernel-level timing of the biasing-force path (libsampx_measure.so):
// `reps` launches of one kernel are captured into a HIP graph through the
// hooks libsampx exports (sxm_enqueue_*), the graph is replayed twice to
// warm up and then kTrials times, each replay between hipEvents on the
// context's stream; the median replay divided by reps is the figure.
// Replaying a graph keeps host launch cost out of it: the kernels run back
// to back on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>

#include "../../include/sampx_measure.h"

namespace {

constexpr int kWarm = 2, kTrials = 5;

// capture reps calls of enq(stream) into a graph, replay it between events
// on `run`; median ms per call into *ms
sx_status time_graph(hipStream_t run, int32_t reps, const std::function<sx_status(hipStream_t)> &enq, float *ms)
{
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SX_EDEVICE;
    sx_status st = SX_OK;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipEvent_t ev[kTrials + 1] = {};
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        for (int r = 0; r < reps && st == SX_OK; ++r) st = enq(cap);
        e = hipStreamEndCapture(cap, &g);
    }
    if (st == SX_OK && e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    for (int i = 0; i <= kTrials && st == SX_OK && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (int i = 0; i < kWarm && st == SX_OK && e == hipSuccess; ++i) e = hipGraphLaunch(ge, run);
    if (st == SX_OK && e == hipSuccess) e = hipEventRecord(ev[0], run);
    for (int i = 1; i <= kTrials && st == SX_OK && e == hipSuccess; ++i) {
        e = hipGraphLaunch(ge, run);
        if (e == hipSuccess) e = hipEventRecord(ev[i], run);
    }
    if (st == SX_OK && e == hipSuccess) e = hipEventSynchronize(ev[kTrials]);
    float t[kTrials] = {};
    for (int i = 0; i < kTrials && st == SX_OK && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
    if (st == SX_OK && e != hipSuccess) st = SX_EDEVICE;
    if (st == SX_OK) {
        std::sort(t, t + kTrials);
        *ms = t[kTrials / 2] / reps;
    }
    // teardown: failures here cannot change the result
    for (int i = 0; i <= kTrials; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    return st;
}

}  // namespace

extern "C" {

sx_status sx_time_hill(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                       float *ms_tiles, float *ms_finalize)
{
    if (!ctx || reps < 1 || !ms_tiles || !ms_finalize) return SX_EINVAL;
    const hipStream_t run = static_cast<hipStream_t>(sxm_stream(ctx));
    sx_status st = sxm_enqueue_hill(ctx, run, pos, dtype, layout, nullptr, 0);
    auto hook = [&](int32_t which, float *f) {
        return [=](hipStream_t s) { return sxm_enqueue_hill(ctx, s, pos, dtype, layout, f, which); };
    };
    if (st == SX_OK) st = time_graph(run, reps, hook(1, nullptr), ms_tiles);
    if (st == SX_OK) st = time_graph(run, reps, hook(2, forces), ms_finalize);
    return st;
}

sx_status sx_time_hill_step(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                            float *ms_pair, float *ms_noop)
{
    if (!ctx || reps < 1 || !ms_pair || !ms_noop) return SX_EINVAL;
    const hipStream_t run = static_cast<hipStream_t>(sxm_stream(ctx));
    sx_status st = sxm_enqueue_hill(ctx, run, pos, dtype, layout, nullptr, 0);
    if (st == SX_OK)
        st = time_graph(run, reps, [=](hipStream_t s) {
            sx_status r = sxm_enqueue_hill(ctx, s, pos, dtype, layout, nullptr, 1);
            return r == SX_OK ? sxm_enqueue_hill(ctx, s, pos, dtype, layout, forces, 2) : r;
        }, ms_pair);
    if (st == SX_OK) st = time_graph(run, reps, [](hipStream_t s) { return sx_probe_noop(s); }, ms_noop);
    return st;
}

sx_status sx_time_cell(sx_ctx *ctx, const void *pos, int32_t dtype, int32_t layout, float *forces, int32_t reps,
                       float *ms_sort, float *ms_pairs, float *ms_vjp)
{
    if (!ctx || reps < 1 || !ms_sort || !ms_pairs || !ms_vjp) return SX_EINVAL;
    const hipStream_t run = static_cast<hipStream_t>(sxm_stream(ctx));
    sx_status st = sxm_enqueue_cell(ctx, run, pos, dtype, layout, nullptr, 0);
    auto hook = [&](int32_t which) {
        return [=](hipStream_t s) { return sxm_enqueue_cell(ctx, s, pos, dtype, layout, forces, which); };
    };
    if (st == SX_OK) st = time_graph(run, reps, hook(1), ms_sort);
    if (st == SX_OK) st = time_graph(run, reps, hook(2), ms_pairs);
    *ms_vjp = 0.f;
    if (st == SX_OK && forces) st = time_graph(run, reps, hook(3), ms_vjp);
    return st;
}

}  // extern "C"
