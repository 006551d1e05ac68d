// Captured rollout chunks: the step launches of a chunk recorded once into a HIP graph and
// replayed with one launch call. The step counter lives on the device, so replays need no
// parameter updates. Because the counter is double-buffered, the chunk is captured once per
// starting slot, and each replay picks the copy for the batch's current slot. Each slot has
// two copies: one whose launches carry the steps as of capture (a replay from the capture
// step: each launch fetches its action rows beside its state, without waiting for the
// counter), and one whose launches carry none (a replay from any other step: the rows
// follow from the counter). A hint that turned out wrong would cost a launch its steps
// twice; picking the copy by the replay's step keeps that from happening. Only one-step
// launches use the hints, so a graph without any has the second kind alone.
#include <hip/hip_runtime.h>

#include <new>

#include "mgx.h"
#include "runtime_internal.hpp"

using namespace mgx;

struct mgx_graph {
    mgx_batch* batch = nullptr;
    // [counter slot][0: launches without step hints, 1: with the capture step's]
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int64_t t_capture = 0;  // host step count when captured
    int64_t n_rows = 0, row0 = 0;
    int32_t hold = 1, n_steps = 0;
    int32_t n_launches = 0;
    bool stats = false;
};

static void release(mgx_graph* g) {
    for (int p = 0; p < 2; ++p)
        for (int h = 0; h < 2; ++h) {
            if (g->exec[p][h]) (void)hipGraphExecDestroy(g->exec[p][h]);
            if (g->graph[p][h]) (void)hipGraphDestroy(g->graph[p][h]);
            g->exec[p][h] = nullptr;
            g->graph[p][h] = nullptr;
        }
}

extern "C" mgx_status mgx_graph_capture(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                        int32_t n_steps, int32_t K, uint32_t flags, mgx_graph** out) {
    if (!b || !out) return fail(MGX_E_INVALID, "NULL argument");
    *out = nullptr;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params has not been called");
    if (!actions) return fail(MGX_E_INVALID, "actions is NULL");
    if (K == 0) K = b->shape_K;
    if (n_steps < 1 || K < 1 || hold < 1 || n_rows < 1) return fail(MGX_E_INVALID, "n_steps, K, hold, n_rows must be >= 1");
    if (flags & ~(MGX_STEP_UNFUSED | MGX_STEP_STATS)) return fail(MGX_E_INVALID, "unknown step flag");
    if (n_steps > (1 << 20)) return fail(MGX_E_INVALID, "n_steps too large for one graph");
    hipDevice_guard guard(b->device);
    mgx_graph* g = new (std::nothrow) mgx_graph();
    if (!g) return fail(MGX_E_NOMEM, "host allocation");
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(nullptr, e, "hipStreamCreateWithFlags");
    }
    hipStream_t saved_stream = b->stream;
    const int saved_slot = b->slot;
    const int32_t per = (flags & MGX_STEP_UNFUSED) ? 1 : K;
    const bool stats = (flags & MGX_STEP_STATS) != 0;
    mgx_status st = MGX_OK;
    b->stream = cap;
    // Only one-step launches use the step hints: a graph without any is captured once per
    // slot, and its hinted copy stays empty.
    const bool any_single = per == 1 || n_steps % per == 1;
    for (int c = 0; c < 4 && st == MGX_OK; ++c) {
        const int p = c >> 1, h = c & 1;  // counter slot; step hints or none
        if (h && !any_single) continue;
        b->slot = p;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            st = hip_fail(nullptr, e, "hipStreamBeginCapture");
            break;
        }
        int32_t launches = 0;
        for (int32_t done = 0; done < n_steps && st == MGX_OK;) {
            const int32_t k = (n_steps - done) < per ? (n_steps - done) : per;
            st = enqueue_step(b, actions, n_rows, row0, hold, k, stats && done + k == n_steps, nullptr, nullptr,
                              b->block, h ? b->host_t + done : -1);
            done += k;
            ++launches;
        }
        g->n_launches = launches;
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (st == MGX_OK && e2 != hipSuccess) st = hip_fail(nullptr, e2, "hipStreamEndCapture");
        if (st == MGX_OK) {
            g->graph[p][h] = graph;
            e2 = hipGraphInstantiate(&g->exec[p][h], graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) st = hip_fail(nullptr, e2, "hipGraphInstantiate");
        } else if (graph) {
            (void)hipGraphDestroy(graph);
        }
    }
    b->stream = saved_stream;
    b->slot = saved_slot;
    b->faulted = false;  // capture records launches only; the batch itself is untouched
    (void)hipStreamDestroy(cap);
    if (st != MGX_OK) {
        release(g);
        delete g;
        return st;
    }
    g->batch = b;
    g->t_capture = b->host_t;
    g->n_rows = n_rows;
    g->row0 = row0;
    g->hold = hold;
    g->n_steps = n_steps;
    g->stats = (flags & MGX_STEP_STATS) != 0;
    b->n_graphs += 1;
    *out = g;
    return MGX_OK;
}

extern "C" mgx_status mgx_graph_replay(mgx_graph* g) {
    if (!g || !g->batch) return fail(MGX_E_INVALID, "graph is NULL");
    mgx_batch* b = g->batch;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    mgx_status v = validate_rows(b, b->host_t, g->n_rows, g->row0, g->hold, g->n_steps);
    if (v != MGX_OK) return v;
    hipDevice_guard guard(b->device);
    const int h = (g->exec[b->slot][1] && b->host_t == g->t_capture) ? 1 : 0;
    hipError_t e = hipGraphLaunch(g->exec[b->slot][h], b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "hipGraphLaunch");
    b->host_t += g->n_steps;
    if (g->n_launches & 1) b->slot = 1 - b->slot;
    if (g->stats) b->stats_step = b->host_t;
    return MGX_OK;
}

extern "C" mgx_status mgx_graph_destroy(mgx_graph* g) {
    if (!g) return MGX_OK;
    if (g->batch) {
        hipDevice_guard guard(g->batch->device);
        (void)hipStreamSynchronize(g->batch->stream);
        g->batch->n_graphs -= 1;
    }
    release(g);
    delete g;
    return MGX_OK;
}
