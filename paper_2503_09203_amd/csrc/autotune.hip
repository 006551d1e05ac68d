// Launch-shape autotuner: times one rollout chunk for every candidate (launch mode, steps
// per launch, block size, persistent grid) with HIP events on the batch's stream, keeps the
// fastest, and caches it per (architecture, precision, class mix, hold, chunk).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mgx.h"
#include "runtime_internal.hpp"

using namespace mgx;

namespace {

struct Entry {
    std::string key;
    mgx_launch_shape shape;
};
std::mutex g_mu;
std::vector<Entry> g_cache;

std::string signature(const mgx_batch* b, int32_t hold, int32_t chunk) {
    std::ostringstream o;
    o << (b->arch.empty() ? "gpu" : b->arch.substr(0, b->arch.find(':'))) << "|p" << b->prec << "|h" << hold << "|c"
      << chunk;
    for (int c = 0; c < b->n_classes; ++c) o << "|" << b->m[c] << "x" << b->npad[c];
    return o.str();
}

bool cache_get(const std::string& key, mgx_launch_shape* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Entry& e : g_cache)
        if (e.key == key) {
            *out = e.shape;
            return true;
        }
    return false;
}

void cache_put(const std::string& key, const mgx_launch_shape& s) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (Entry& e : g_cache)
        if (e.key == key) {
            e.shape = s;
            return;
        }
    g_cache.push_back({key, s});
}

void apply(mgx_batch* b, const mgx_launch_shape& s) {
    b->mode = s.mode;
    b->shape_K = s.K;
    b->block = s.block;
    b->grid_per_cu = s.grid_per_cu;
}

}  // namespace

#define HIP_TRY_T(call)                                        \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) {                                \
            st = hip_fail(b, e_, #call);                       \
            goto done;                                         \
        }                                                      \
    } while (0)

extern "C" mgx_status mgx_autotune(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                   int32_t chunk, mgx_launch_shape* out) {
    if (!b || !actions) return fail(MGX_E_INVALID, "NULL argument");
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params has not been called");
    if (chunk < 1 || chunk > 4096 || hold < 1 || n_rows < 1) return fail(MGX_E_INVALID, "chunk in [1,4096], hold, n_rows >= 1");
    mgx_status v = validate_rows(b, b->host_t, n_rows, row0, hold, chunk);
    if (v != MGX_OK) return v;
    const std::string key = signature(b, hold, chunk);
    mgx_launch_shape best;
    std::memset(&best, 0, sizeof best);
    if (cache_get(key, &best)) {
        apply(b, best);
        best.from_cache = 1;
        if (out) *out = best;
        return MGX_OK;
    }

    hipDevice_guard guard(b->device);
    std::vector<mgx_launch_shape> cand;
    for (int K = 1; K <= chunk; K *= 2) {
        if (chunk % K) continue;
        for (int blk : {64, 128, 256}) {
            mgx_launch_shape s{MGX_LAUNCH_PER_CLASS, K, blk, 1, 0.0, 0, 0};
            cand.push_back(s);
        }
        if (b->prec == MGX_FP32)
            for (int g : {1, 2, 4}) {
                mgx_launch_shape s{MGX_LAUNCH_PERSISTENT, K, 256, g, 0.0, 0, 0};
                cand.push_back(s);
            }
    }
    if (chunk & (chunk - 1)) {  // not a power of two: the whole chunk in one launch too
        mgx_launch_shape s{MGX_LAUNCH_PER_CLASS, chunk, 256, 1, 0.0, 0, 0};
        cand.push_back(s);
        if (b->prec == MGX_FP32) cand.push_back({MGX_LAUNCH_PERSISTENT, chunk, 256, 2, 0.0, 0, 0});
    }

    const mgx_launch_shape saved{b->mode, b->shape_K, b->block, b->grid_per_cu, 0.0, 0, 0};
    const int64_t t_start = b->host_t;
    const size_t bytes = (size_t)b->prec * b->state_elems;
    void* snap = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mgx_status st = MGX_OK;
    double best_us = 1e30;
    {
        hipError_t ea;
        snap = b->dev_alloc(bytes, &ea);
        HIP_TRY_T(ea);
    }
    HIP_TRY_T(hipEventCreate(&e0));
    HIP_TRY_T(hipEventCreate(&e1));
    HIP_TRY_T(hipMemcpyAsync(snap, b->d_state, bytes, hipMemcpyDeviceToDevice, b->stream));
    for (const mgx_launch_shape& c : cand) {
        apply(b, c);
        float best_ms = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {  // first repetition warms up
            HIP_TRY_T(hipMemcpyAsync(b->d_state, snap, bytes, hipMemcpyDeviceToDevice, b->stream));
            HIP_TRY_T(launch_set_counter(b->d_misc, b->slot, t_start, b->stream));
            HIP_TRY_T(hipEventRecord(e0, b->stream));
            for (int32_t done = 0; done < chunk; done += c.K) {
                st = enqueue_step(b, actions, n_rows, row0, hold, c.K, false, nullptr, nullptr, c.block,
                                  t_start + done);
                if (st != MGX_OK) goto done;
            }
            HIP_TRY_T(hipEventRecord(e1, b->stream));
            HIP_TRY_T(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_TRY_T(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best_ms) best_ms = ms;
        }
        if (best_ms * 1e3 < best_us) {
            best_us = best_ms * 1e3;
            best = c;
        }
    }
    best.us_per_chunk = best_us;
    best.candidates = (int32_t)cand.size();
    best.from_cache = 0;
    // restore the batch: state, counter, then the winning shape
    HIP_TRY_T(hipMemcpyAsync(b->d_state, snap, bytes, hipMemcpyDeviceToDevice, b->stream));
    HIP_TRY_T(launch_set_counter(b->d_misc, b->slot, t_start, b->stream));
    HIP_TRY_T(hipStreamSynchronize(b->stream));
    apply(b, best);
    cache_put(key, best);
    if (out) *out = best;
done:
    if (st != MGX_OK) apply(b, saved);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->dev_free(snap);
    return st;
}

extern "C" mgx_status mgx_autotune_save(const char* path) {
    if (!path) return fail(MGX_E_INVALID, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(MGX_E_INVALID, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(g_mu);
    std::fprintf(f, "# mgx launch shapes: key mode K block grid_per_cu us_per_chunk candidates\n");
    for (const Entry& e : g_cache)
        std::fprintf(f, "%s %d %d %d %d %.3f %d\n", e.key.c_str(), e.shape.mode, e.shape.K, e.shape.block,
                     e.shape.grid_per_cu, e.shape.us_per_chunk, e.shape.candidates);
    std::fclose(f);
    return MGX_OK;
}

extern "C" mgx_status mgx_autotune_load(const char* path) {
    if (!path) return fail(MGX_E_INVALID, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(MGX_E_INVALID, "cannot open %s", path);
    char line[1024];
    int n_bad = 0;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char key[512];
        mgx_launch_shape s;
        std::memset(&s, 0, sizeof s);
        if (std::sscanf(line, "%511s %d %d %d %d %lf %d", key, &s.mode, &s.K, &s.block, &s.grid_per_cu,
                        &s.us_per_chunk, &s.candidates) != 7 ||
            (s.mode != MGX_LAUNCH_PER_CLASS && s.mode != MGX_LAUNCH_PERSISTENT) || s.K < 1 ||
            (s.block != 64 && s.block != 128 && s.block != 256) || s.grid_per_cu < 1 || s.grid_per_cu > 8) {
            ++n_bad;
            continue;
        }
        cache_put(key, s);
    }
    std::fclose(f);
    if (n_bad) return fail(MGX_E_INVALID, "%d malformed line(s) skipped in %s", n_bad, path);
    return MGX_OK;
}
