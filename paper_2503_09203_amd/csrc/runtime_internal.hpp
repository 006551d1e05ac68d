// Host-side batch object shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "kernels.hpp"
#include "mgx.h"

namespace mgx {

extern thread_local std::string g_err;
extern thread_local int32_t g_hip_err;
mgx_status fail(mgx_status s, const char* fmt, ...);

// Makes `dev` current for the scope, restoring the previous device afterwards.
class hipDevice_guard {
   public:
    explicit hipDevice_guard(int dev) {
        e_ = hipGetDevice(&prev_);
        if (e_ == hipSuccess && prev_ != dev) e_ = hipSetDevice(dev);
        if (e_ != hipSuccess) prev_ = -1;
    }
    ~hipDevice_guard() {
        int cur = -1;
        if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return e_ == hipSuccess; }
    hipError_t err() const { return e_; }

   private:
    int prev_ = -1;
    hipError_t e_ = hipSuccess;
};

}  // namespace mgx

struct mgx_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int prec = MGX_FP32;
    double dt = 0.01;
    uint32_t flags = 0;
    int n_classes = 0;
    std::vector<mgx_class_desc> cls;
    int m[MGX_MAX_CLASSES] = {};
    int64_t n[MGX_MAX_CLASSES] = {}, npad[MGX_MAX_CLASSES] = {}, env_off[MGX_MAX_CLASSES] = {},
            pad_off[MGX_MAX_CLASSES] = {}, state_off[MGX_MAX_CLASSES] = {}, rec_off[MGX_MAX_CLASSES] = {},
            act_off[MGX_MAX_CLASSES] = {}, force_off[MGX_MAX_CLASSES] = {}, part_off[MGX_MAX_CLASSES] = {};
    int64_t n_total = 0, npad_total = 0, state_elems = 0, rec_elems = 0, row_elems = 0, force_row_elems = 0,
            max_blocks = 0;

    void* d_state = nullptr;
    void* d_rec = nullptr;
    bool own_state = true, own_rec = true;  // false: adopted from the caller, never freed
    // Device allocator of every buffer the batch allocates (default hipMalloc / hipFree).
    void* (*alloc_fn)(size_t, void*) = nullptr;
    void (*free_fn)(void*, void*) = nullptr;
    void* alloc_ctx = nullptr;
    mgx::DevMisc* d_misc = nullptr;
    mgx::ClassDesc64* d_classdesc = nullptr;
    mgx::ClassT<float>* d_class_f = nullptr;
    mgx::ClassT<double>* d_class_d = nullptr;
    float* d_partials = nullptr;
    double* d_stats = nullptr;
    int64_t* d_ids = nullptr;
    double* d_param_stage = nullptr;
    mgx::ClassT<float> h_class_f[MGX_MAX_CLASSES];
    mgx::ClassT<double> h_class_d[MGX_MAX_CLASSES];

    bool faulted = false;
    bool params_set = false;
    int64_t host_t = 0;
    int slot = 0;  // step-counter slot the next launch reads
    int64_t stats_step = 0;
    int64_t h_t_stage = 0;
    int block = 256;
    int n_graphs = 0;  // live graphs captured from this batch
    int n_stations = 0;  // live station-keeping tasks on this batch
    // launch shape
    int mode = MGX_LAUNCH_PER_CLASS;
    int shape_K = 16;
    int grid_per_cu = 2;
    int n_cu = 256;
    std::string arch;
    // persistent launch: tile table (class, first env), heaviest class first
    int32_t n_tiles = 0;
    int32_t* d_tiles = nullptr;
    mgx::SegDesc* d_segs = nullptr;
    float* d_tile_partials = nullptr;
    // differentiable rollout: checkpoints, segment scratch, and the last forward's arguments
    void* d_ckpt = nullptr;
    void* d_seg = nullptr;
    void* d_tape = nullptr;
    size_t ckpt_bytes = 0, seg_bytes = 0, tape_bytes = 0;
    void* ro_ckpt_mem = nullptr;  // checkpoints and segment scratch of the last forward pass:
    void* ro_seg_mem = nullptr;   // the batch's own buffers, or the static scratch array
    void* ro_tape_mem = nullptr;
    uint64_t ro_static_gen = 0;   // static scratch: the generation the forward pass wrote
    const void* ro_actions = nullptr;
    int64_t ro_n_rows = 0, ro_row0 = 0, ro_t0 = 0;
    int32_t ro_hold = 1, ro_H = 0, ro_ckpt = 32;
    bool ro_valid = false;

    // Allocation through the batch's allocator; *e = hipErrorOutOfMemory when a caller's
    // allocator returns NULL.
    void* dev_alloc(size_t bytes, hipError_t* e) {
        void* p = nullptr;
        if (!bytes) bytes = 16;
        if (alloc_fn) {
            p = alloc_fn(bytes, alloc_ctx);
            *e = p ? hipSuccess : hipErrorOutOfMemory;
        } else {
            *e = hipMalloc(&p, bytes);
        }
        return *e == hipSuccess ? p : nullptr;
    }
    void dev_free(void* p) {
        if (!p) return;
        if (free_fn)
            free_fn(p, alloc_ctx);
        else
            (void)hipFree(p);
    }

    void* seg_state(int c) const { return (char*)d_state + (size_t)prec * state_off[c]; }
    void* seg_rec(int c) const { return (char*)d_rec + (size_t)prec * rec_off[c]; }
    // record rows of class c: the off-diagonal dt M^-1 rows only for a payload class
    int rec_len(int c) const {
        const mgx_class_desc& d = cls[c];
        return (d.rg[0] != 0.0 || d.rg[1] != 0.0 || d.rg[2] != 0.0) ? mgx::kRecLenPayload : mgx::kRecLen;
    }
    int class_of(int64_t gid) const {
        int c = 0;
        while (c + 1 < n_classes && gid >= env_off[c + 1]) ++c;
        return c;
    }
};

namespace mgx {
mgx_status hip_fail(mgx_batch* b, hipError_t e, const char* what);
bool get_class(int32_t id, mgx_class_desc* out);
ClassDesc64 to_desc64(const mgx_class_desc& c);
// Enqueues K steps of every class and flips the counter slot. t_hint: the step count the
// launches are expected to start at when they run (-1 if unknown); any value is correct,
// a matching one saves the single-step launch a dependent memory round trip.
mgx_status enqueue_step(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold, int32_t K,
                        bool stats, void* traj, void* forces, int block, int64_t t_hint);
mgx_status validate_rows(const mgx_batch* b, int64_t t0, int64_t n_rows, int64_t row0, int32_t hold, int64_t K);
// Redraws the parameters of the environments whose byte in `mask` is set, with epochs[e] as
// the draw's epoch (both device arrays of n_pad_total, environment e of class c at
// pad_off[c] + e), as mgx_batch_resample does for listed environments.
mgx_status resample_masked(mgx_batch* b, const mgx_dr_spec* spec, const double* nominal, const uint8_t* mask,
                           const int32_t* epochs, uint64_t seed);
}  // namespace mgx
