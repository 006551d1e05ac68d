// Host runtime of the C ABI declared in include/mgx.h: validation, allocation, layout,
// launches and error state. No torch types; plain pointers and sizes only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"

using namespace mgx;

namespace mgx {
thread_local std::string g_err;
thread_local int32_t g_hip_err = 0;

mgx_status fail(mgx_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

mgx_status hip_fail(mgx_batch* b, hipError_t e, const char* what) {
    g_hip_err = (int32_t)e;
    if (b) b->faulted = true;
    return fail(MGX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static std::mutex g_cls_mu;
static std::vector<mgx_class_desc> g_classes;

bool get_class(int32_t id, mgx_class_desc* out) {
    std::lock_guard<std::mutex> lk(g_cls_mu);
    if (id < 0 || id >= (int32_t)g_classes.size()) return false;
    *out = g_classes[id];
    return true;
}

ClassDesc64 to_desc64(const mgx_class_desc& c) {
    ClassDesc64 d;
    std::memset(&d, 0, sizeof d);
    d.m = c.m;
    std::memcpy(d.r, c.r, sizeof d.r);
    std::memcpy(d.e, c.e, sizeof d.e);
    std::memcpy(d.k, c.k, sizeof d.k);
    std::memcpy(d.tau, c.tau, sizeof d.tau);
    std::memcpy(d.dz, c.deadzone, sizeof d.dz);
    std::memcpy(d.k_rev, c.k_rev, sizeof d.k_rev);
    std::memcpy(d.reaction, c.reaction, sizeof d.reaction);
    std::memcpy(d.kind, c.kind, sizeof d.kind);
    std::memcpy(d.span, c.span, sizeof d.span);
    std::memcpy(d.fin_max, c.fin_max, sizeof d.fin_max);
    std::memcpy(d.fin_lift, c.fin_lift, sizeof d.fin_lift);
    std::memcpy(d.fin_drag0, c.fin_drag0, sizeof d.fin_drag0);
    std::memcpy(d.fin_drag, c.fin_drag, sizeof d.fin_drag);
    std::memcpy(d.rg, c.rg, sizeof d.rg);
    std::memcpy(d.inertia, c.inertia, sizeof d.inertia);
    std::memcpy(d.rb, c.rb, sizeof d.rb);
    d.g0 = c.g0;
    return d;
}
}  // namespace mgx

#define HIP_TRY(b, call)                                             \
    do {                                                             \
        hipError_t e_ = (call);                                      \
        if (e_ != hipSuccess) return mgx::hip_fail((b), e_, #call); \
    } while (0)

#define CHECK_BATCH(b)                                                                                  \
    do {                                                                                                \
        if (!(b)) return fail(MGX_E_INVALID, "batch is NULL");                                          \
        if ((b)->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");         \
    } while (0)

// ----------------------------------------------------------------------------- errors, info

extern "C" const char* mgx_status_string(mgx_status s) {
    switch (s) {
        case MGX_OK: return "ok";
        case MGX_E_INVALID: return "invalid argument";
        case MGX_E_NOMEM: return "out of memory";
        case MGX_E_DEVICE: return "device error";
        case MGX_E_NOT_SPD: return "mass matrix not positive definite";
        case MGX_E_NONFINITE: return "non-finite state";
        case MGX_E_BUDGET: return "memory budget exceeded";
        case MGX_E_STATE: return "invalid state";
        default: return "unknown status";
    }
}

extern "C" size_t mgx_last_error(char* buf, size_t len) {
    if (buf && len) {
        size_t n = g_err.size() < len - 1 ? g_err.size() : len - 1;
        std::memcpy(buf, g_err.data(), n);
        buf[n] = 0;
    }
    return g_err.size();
}

extern "C" int32_t mgx_last_hip_error(void) { return g_hip_err; }
extern "C" int32_t mgx_version(void) { return 100; }

#ifndef MGX_BUILD_HASH
#define MGX_BUILD_HASH "unknown"
#endif
extern "C" const char* mgx_build_hash(void) { return MGX_BUILD_HASH; }

extern "C" mgx_status mgx_device_count(int32_t* count) {
    if (!count) return fail(MGX_E_INVALID, "count is NULL");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        *count = 0;
        g_hip_err = (int32_t)e;
        return fail(MGX_E_DEVICE, "no HIP device visible (%s)", hipGetErrorString(e));
    }
    *count = n;
    return MGX_OK;
}

// ----------------------------------------------------------------------------- classes

static bool is_fin(double x) { return std::isfinite(x); }

extern "C" mgx_status mgx_class_define(const mgx_class_desc* d, int32_t* class_id) {
    if (!d || !class_id) return fail(MGX_E_INVALID, "NULL argument");
    if (d->m < 1 || d->m > MGX_MAX_THRUSTERS) return fail(MGX_E_INVALID, "m=%d outside [1,%d]", d->m, MGX_MAX_THRUSTERS);
    for (int i = 0; i < d->m; ++i) {
        double l2 = 0;
        for (int j = 0; j < 3; ++j) {
            if (!is_fin(d->r[i][j]) || !is_fin(d->e[i][j])) return fail(MGX_E_INVALID, "thruster %d: non-finite r/e", i);
            l2 += d->e[i][j] * d->e[i][j];
        }
        if (!(l2 > 1e-24)) return fail(MGX_E_INVALID, "thruster %d: zero-length axis", i);
        if (d->kind[i] != MGX_ACT_PROPELLER && d->kind[i] != MGX_ACT_FIN)
            return fail(MGX_E_INVALID, "actuator %d: kind must be MGX_ACT_PROPELLER or MGX_ACT_FIN", i);
        if (!(d->tau[i] >= 0) || !is_fin(d->tau[i])) return fail(MGX_E_INVALID, "thruster %d: tau must be >= 0", i);
        if (d->kind[i] == MGX_ACT_FIN) {
            double s2 = 0, es = 0;
            for (int j = 0; j < 3; ++j) {
                if (!is_fin(d->span[i][j])) return fail(MGX_E_INVALID, "fin %d: non-finite span", i);
                s2 += d->span[i][j] * d->span[i][j];
                es += d->e[i][j] * d->span[i][j];
            }
            if (!(s2 > 1e-24)) return fail(MGX_E_INVALID, "fin %d: zero-length span", i);
            if (!(l2 - es * es / s2 > 1e-12 * l2)) return fail(MGX_E_INVALID, "fin %d: chord parallel to the span", i);
            if (!(d->fin_max[i] > 0 && d->fin_max[i] <= 1.5707963267948966))
                return fail(MGX_E_INVALID, "fin %d: fin_max must be in (0, pi/2]", i);
            if (!(d->fin_lift[i] >= 0) || !is_fin(d->fin_lift[i]) || !(d->fin_drag0[i] >= 0) ||
                !is_fin(d->fin_drag0[i]) || !(d->fin_drag[i] >= 0) || !is_fin(d->fin_drag[i]))
                return fail(MGX_E_INVALID, "fin %d: lift and drag gains must be finite and >= 0", i);
            continue;
        }
        if (!(d->k[i] > 0) || !is_fin(d->k[i])) return fail(MGX_E_INVALID, "thruster %d: k must be > 0", i);
        if (!(d->deadzone[i] >= 0 && d->deadzone[i] < 1)) return fail(MGX_E_INVALID, "thruster %d: deadzone in [0,1)", i);
        if (!(d->k_rev[i] >= 0) || !is_fin(d->k_rev[i])) return fail(MGX_E_INVALID, "thruster %d: k_rev must be >= 0", i);
        if (!is_fin(d->reaction[i])) return fail(MGX_E_INVALID, "thruster %d: reaction must be finite", i);
    }
    for (int j = 0; j < 3; ++j) {
        if (!(d->inertia[j] > 0) || !is_fin(d->inertia[j])) return fail(MGX_E_INVALID, "inertia must be > 0");
        if (!is_fin(d->rb[j])) return fail(MGX_E_INVALID, "r_b must be finite");
        if (!is_fin(d->rg[j]) || !(std::fabs(d->rg[j]) < 10.0)) return fail(MGX_E_INVALID, "r_g must be finite and within 10 m");
    }
    if (!(d->g0 > 0) || !is_fin(d->g0)) return fail(MGX_E_INVALID, "g0 must be > 0");
    std::lock_guard<std::mutex> lk(g_cls_mu);
    if (g_classes.size() >= 4096) return fail(MGX_E_INVALID, "too many classes");
    g_classes.push_back(*d);
    *class_id = (int32_t)g_classes.size() - 1;
    return MGX_OK;
}

// ----------------------------------------------------------------------------- batches

static void free_batch_mem(mgx_batch* b) {
    void* ptrs[] = {b->own_state ? b->d_state : nullptr, b->own_rec ? b->d_rec : nullptr, b->d_misc, b->d_classdesc,
                    b->d_class_f, b->d_class_d, b->d_partials, b->d_stats, b->d_ids, b->d_param_stage, b->d_tiles,
                    b->d_segs, b->d_tile_partials, b->d_ckpt, b->d_seg, b->d_tape};
    for (void* p : ptrs) b->dev_free(p);
}

// Validates a batch description and fills the layout of the batch it describes (no device
// work). rec_elems receives the parameter-record size in elements.
static mgx_status plan_batch(const mgx_batch_desc* d, std::vector<mgx_class_desc>* cls_out, mgx_batch* b) {
    if (d->n_classes < 1 || d->n_classes > MGX_MAX_CLASSES)
        return fail(MGX_E_INVALID, "n_classes=%d outside [1,%d]", d->n_classes, MGX_MAX_CLASSES);
    if (d->precision != MGX_FP32 && d->precision != MGX_FP64) return fail(MGX_E_INVALID, "precision must be 4 or 8");
    if (!d->class_ids || !d->n_envs) return fail(MGX_E_INVALID, "class_ids / n_envs NULL");
    if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(MGX_E_INVALID, "dt must be > 0");
    if (d->flags & ~(MGX_FLAG_NO_AMC | MGX_FLAG_LAG_EULER)) return fail(MGX_E_INVALID, "unknown batch flag");
    if ((d->alloc == nullptr) != (d->free == nullptr)) return fail(MGX_E_INVALID, "alloc and free: both or neither");
    std::vector<mgx_class_desc> cls(d->n_classes);
    for (int c = 0; c < d->n_classes; ++c) {
        if (!get_class(d->class_ids[c], &cls[c])) return fail(MGX_E_INVALID, "class id %d unknown", d->class_ids[c]);
        if (d->n_envs[c] < 1 || d->n_envs[c] > (int64_t)1 << 30)
            return fail(MGX_E_INVALID, "n_envs[%d]=%lld outside [1, 2^30]", c, (long long)d->n_envs[c]);
    }
    b->prec = d->precision;
    b->dt = d->dt;
    b->flags = d->flags;
    b->n_classes = d->n_classes;
    b->cls = cls;
    int64_t soff = 0, aoff = 0, foff = 0, eoff = 0, poff = 0, roff = 0, max_blocks = 0;
    for (int c = 0; c < d->n_classes; ++c) {
        const int m = cls[c].m;
        const int64_t n = d->n_envs[c], np = (n + kWave - 1) / kWave * kWave;
        b->m[c] = m;
        b->n[c] = n;
        b->npad[c] = np;
        b->env_off[c] = eoff;
        b->pad_off[c] = poff;
        b->state_off[c] = soff;
        b->rec_off[c] = roff;
        b->act_off[c] = aoff;
        b->force_off[c] = foff;
        b->part_off[c] = max_blocks * kStats;
        eoff += n;
        poff += np;
        soff += (kStateFixed + m) * np;
        roff += (int64_t)b->rec_len(c) * np;
        aoff += (int64_t)m * np;
        foff += (int64_t)kForceLen * np;
        max_blocks += np / kWave;
    }
    b->n_total = eoff;
    b->npad_total = poff;
    b->state_elems = soff;
    b->rec_elems = roff;
    b->row_elems = aoff;
    b->force_row_elems = foff;
    b->max_blocks = max_blocks;
    if (cls_out) *cls_out = cls;
    return MGX_OK;
}

static void fill_layout(const mgx_batch* b, mgx_layout* out) {
    std::memset(out, 0, sizeof *out);
    out->n_classes = b->n_classes;
    out->precision = b->prec;
    out->n_total = b->n_total;
    out->n_pad_total = b->npad_total;
    out->state_elems = b->state_elems;
    out->row_elems = b->row_elems;
    out->force_row_elems = b->force_row_elems;
    out->record_elems = b->rec_elems;
    for (int c = 0; c < b->n_classes; ++c) {
        out->m[c] = b->m[c];
        out->n[c] = b->n[c];
        out->n_pad[c] = b->npad[c];
        out->env_off[c] = b->env_off[c];
        out->state_off[c] = b->state_off[c];
        out->action_off[c] = b->act_off[c];
        out->force_off[c] = b->force_off[c];
        out->record_off[c] = b->rec_off[c];
    }
}

extern "C" mgx_status mgx_batch_plan(const mgx_batch_desc* d, mgx_layout* out) {
    if (!d || !out) return fail(MGX_E_INVALID, "NULL argument");
    mgx_batch tmp;
    mgx_status st = plan_batch(d, nullptr, &tmp);
    if (st != MGX_OK) return st;
    fill_layout(&tmp, out);
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_create(const mgx_batch_desc* d, mgx_batch** out) {
    if (!d || !out) return fail(MGX_E_INVALID, "NULL argument");
    *out = nullptr;
    mgx_batch* b = new (std::nothrow) mgx_batch();
    if (!b) return fail(MGX_E_NOMEM, "host allocation");
    std::vector<mgx_class_desc> cls;
    {
        mgx_status st = plan_batch(d, &cls, b);
        if (st != MGX_OK) {
            delete b;
            return st;
        }
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        delete b;
        g_hip_err = (int32_t)e;
        return fail(MGX_E_DEVICE, "no HIP device visible");
    }
    int dev = d->device;
    if (dev < 0) {
        e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete b;
            return hip_fail(nullptr, e, "hipGetDevice");
        }
    }
    if (dev >= ndev) {
        delete b;
        return fail(MGX_E_INVALID, "device %d of %d", dev, ndev);
    }
    b->device = dev;
    b->stream = (hipStream_t)d->stream;
    b->alloc_fn = d->alloc;
    b->free_fn = d->free;
    b->alloc_ctx = d->alloc_ctx;
    const int64_t max_blocks = b->max_blocks;

    hipDevice_guard g(dev);
    if (!g.ok()) {
        delete b;
        return hip_fail(nullptr, g.err(), "hipSetDevice");
    }
    const size_t P = (size_t)b->prec;
    e = hipSuccess;
    if (d->state) {
        b->d_state = d->state;
        b->own_state = false;
    } else {
        b->d_state = b->dev_alloc(P * b->state_elems, &e);
    }
    if (e == hipSuccess && d->record) {
        b->d_rec = d->record;
        b->own_rec = false;
    } else if (e == hipSuccess) {
        b->d_rec = b->dev_alloc(P * b->rec_elems, &e);
    }
    if (e == hipSuccess) b->d_misc = (DevMisc*)b->dev_alloc(sizeof(DevMisc), &e);
    if (e == hipSuccess) b->d_classdesc = (ClassDesc64*)b->dev_alloc(sizeof(ClassDesc64) * MGX_MAX_CLASSES, &e);
    if (e == hipSuccess) b->d_class_f = (ClassT<float>*)b->dev_alloc(sizeof(ClassT<float>) * MGX_MAX_CLASSES, &e);
    if (e == hipSuccess) b->d_class_d = (ClassT<double>*)b->dev_alloc(sizeof(ClassT<double>) * MGX_MAX_CLASSES, &e);
    if (e == hipSuccess) b->d_partials = (float*)b->dev_alloc(sizeof(float) * kStats * max_blocks, &e);
    if (e == hipSuccess) b->d_stats = (double*)b->dev_alloc(sizeof(double) * kStats * MGX_MAX_CLASSES, &e);
    if (e == hipSuccess) b->d_ids = (int64_t*)b->dev_alloc(sizeof(int64_t) * b->n_total, &e);
    b->n_tiles = (int32_t)(b->npad_total / kWave);
    if (e == hipSuccess) b->d_tiles = (int32_t*)b->dev_alloc(sizeof(int32_t) * 2 * b->n_tiles, &e);
    if (e == hipSuccess) b->d_segs = (SegDesc*)b->dev_alloc(sizeof(SegDesc) * MGX_MAX_CLASSES, &e);
    if (e == hipSuccess) b->d_tile_partials = (float*)b->dev_alloc(sizeof(float) * kStats * b->n_tiles, &e);
    if (e != hipSuccess) {
        free_batch_mem(b);
        delete b;
        g_hip_err = (int32_t)e;
        return fail(e == hipErrorOutOfMemory ? MGX_E_NOMEM : MGX_E_DEVICE, "device allocation: %s",
                    hipGetErrorString(e));
    }
    // Class constants in double on the device, then fetched back: they travel to the step
    // kernels as kernel arguments (scalar registers).
    std::vector<ClassDesc64> d64(MGX_MAX_CLASSES);
    for (int c = 0; c < b->n_classes; ++c) d64[c] = to_desc64(cls[c]);
    // Persistent launch: tiles of 64 environments, heaviest class (most thrusters) first.
    std::vector<int32_t> tiles;
    std::vector<int> order(b->n_classes);
    for (int c = 0; c < b->n_classes; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->m[x] > b->m[y]; });
    for (int c : order)
        for (int64_t e0 = 0; e0 < b->npad[c]; e0 += kWave) {
            tiles.push_back(c);
            tiles.push_back((int32_t)e0);
        }
    std::vector<SegDesc> segs(MGX_MAX_CLASSES);
    for (int c = 0; c < b->n_classes; ++c) {
        segs[c].state = b->seg_state(c);
        segs[c].rec = b->seg_rec(c);
        segs[c].act_off = b->act_off[c];
        segs[c].npad = (int32_t)b->npad[c];
        segs[c].nvalid = (int32_t)b->n[c];
        segs[c].m = b->m[c];
        segs[c].shaped = shaped_thrust(d64[c]) ? 1 : 0;
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            b->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
            b->arch = prop.gcnArchName;
        }
    }
    // Default block: one wave per block while the batch has fewer waves than the device has
    // SIMDs (four per compute unit), so that a small batch spreads over as many compute units
    // instead of sharing a quarter as many (1024 environments x 1000 steps in FP64: 1.31 ->
    // 1.23 ms); blocks of four waves from one wave per SIMD on.
    b->block = b->npad_total / kWave < 4 * (int64_t)b->n_cu ? kWave : 256;
    mgx_status st = MGX_OK;
    auto run = [&]() -> mgx_status {
        HIP_TRY(b, hipMemcpyAsync(b->d_classdesc, d64.data(), sizeof(ClassDesc64) * MGX_MAX_CLASSES,
                                  hipMemcpyHostToDevice, b->stream));
        HIP_TRY(b, launch_class_setup(b->d_classdesc, b->d_class_f, b->d_class_d, b->n_classes, b->dt, b->flags,
                                      b->stream));
        HIP_TRY(b, hipMemcpyAsync(b->h_class_f, b->d_class_f, sizeof(ClassT<float>) * MGX_MAX_CLASSES,
                                  hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(b, hipMemcpyAsync(b->h_class_d, b->d_class_d, sizeof(ClassT<double>) * MGX_MAX_CLASSES,
                                  hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(b, hipMemsetAsync(b->d_misc, 0, sizeof(DevMisc), b->stream));
        HIP_TRY(b, hipMemcpyAsync(b->d_tiles, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice,
                                  b->stream));
        HIP_TRY(b, hipMemcpyAsync(b->d_segs, segs.data(), sizeof(SegDesc) * MGX_MAX_CLASSES, hipMemcpyHostToDevice,
                                  b->stream));
        HIP_TRY(b, hipMemsetAsync(b->d_stats, 0, sizeof(double) * kStats * MGX_MAX_CLASSES, b->stream));
        for (int c = 0; c < b->n_classes; ++c) {
            if (b->prec == MGX_FP32) {
                // an adopted state keeps its valid slots; padded slots are always set to rest
                HIP_TRY(b, launch_init_padding<float>((float*)b->seg_state(c), (float*)b->seg_rec(c), b->m[c],
                                                      (int32_t)b->npad[c], b->own_state ? 0 : b->n[c], b->stream,
                                                      b->rec_len(c)));
            } else {
                HIP_TRY(b, launch_init_padding<double>((double*)b->seg_state(c), (double*)b->seg_rec(c), b->m[c],
                                                       (int32_t)b->npad[c], b->own_state ? 0 : b->n[c], b->stream,
                                                       b->rec_len(c)));
            }
        }
        HIP_TRY(b, hipStreamSynchronize(b->stream));
        return MGX_OK;
    };
    st = run();
    if (st != MGX_OK) {
        free_batch_mem(b);
        delete b;
        return st;
    }
    *out = b;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_destroy(mgx_batch* b) {
    if (!b) return MGX_OK;
    if (b->n_graphs > 0) return fail(MGX_E_STATE, "destroy the %d graph(s) of this batch first", b->n_graphs);
    if (b->n_stations > 0)
        return fail(MGX_E_STATE, "destroy the %d station task(s) of this batch first", b->n_stations);
    hipDevice_guard g(b->device);
    (void)hipStreamSynchronize(b->stream);
    free_batch_mem(b);
    delete b;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_layout(const mgx_batch* b, mgx_layout* out) {
    if (!b || !out) return fail(MGX_E_INVALID, "NULL argument");
    fill_layout(b, out);
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_set_params(mgx_batch* b, const mgx_env_params* p, int32_t on_device) {
    CHECK_BATCH(b);
    if (on_device < 0 || on_device > 2) return fail(MGX_E_INVALID, "on_device must be 0, 1 or 2");
    if (!p || !p->mass || !p->added || !p->dlin || !p->dquad || !p->buoy || !p->current)
        return fail(MGX_E_INVALID, "NULL parameter array");
    const int64_t N = b->n_total;
    hipDevice_guard g(b->device);
    ParamPtrs pp;
    pp.n_total = N;
    if (on_device) {
        pp.mass = p->mass;
        pp.added = p->added;
        pp.dlin = p->dlin;
        pp.dquad = p->dquad;
        pp.buoy = p->buoy;
        pp.current = p->current;
    } else {
        for (int64_t i = 0; i < N; ++i) {
            if (!(p->mass[i] > 0) || !is_fin(p->mass[i])) return fail(MGX_E_INVALID, "mass[%lld] must be > 0", (long long)i);
            if (!(p->buoy[i] >= 0) || !is_fin(p->buoy[i])) return fail(MGX_E_INVALID, "buoy[%lld] must be >= 0", (long long)i);
            for (int j = 0; j < 6; ++j) {
                const double a = p->added[j * N + i], l = p->dlin[j * N + i], q = p->dquad[j * N + i];
                if (!(l >= 0 && q >= 0) || !is_fin(a) || !is_fin(l) || !is_fin(q))
                    return fail(MGX_E_INVALID, "added[%d][%lld] must be finite, dlin/dquad finite and >= 0", j,
                                (long long)i);
            }
            for (int j = 0; j < 3; ++j)
                if (!is_fin(p->current[j * N + i])) return fail(MGX_E_INVALID, "current must be finite");
        }
        if (!b->d_param_stage) {
            hipError_t e;
            b->d_param_stage = (double*)b->dev_alloc(sizeof(double) * 23 * N, &e);
            if (!b->d_param_stage) return hip_fail(nullptr, e, "hipMalloc(param stage)");
        }
        double* s = b->d_param_stage;
        // Synchronous copies: the host arrays may be released as soon as this call returns.
        HIP_TRY(b, hipMemcpy(s, p->mass, sizeof(double) * N, hipMemcpyHostToDevice));
        HIP_TRY(b, hipMemcpy(s + N, p->added, sizeof(double) * 6 * N, hipMemcpyHostToDevice));
        HIP_TRY(b, hipMemcpy(s + 7 * N, p->dlin, sizeof(double) * 6 * N, hipMemcpyHostToDevice));
        HIP_TRY(b, hipMemcpy(s + 13 * N, p->dquad, sizeof(double) * 6 * N, hipMemcpyHostToDevice));
        HIP_TRY(b, hipMemcpy(s + 19 * N, p->buoy, sizeof(double) * N, hipMemcpyHostToDevice));
        HIP_TRY(b, hipMemcpy(s + 20 * N, p->current, sizeof(double) * 3 * N, hipMemcpyHostToDevice));
        pp.mass = s;
        pp.added = s + N;
        pp.dlin = s + 7 * N;
        pp.dquad = s + 13 * N;
        pp.buoy = s + 19 * N;
        pp.current = s + 20 * N;
    }
    if (on_device == 2) {
        // unchecked device arrays: the record build alone, asynchronous; invalid values reach
        // the batch's error word (mgx_batch_check) and NaN records
        for (int c = 0; c < b->n_classes; ++c) {
            if (b->prec == MGX_FP32) {
                HIP_TRY(b, launch_env_setup<float>(pp, b->env_off[c], b->n[c], (int32_t)b->npad[c], b->d_classdesc, c,
                                                   b->dt, (float*)b->seg_rec(c), &b->d_misc->err, b->stream));
            } else {
                HIP_TRY(b, launch_env_setup<double>(pp, b->env_off[c], b->n[c], (int32_t)b->npad[c], b->d_classdesc,
                                                    c, b->dt, (double*)b->seg_rec(c), &b->d_misc->err, b->stream));
            }
        }
        b->params_set = true;
        return MGX_OK;
    }
    // Every environment's values and mass matrix are checked on the device before any
    // record is written, so a refused call leaves the batch unchanged. The check word is
    // cleared by a one-thread kernel rather than a memset node.
    HIP_TRY(b, launch_clear_word(&b->d_misc->check, b->stream));
    for (int c = 0; c < b->n_classes; ++c)
        HIP_TRY(b, launch_check_params(pp, b->env_off[c], b->n[c], b->d_classdesc, c, &b->d_misc->check, b->stream));
    int32_t chk = 0;
    HIP_TRY(b, hipMemcpyAsync(&chk, &b->d_misc->check, sizeof chk, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    if (chk & kErrParam)
        return fail(MGX_E_INVALID, "a device parameter is not finite or out of range (mass > 0; damping, buoyancy >= 0)");
    if (chk & kErrNotSpd) return fail(MGX_E_NOT_SPD, "M_RB + M_A of some environment is not positive definite");
    for (int c = 0; c < b->n_classes; ++c) {
        if (b->prec == MGX_FP32) {
            HIP_TRY(b, launch_env_setup<float>(pp, b->env_off[c], b->n[c], (int32_t)b->npad[c], b->d_classdesc, c, b->dt,
                                               (float*)b->seg_rec(c), &b->d_misc->err, b->stream));
        } else {
            HIP_TRY(b, launch_env_setup<double>(pp, b->env_off[c], b->n[c], (int32_t)b->npad[c], b->d_classdesc, c,
                                                b->dt, (double*)b->seg_rec(c), &b->d_misc->err, b->stream));
        }
    }
    b->params_set = true;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_reset(mgx_batch* b, const int64_t* env_ids, int64_t n, const void* init_state,
                                      uint64_t seed) {
    CHECK_BATCH(b);
    if (env_ids && (n < 0 || n > b->n_total)) return fail(MGX_E_INVALID, "n=%lld outside [0, n_total]", (long long)n);
    hipDevice_guard g(b->device);
    // Split the id list by class into local ids (host), then upload once.
    std::vector<int64_t> local;
    std::vector<int64_t> cnt(b->n_classes, 0), start(b->n_classes, 0);
    if (env_ids) {
        std::vector<std::vector<int64_t>> per(b->n_classes);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t gid = env_ids[i];
            if (gid < 0 || gid >= b->n_total) return fail(MGX_E_INVALID, "env id %lld out of range", (long long)gid);
            int c = b->class_of(gid);
            per[c].push_back(gid - b->env_off[c]);
        }
        for (int c = 0; c < b->n_classes; ++c) {
            start[c] = (int64_t)local.size();
            cnt[c] = (int64_t)per[c].size();
            local.insert(local.end(), per[c].begin(), per[c].end());
        }
        if (!local.empty())
            HIP_TRY(b, hipMemcpy(b->d_ids, local.data(), sizeof(int64_t) * local.size(), hipMemcpyHostToDevice));
    }
    for (int c = 0; c < b->n_classes; ++c) {
        const int64_t* ids = env_ids ? b->d_ids + start[c] : nullptr;
        const int64_t nid = env_ids ? cnt[c] : b->n[c];
        if (nid == 0) continue;
        if (b->prec == MGX_FP32) {
            if (init_state) {
                HIP_TRY(b, launch_reset_copy<float>((float*)b->seg_state(c), (const float*)init_state + b->state_off[c],
                                                    b->m[c], (int32_t)b->npad[c], ids, nid, b->stream));
            } else {
                HIP_TRY(b, launch_reset_seeded<float>((float*)b->seg_state(c), b->m[c], (int32_t)b->npad[c], b->env_off[c],
                                                      b->n[c], ids, nid, seed, b->stream));
            }
        } else {
            if (init_state) {
                HIP_TRY(b, launch_reset_copy<double>((double*)b->seg_state(c),
                                                     (const double*)init_state + b->state_off[c], b->m[c],
                                                     (int32_t)b->npad[c], ids, nid, b->stream));
            } else {
                HIP_TRY(b, launch_reset_seeded<double>((double*)b->seg_state(c), b->m[c], (int32_t)b->npad[c],
                                                       b->env_off[c], b->n[c], ids, nid, seed, b->stream));
            }
        }
    }
    return MGX_OK;
}

static int64_t floor_div_h(int64_t a, int64_t b) {
    int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

namespace mgx {
// Enqueues K steps of every class; `advance` of the last class launch moves the counter.
mgx_status enqueue_step(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold, int32_t K,
                        bool stats, void* traj, void* forces, int block, int64_t t_hint) {
    const size_t P = (size_t)b->prec;
    bool fins = false;
    for (int c = 0; c < b->n_classes; ++c) fins = fins || b->h_class_f[c].fin_mask != 0 || b->h_class_f[c].payload != 0;
    // classes with fins or a payload run their own k_step instantiations; the persistent
    // kernel holds the plain and shaped propeller bodies only
    if (b->mode == MGX_LAUNCH_PERSISTENT && !traj && !forces && b->prec == MGX_FP32 && !fins) {
        PersistArgs pa;
        std::memset(&pa, 0, sizeof pa);
        pa.segs = b->d_segs;
        pa.cls = b->d_class_f;
        pa.tiles = b->d_tiles;
        pa.n_classes = b->n_classes;
        pa.n_tiles = b->n_tiles;
        pa.actions = actions;
        pa.row_stride = b->row_elems;
        pa.n_rows = n_rows;
        pa.row0 = row0;
        pa.hold = hold;
        pa.K = K;
        pa.misc = b->d_misc;
        pa.rd = b->slot;
        pa.wr = 1 - b->slot;
        pa.advance = K;
        pa.tile_partials = stats ? b->d_tile_partials : nullptr;
        pa.stats = b->d_stats;
        for (int c = 0; c < b->n_classes; ++c) pa.any_shaped |= b->h_class_f[c].shaped != 0 ? 1 : 0;
        const int waves_per_block = block / kWave;
        int grid = b->n_cu * b->grid_per_cu;
        const int needed = (b->n_tiles + waves_per_block - 1) / waves_per_block;
        if (grid > needed) grid = needed;
        if (grid < 1) grid = 1;
        hipError_t e = launch_persistent<float>(pa, grid, block, b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "persistent launch");
        b->slot = 1 - b->slot;
        return MGX_OK;
    }
    for (int c = 0; c < b->n_classes; ++c) {
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.state = b->seg_state(c);
        a.rec = b->seg_rec(c);
        a.actions = (const char*)actions + P * b->act_off[c];
        a.row_stride = b->row_elems;
        a.n_rows = n_rows;
        a.row0 = row0;
        a.hold = hold;
        a.K = K;
        a.npad = (int32_t)b->npad[c];
        a.nvalid = (int32_t)b->n[c];
        a.misc = b->d_misc;
        a.class_index = c;
        a.advance = (c == b->n_classes - 1) ? K : 0;
        a.rd = b->slot;
        a.wr = 1 - b->slot;
        // a hint whose row lies outside the buffer is dropped: the launch then finds (and
        // reports) the row the device counter names
        const int64_t rh = t_hint >= 0 ? floor_div_h(t_hint, hold) - row0 : -1;
        const bool hint = t_hint >= 0 && rh >= 0 && rh < n_rows;
        a.t_hint = hint ? t_hint : -1;
        a.row_hint = hint ? rh : 0;
        a.traj = traj ? (char*)traj + P * b->state_off[c] : nullptr;
        a.traj_stride = b->state_elems;
        a.forces = forces ? (char*)forces + P * b->force_off[c] : nullptr;
        a.force_stride = b->force_row_elems;
        a.partials = stats ? b->d_partials + b->part_off[c] : nullptr;
        a.stats = b->d_stats + (int64_t)kStats * c;
        hipError_t e;
        if (b->prec == MGX_FP32) {
            StepLaunch<float> L{a, b->h_class_f[c]};
            e = launch_step<float>(L, b->m[c], block, b->stream);
        } else {
            StepLaunch<double> L{a, b->h_class_d[c]};
            e = launch_step<double>(L, b->m[c], block, b->stream);
        }
        if (e != hipSuccess) return hip_fail(b, e, "step launch");
    }
    b->slot = 1 - b->slot;
    return MGX_OK;
}

mgx_status validate_rows(const mgx_batch* b, int64_t t0, int64_t n_rows, int64_t row0, int32_t hold, int64_t K) {
    const int64_t first = floor_div_h(t0, hold) - row0, last = floor_div_h(t0 + K - 1, hold) - row0;
    if (first < 0 || last >= n_rows)
        return fail(MGX_E_INVALID, "steps %lld..%lld need action rows %lld..%lld; buffer has [0, %lld)",
                    (long long)t0, (long long)(t0 + K - 1), (long long)first, (long long)last, (long long)n_rows);
    return MGX_OK;
}
}  // namespace mgx

extern "C" mgx_status mgx_batch_step(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                     int32_t K, uint32_t flags, void* traj, void* forces) {
    CHECK_BATCH(b);
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params has not been called");
    if (!actions) return fail(MGX_E_INVALID, "actions is NULL");
    if (K == 0) K = b->shape_K;
    if (K < 1) return fail(MGX_E_INVALID, "K=%d must be >= 1 (or 0)", K);
    if (hold < 1) return fail(MGX_E_INVALID, "hold=%d must be >= 1", hold);
    if (n_rows < 1) return fail(MGX_E_INVALID, "n_rows must be >= 1");
    if (flags & ~(MGX_STEP_UNFUSED | MGX_STEP_STATS)) return fail(MGX_E_INVALID, "unknown step flag");
    mgx_status v = validate_rows(b, b->host_t, n_rows, row0, hold, K);
    if (v != MGX_OK) return v;
    hipDevice_guard g(b->device);
    const bool stats = (flags & MGX_STEP_STATS) != 0;
    if (flags & MGX_STEP_UNFUSED) {
        const size_t P = (size_t)b->prec;
        for (int32_t k = 0; k < K; ++k) {
            mgx_status s = enqueue_step(b, actions, n_rows, row0, hold, 1, stats && k == K - 1,
                                        traj ? (char*)traj + P * k * b->state_elems : nullptr,
                                        forces ? (char*)forces + P * k * b->force_row_elems : nullptr, b->block,
                                        b->host_t + k);
            if (s != MGX_OK) return s;
        }
    } else {
        mgx_status s = enqueue_step(b, actions, n_rows, row0, hold, K, stats, traj, forces, b->block, b->host_t);
        if (s != MGX_OK) return s;
    }
    b->host_t += K;
    if (stats) b->stats_step = b->host_t;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_get_step(const mgx_batch* b, int64_t* t) {
    if (!b || !t) return fail(MGX_E_INVALID, "NULL argument");
    *t = b->host_t;
    return MGX_OK;
}

extern "C" mgx_status mgx_diag_set_device_step(mgx_batch* b, int64_t t) {
    CHECK_BATCH(b);
    if (t < 0) return fail(MGX_E_INVALID, "t must be >= 0");
    hipDevice_guard g(b->device);
    HIP_TRY(b, launch_set_counter(b->d_misc, b->slot, t, b->stream));
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_set_step(mgx_batch* b, int64_t t) {
    CHECK_BATCH(b);
    if (t < 0) return fail(MGX_E_INVALID, "t must be >= 0");
    hipDevice_guard g(b->device);
    HIP_TRY(b, launch_set_counter(b->d_misc, b->slot, t, b->stream));
    b->host_t = t;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_get_state(mgx_batch* b, void* out, int32_t to_host) {
    CHECK_BATCH(b);
    if (!out) return fail(MGX_E_INVALID, "out is NULL");
    hipDevice_guard g(b->device);
    const size_t bytes = (size_t)b->prec * b->state_elems;
    HIP_TRY(b, hipMemcpyAsync(out, b->d_state, bytes, to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                              b->stream));
    if (to_host) HIP_TRY(b, hipStreamSynchronize(b->stream));
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_set_state(mgx_batch* b, const void* in, int32_t from_host) {
    CHECK_BATCH(b);
    if (!in) return fail(MGX_E_INVALID, "in is NULL");
    hipDevice_guard g(b->device);
    const size_t bytes = (size_t)b->prec * b->state_elems;
    if (from_host) {
        HIP_TRY(b, hipMemcpyAsync(b->d_state, in, bytes, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(b, hipStreamSynchronize(b->stream));
    } else {
        HIP_TRY(b, hipMemcpyAsync(b->d_state, in, bytes, hipMemcpyDeviceToDevice, b->stream));
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_sync(mgx_batch* b) {
    CHECK_BATCH(b);
    hipDevice_guard g(b->device);
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_get_stats(mgx_batch* b, mgx_stats* out) {
    CHECK_BATCH(b);
    if (!out) return fail(MGX_E_INVALID, "out is NULL");
    hipDevice_guard g(b->device);
    double h[kStats * MGX_MAX_CLASSES];
    HIP_TRY(b, hipMemcpyAsync(h, b->d_stats, sizeof h, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    std::memset(out, 0, sizeof *out);
    out->step = b->stats_step;
    for (int c = 0; c < b->n_classes; ++c) {
        const double* s = h + kStats * c;
        const double nv = (double)b->n[c] - s[kStNonFinite];
        out->n_nonfinite[c] = (int64_t)s[kStNonFinite];
        out->n_renorm64[c] = (int64_t)s[kStRenorm];
        out->max_speed[c] = s[kStMaxSpeed];
        out->max_rate[c] = s[kStMaxRate];
        out->max_qdrift[c] = s[kStMaxDrift];
        out->mean_speed[c] = nv > 0 ? s[kStSumSpeed] / nv : 0.0;
        out->mean_rate[c] = nv > 0 ? s[kStSumRate] / nv : 0.0;
        out->mean_kinetic[c] = nv > 0 ? s[kStSumKin] / nv : 0.0;
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_check(mgx_batch* b, int64_t* n_nonfinite) {
    CHECK_BATCH(b);
    hipDevice_guard g(b->device);
    DevMisc m;
    double h[kStats * MGX_MAX_CLASSES];
    HIP_TRY(b, hipMemcpyAsync(&m, b->d_misc, sizeof m, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipMemcpyAsync(h, b->d_stats, sizeof h, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    int64_t nf = 0;
    for (int c = 0; c < b->n_classes; ++c) nf += (int64_t)h[kStats * c + kStNonFinite];
    if (n_nonfinite) *n_nonfinite = nf;
    if (m.err & kErrNotSpd)
        return fail(MGX_E_NOT_SPD, "a parameter record was built from a mass matrix that is not positive definite");
    if (m.err & kErrParam) return fail(MGX_E_INVALID, "a parameter record was built from an invalid value");
    if (m.err) return fail(MGX_E_INVALID, "a kernel met an action row outside its buffer (err=%d)", m.err);
    if (nf) return fail(MGX_E_NONFINITE, "%lld environments hold non-finite values", (long long)nf);
    return MGX_OK;
}

extern "C" mgx_status mgx_gen_actions(mgx_batch* b, void* out, int64_t rows, int64_t row_offset, uint64_t seed) {
    CHECK_BATCH(b);
    if (!out) return fail(MGX_E_INVALID, "out is NULL");
    if (rows < 1 || rows > 65535) return fail(MGX_E_INVALID, "rows=%lld outside [1, 65535]", (long long)rows);
    if (row_offset < 0) return fail(MGX_E_INVALID, "row_offset must be >= 0");
    hipDevice_guard g(b->device);
    const size_t P = (size_t)b->prec;
    for (int c = 0; c < b->n_classes; ++c) {
        hipError_t e;
        if (b->prec == MGX_FP32)
            e = launch_gen_actions<float>((float*)((char*)out + P * b->act_off[c]), b->m[c], (int32_t)b->npad[c], b->n[c],
                                          b->env_off[c], rows, b->row_elems, row_offset, seed, b->stream);
        else
            e = launch_gen_actions<double>((double*)((char*)out + P * b->act_off[c]), b->m[c], (int32_t)b->npad[c],
                                           b->n[c], b->env_off[c], rows, b->row_elems, row_offset, seed, b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "gen_actions launch");
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_get_shape(const mgx_batch* b, mgx_launch_shape* out) {
    if (!b || !out) return fail(MGX_E_INVALID, "NULL argument");
    std::memset(out, 0, sizeof *out);
    out->mode = b->mode;
    out->K = b->shape_K;
    out->block = b->block;
    out->grid_per_cu = b->grid_per_cu;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_set_shape(mgx_batch* b, const mgx_launch_shape* in) {
    CHECK_BATCH(b);
    if (!in) return fail(MGX_E_INVALID, "NULL argument");
    if (in->mode != MGX_LAUNCH_PER_CLASS && in->mode != MGX_LAUNCH_PERSISTENT) return fail(MGX_E_INVALID, "unknown mode");
    if (in->mode == MGX_LAUNCH_PERSISTENT && b->prec != MGX_FP32)
        return fail(MGX_E_INVALID, "the persistent launch is for float batches");
    if (in->K < 1 || in->K > 65536) return fail(MGX_E_INVALID, "K=%d outside [1, 65536]", in->K);
    if (in->block != 64 && in->block != 128 && in->block != 256) return fail(MGX_E_INVALID, "block must be 64, 128 or 256");
    if (in->grid_per_cu < 1 || in->grid_per_cu > 8) return fail(MGX_E_INVALID, "grid_per_cu outside [1, 8]");
    b->mode = in->mode;
    b->shape_K = in->K;
    b->block = in->block;
    b->grid_per_cu = in->grid_per_cu;
    return MGX_OK;
}
