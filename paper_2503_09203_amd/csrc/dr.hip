// On-device domain randomisation (Sec. III-C): per-environment parameters drawn from
// uniform, Gaussian or piecewise distributions for chosen environments, then the record
// rebuilt from them in double, as the parameter setup does.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "env_loop.hpp"
#include "kernels.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"

namespace mgx {

constexpr uint32_t kStreamDr = 7u;

struct DrNominal {
    double v[23];  // mass, added[6], dlin[6], dquad[6], buoyancy, current[3]
};

// One draw of a distribution from a pair of uniforms.
__device__ double dr_draw(const mgx_dr_dist& d, double u1, double u2) {
    if (d.kind == MGX_DR_UNIFORM) return d.lo + (d.hi - d.lo) * u1;
    if (d.kind == MGX_DR_GAUSSIAN) {
        const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
        return fmin(fmax(d.mean + d.std * z, d.lo), d.hi);
    }
    // piecewise: invert the running sums of the bin weights
    double S[MGX_DR_MAX_BINS + 1];
    S[0] = 0.0;
    int last = 0;
    for (int k = 0; k < d.n_bins; ++k) {
        S[k + 1] = S[k] + d.weights[k];
        if (d.weights[k] > 0.0) last = k;
    }
    const double t = u1 * S[d.n_bins];
    int k = last;
    for (int j = 0; j < d.n_bins; ++j)
        if (t < S[j + 1]) {
            k = j;
            break;
        }
    return fmin(d.edges[k] + (t - S[k]) / d.weights[k] * (d.edges[k + 1] - d.edges[k]), d.edges[k + 1]);
}

// Values of one group (size entries starting at nominal offset off, uniform pairs from
// slot) into out.
__device__ void dr_group(const mgx_dr_dist& d, const double* nom, const double* u, int slot, int size, double* out) {
    for (int i = 0; i < size; ++i) {
        if (d.kind == MGX_DR_FIXED) {
            out[i] = nom[i];
            continue;
        }
        const int s = d.shared ? slot : slot + 2 * i;
        const double x = dr_draw(d, u[s], u[s + 1]);
        out[i] = d.relative ? nom[i] * x : x;
    }
}

// The per-lane draw of environment e (its 23 generator calls in sequence) and its record.
template <typename T>
__device__ void dr_resample_one(const mgx_dr_spec& spec, const DrNominal& nom, const ClassDesc64& cls, double dt,
                                T* rec, int64_t npad, int64_t env_off, int64_t e, uint64_t seed, uint64_t epoch,
                                int32_t* err) {
    const uint64_t g = (uint64_t)(env_off + e);
    double u[46];
    for (int j = 0; j < 23; ++j) {
        uint32_t c[4] = {(uint32_t)g, (uint32_t)epoch, (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)seed, kStreamDr << 24);
        u[2 * j] = u53(c[0], c[1]);
        u[2 * j + 1] = u53(c[2], c[3]);
    }
    double mass, added[6], dlin[6], dquad[6], buoy, cur[3];
    dr_group(spec.mass, nom.v + 0, u, 0, 1, &mass);
    dr_group(spec.added, nom.v + 1, u, 2, 6, added);
    dr_group(spec.dlin, nom.v + 7, u, 14, 6, dlin);
    dr_group(spec.dquad, nom.v + 13, u, 26, 6, dquad);
    dr_group(spec.buoy, nom.v + 19, u, 38, 1, &buoy);
    dr_group(spec.current, nom.v + 20, u, 40, 3, cur);
    const int32_t f = write_record<T>(cls.inertia, cls.g0, dt, mass, added, dlin, dquad, buoy, cur, rec, npad, e, cls.rg);
    if (f) atomicOr(err, f);
}

// Masked redraw: the environments e < n whose mask byte is set, epoch epochs[e]. Few lanes
// of a wave are set (episodes that just restarted), so each one's draw is spread over the
// wave: parameter j (mass; added mass 1-6; linear damping 7-12; quadratic damping 13-18;
// buoyancy 19; current 20-22) is drawn on lane j from generator call j, the call whose
// uniform pair the per-lane path gives that parameter (a shared group uses its first
// entry's pair, taken by a lane shuffle), and the restarting lane gathers the 23 values and
// rebuilds its record. The values are those of the per-lane path; the wave spends about
// one parameter's draw per restart instead of the 23 in sequence. A wave with more than
// kSpreadDraws set lanes (all of them after a reset) takes the per-lane path instead.
constexpr int kSpreadDraws = 8;

template <typename T>
__device__ void dr_resample_spread(const mgx_dr_spec& spec, const DrNominal& nom, const ClassDesc64& cls, double dt,
                                   T* rec, int64_t npad, int64_t env_off, int64_t n, uint64_t seed,
                                   const uint8_t* mask, const int32_t* epochs, int32_t* err) {
    __shared__ mgx_dr_dist sd[6];
    __shared__ double snom[23];
    if (threadIdx.x == 0) {
        sd[0] = spec.mass;
        sd[1] = spec.added;
        sd[2] = spec.dlin;
        sd[3] = spec.dquad;
        sd[4] = spec.buoy;
        sd[5] = spec.current;
        for (int j = 0; j < 23; ++j) snom[j] = nom.v[j];
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool want = t < n && mask[t];
    const int32_t ep_own = want ? epochs[t] : 0;
    const int lane = __lane_id();
    const int j = lane < 23 ? lane : 0;
    const int grp = j == 0 ? 0 : j < 7 ? 1 : j < 13 ? 2 : j < 19 ? 3 : j == 19 ? 4 : 5;
    const int first = grp == 0 ? 0 : grp == 1 ? 1 : grp == 2 ? 7 : grp == 3 ? 13 : grp == 4 ? 19 : 20;
    const mgx_dr_dist& d = sd[grp];
    uint64_t need = __ballot(want);
    if (__popcll(need) > kSpreadDraws) {
        if (want) dr_resample_one<T>(spec, nom, cls, dt, rec, npad, env_off, t, seed, (uint32_t)ep_own, err);
        return;
    }
    while (need) {
        const int src = __ffsll((unsigned long long)need) - 1;
        need &= need - 1;
        const int64_t e = __shfl(t, src);
        uint32_t c[4] = {(uint32_t)(env_off + e), (uint32_t)__shfl(ep_own, src), (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)seed, kStreamDr << 24);
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const int from = d.shared ? first : j;
        const double v1 = __shfl(u1, from), v2 = __shfl(u2, from);
        double val = snom[j];
        if (d.kind != MGX_DR_FIXED) {
            const double x = dr_draw(d, v1, v2);
            val = d.relative ? snom[j] * x : x;
        }
        double p[23];
#pragma unroll
        for (int i = 0; i < 23; ++i) p[i] = __shfl(val, i);
        if (lane == src) {
            const int32_t f =
                write_record<T>(cls.inertia, cls.g0, dt, p[0], p + 1, p + 7, p + 13, p[19], p + 20, rec, npad, e, cls.rg);
            if (f) atomicOr(err, f);
        }
    }
}

// Environments `ids[t]` (or t) at epoch `epoch`; or, with `mask`, the environments e < n_ids
// whose mask byte is set, at epochs[e] (spread over the wave, above).
template <typename T>
__global__ void k_dr_resample(mgx_dr_spec spec, DrNominal nom, const ClassDesc64* cls, int ci, double dt, T* rec,
                              int64_t npad, int64_t env_off, const int64_t* ids, int64_t n_ids, uint64_t seed,
                              uint64_t epoch, const uint8_t* mask, const int32_t* epochs, int32_t* err) {
    if (mask) {
        dr_resample_spread<T>(spec, nom, cls[ci], dt, rec, npad, env_off, n_ids, seed, mask, epochs, err);
        return;
    }
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ids) return;
    const int64_t e = ids ? ids[t] : t;
    dr_resample_one<T>(spec, nom, cls[ci], dt, rec, npad, env_off, e, seed, epoch, err);
}

// Smallest value a distribution can produce (for validation).
static double dist_min(const mgx_dr_dist& d) {
    if (d.kind == MGX_DR_PIECEWISE) return d.edges[0];
    return d.lo;
}

static mgx_status check_dist(const mgx_dr_dist& d, const char* name, int size, const double* nom_all, int n_classes,
                             int off, bool positive, bool any_sign) {
    if (d.kind < MGX_DR_FIXED || d.kind > MGX_DR_PIECEWISE) return fail(MGX_E_INVALID, "%s: unknown kind", name);
    if (d.kind == MGX_DR_FIXED) return MGX_OK;
    if (d.kind == MGX_DR_UNIFORM || d.kind == MGX_DR_GAUSSIAN) {
        if (!std::isfinite(d.lo) || !std::isfinite(d.hi) || !(d.lo <= d.hi))
            return fail(MGX_E_INVALID, "%s: need finite lo <= hi", name);
        if (d.kind == MGX_DR_GAUSSIAN && (!std::isfinite(d.mean) || !(d.std >= 0) || !std::isfinite(d.std)))
            return fail(MGX_E_INVALID, "%s: need a finite mean and std >= 0", name);
    } else {
        if (d.n_bins < 1 || d.n_bins > MGX_DR_MAX_BINS) return fail(MGX_E_INVALID, "%s: n_bins outside [1, 8]", name);
        double sum = 0;
        for (int k = 0; k <= d.n_bins; ++k) {
            if (!std::isfinite(d.edges[k])) return fail(MGX_E_INVALID, "%s: non-finite edge", name);
            if (k > 0 && !(d.edges[k] > d.edges[k - 1])) return fail(MGX_E_INVALID, "%s: edges must increase", name);
        }
        for (int k = 0; k < d.n_bins; ++k) {
            if (!(d.weights[k] >= 0) || !std::isfinite(d.weights[k])) return fail(MGX_E_INVALID, "%s: bad weight", name);
            sum += d.weights[k];
        }
        if (!(sum > 0)) return fail(MGX_E_INVALID, "%s: weights sum to zero", name);
    }
    if (any_sign) return MGX_OK;
    const double lo = dist_min(d);
    for (int c = 0; c < n_classes; ++c)
        for (int i = 0; i < size; ++i) {
            const double v = d.relative ? lo * nom_all[23 * c + off + i] : lo;
            if (positive ? !(v > 0) : !(v >= 0))
                return fail(MGX_E_INVALID, "%s: the distribution can produce %g for class %d", name, v, c);
        }
    return MGX_OK;
}

}  // namespace mgx

using namespace mgx;

#define HIP_TRY_DR(b, call)                                       \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((b), e_, #call);    \
    } while (0)

namespace mgx {

static mgx_status check_spec(const mgx_batch* b, const mgx_dr_spec* spec, const double* nominal) {
    for (int c = 0; c < b->n_classes; ++c)
        for (int j = 0; j < 23; ++j) {
            const double v = nominal[23 * c + j];
            if (!std::isfinite(v) || (j < 20 && !(v >= 0)) || (j == 0 && !(v > 0)))
                return fail(MGX_E_INVALID, "nominal value %d of class %d invalid", j, c);
        }
    mgx_status s;
    if ((s = check_dist(spec->mass, "mass", 1, nominal, b->n_classes, 0, true, false)) != MGX_OK) return s;
    if ((s = check_dist(spec->added, "added", 6, nominal, b->n_classes, 1, false, false)) != MGX_OK) return s;
    if ((s = check_dist(spec->dlin, "dlin", 6, nominal, b->n_classes, 7, false, false)) != MGX_OK) return s;
    if ((s = check_dist(spec->dquad, "dquad", 6, nominal, b->n_classes, 13, false, false)) != MGX_OK) return s;
    if ((s = check_dist(spec->buoy, "buoy", 1, nominal, b->n_classes, 19, false, false)) != MGX_OK) return s;
    if ((s = check_dist(spec->current, "current", 3, nominal, b->n_classes, 20, false, true)) != MGX_OK) return s;
    return MGX_OK;
}

template <typename T>
static void launch_resample(mgx_batch* b, const mgx_dr_spec& spec, const double* nominal, int c, const int64_t* ids,
                            int64_t nid, uint64_t seed, uint64_t epoch, const uint8_t* mask, const int32_t* epochs) {
    DrNominal nom;
    for (int j = 0; j < 23; ++j) nom.v[j] = nominal[23 * c + j];
    const unsigned grid = (unsigned)((nid + 127) / 128);
    hipLaunchKernelGGL(k_dr_resample<T>, dim3(grid), dim3(128), 0, b->stream, spec, nom, b->d_classdesc, c, b->dt,
                       (T*)b->seg_rec(c), b->npad[c], b->env_off[c], ids, nid, seed, epoch, mask, epochs,
                       &b->d_misc->err);
}

mgx_status resample_masked(mgx_batch* b, const mgx_dr_spec* spec, const double* nominal, const uint8_t* mask,
                           const int32_t* epochs, uint64_t seed) {
    if (!spec || !nominal) return fail(MGX_E_INVALID, "spec / nominal is NULL");
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params or a full resample first");
    mgx_status st = check_spec(b, spec, nominal);
    if (st != MGX_OK) return st;
    hipDevice_guard g(b->device);
    for (int c = 0; c < b->n_classes; ++c) {
        if (b->prec == MGX_FP32)
            launch_resample<float>(b, *spec, nominal, c, nullptr, b->n[c], seed, 0, mask + b->pad_off[c],
                                   epochs + b->pad_off[c]);
        else
            launch_resample<double>(b, *spec, nominal, c, nullptr, b->n[c], seed, 0, mask + b->pad_off[c],
                                    epochs + b->pad_off[c]);
        HIP_TRY_DR(b, hipGetLastError());
    }
    return MGX_OK;
}

}  // namespace mgx

extern "C" mgx_status mgx_batch_resample(mgx_batch* b, const mgx_dr_spec* spec, const double* nominal,
                                         const int64_t* env_ids, int64_t n, uint64_t seed, uint64_t epoch) {
    if (!b) return fail(MGX_E_INVALID, "batch is NULL");
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!spec || !nominal) return fail(MGX_E_INVALID, "spec / nominal is NULL");
    if (env_ids && !b->params_set) return fail(MGX_E_STATE, "resample every environment (env_ids = NULL) first");
    if (env_ids && (n < 0 || n > b->n_total)) return fail(MGX_E_INVALID, "n outside [0, n_total]");
    mgx_status s = check_spec(b, spec, nominal);
    if (s != MGX_OK) return s;
    hipDevice_guard g(b->device);
    std::vector<int64_t> local;
    std::vector<int64_t> cnt(b->n_classes, 0), start(b->n_classes, 0);
    if (env_ids) {
        std::vector<std::vector<int64_t>> per(b->n_classes);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t gid = env_ids[i];
            if (gid < 0 || gid >= b->n_total) return fail(MGX_E_INVALID, "env id %lld out of range", (long long)gid);
            const int c = b->class_of(gid);
            per[c].push_back(gid - b->env_off[c]);
        }
        for (int c = 0; c < b->n_classes; ++c) {
            start[c] = (int64_t)local.size();
            cnt[c] = (int64_t)per[c].size();
            local.insert(local.end(), per[c].begin(), per[c].end());
        }
        if (!local.empty())
            HIP_TRY_DR(b, hipMemcpy(b->d_ids, local.data(), sizeof(int64_t) * local.size(), hipMemcpyHostToDevice));
    }
    for (int c = 0; c < b->n_classes; ++c) {
        const int64_t* ids = env_ids ? b->d_ids + start[c] : nullptr;
        const int64_t nid = env_ids ? cnt[c] : b->n[c];
        if (nid == 0) continue;
        if (b->prec == MGX_FP32)
            launch_resample<float>(b, *spec, nominal, c, ids, nid, seed, epoch, nullptr, nullptr);
        else
            launch_resample<double>(b, *spec, nominal, c, ids, nid, seed, epoch, nullptr, nullptr);
        HIP_TRY_DR(b, hipGetLastError());
    }
    if (!env_ids) b->params_set = true;
    return MGX_OK;
}

extern "C" mgx_status mgx_batch_get_params(const mgx_batch* b, double* mass, double* added, double* dlin,
                                           double* dquad, double* buoy, double* current) {
    if (!b) return fail(MGX_E_INVALID, "batch is NULL");
    if (!mass || !added || !dlin || !dquad || !buoy || !current) return fail(MGX_E_INVALID, "NULL output");
    if (!b->params_set) return fail(MGX_E_STATE, "no parameters set");
    hipDevice_guard g(b->device);
    const int64_t N = b->n_total;
    for (int c = 0; c < b->n_classes; ++c) {
        const int64_t np = b->npad[c], n = b->n[c], off = b->env_off[c];
        std::vector<double> r((size_t)kRecLen * np);
        if (b->prec == MGX_FP32) {
            std::vector<float> f((size_t)kRecLen * np);
            if (hipMemcpyAsync(f.data(), b->seg_rec(c), sizeof(float) * f.size(), hipMemcpyDeviceToHost, b->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(b->stream) != hipSuccess)
                return fail(MGX_E_DEVICE, "record copy failed");
            for (size_t k = 0; k < f.size(); ++k) r[k] = f[k];
        } else {
            if (hipMemcpyAsync(r.data(), b->seg_rec(c), sizeof(double) * r.size(), hipMemcpyDeviceToHost, b->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(b->stream) != hipSuccess)
                return fail(MGX_E_DEVICE, "record copy failed");
        }
        for (int64_t i = 0; i < n; ++i) {
            mass[off + i] = r[(size_t)kRecMass * np + i];
            buoy[off + i] = r[(size_t)kRecBuoy * np + i];
            for (int j = 0; j < 6; ++j) {
                added[j * N + off + i] = r[(size_t)(kRecAdded + j) * np + i];
                dlin[j * N + off + i] = r[(size_t)(kRecDlin + j) * np + i];
                dquad[j * N + off + i] = r[(size_t)(kRecDquad + j) * np + i];
            }
            for (int j = 0; j < 3; ++j) current[j * N + off + i] = r[(size_t)(kRecCurrent + j) * np + i];
        }
    }
    return MGX_OK;
}
