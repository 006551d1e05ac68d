// Device kernels of the batched underwater-vehicle step (gfx950, wave64).
//
// Layout: structure-of-arrays per class segment, component-major, so that lane j of a
// wavefront touches consecutive addresses for every component (coalesced 256-byte rows
// per wave in float). One environment per lane; the state stays in VGPRs for all K steps
// of a launch; per-class constants arrive as kernel arguments (scalar registers).
#include <hip/hip_runtime.h>

#include "env_loop.hpp"
#include "kernels.hpp"
#include "runtime_internal.hpp"

namespace mgx {


// ----------------------------------------------------------------------------- setup (double)

__global__ void k_class_setup(const ClassDesc64* in, ClassT<float>* outf, ClassT<double>* outd, int n, double dt,
                              uint32_t flags) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    ClassT<double> D;
    ClassT<float> F;
    class_setup_one(in[c], dt, flags, D, F);
    outd[c] = D;
    outf[c] = F;
}

// Per-environment parameters of global env g (double arrays over the global env id).
__device__ __forceinline__ void load_params(const ParamPtrs& p, int64_t g, double added[6], double dlin[6],
                                            double dquad[6], double cur[3]) {
    const int64_t N = p.n_total;
    for (int j = 0; j < 6; ++j) {
        added[j] = p.added[j * N + g];
        dlin[j] = p.dlin[j * N + g];
        dquad[j] = p.dquad[j * N + g];
    }
    for (int j = 0; j < 3; ++j) cur[j] = p.current[j * N + g];
}

// Per-environment record: dt M^-1 (M = M_RB + M_A), mass, added mass, damping, W - B, B,
// current; derived in double, rounded once. Invalid parameters set bits of *err.
template <typename T>
__global__ void k_env_setup(ParamPtrs p, int64_t env_off, int64_t n, int32_t npad, const ClassDesc64* cls,
                            int ci, double dt, T* rec, int32_t* err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g = env_off + i;
    double added[6], dlin[6], dquad[6], cur[3];
    load_params(p, g, added, dlin, dquad, cur);
    const int32_t f = write_record<T>(cls[ci].inertia, cls[ci].g0, dt, p.mass[g], added, dlin, dquad, p.buoy[g], cur,
                                      rec, npad, i, cls[ci].rg);
    if (f) atomicOr(err, f);
}

// The checks of k_env_setup alone, nothing written but the error bits.
__global__ void k_check_params(ParamPtrs p, int64_t env_off, int64_t n, const ClassDesc64* cls, int ci,
                               int32_t* err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g = env_off + i;
    double added[6], dlin[6], dquad[6], cur[3];
    load_params(p, g, added, dlin, dquad, cur);
    const int32_t f = params_flags(cls[ci].inertia, p.mass[g], added, dlin, dquad, p.buoy[g], cur, cls[ci].rg);
    if (f) atomicOr(err, f);
}

// Every slot of a segment to rest at the identity attitude; record zeroed (dt M^-1 = 0
// keeps padded slots fixed).
template <typename T>
__global__ void k_init_padding(T* state, T* rec, int m, int32_t npad, int64_t first, int rec_len) {
    int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    for (int j = 0; j < kStateFixed + m; ++j) state[j * (int64_t)npad + i] = (T)(j == 3 ? 1 : 0);
    for (int j = 0; j < rec_len; ++j) rec[j * (int64_t)npad + i] = (T)0;
}

// ----------------------------------------------------------------------------- reset

template <typename T>
__global__ void k_reset_seeded(T* state, int m, int32_t npad, int64_t env_off, int64_t n_local, const int64_t* ids,
                               int64_t n_ids, uint64_t seed) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ids) return;
    const int64_t e = ids ? ids[t] : t;
    if (e < 0 || e >= n_local) return;
    seeded_state<T>((uint64_t)(env_off + e), seed, m, state, npad, e);
}

template <typename T>
__global__ void k_reset_copy(T* state, const T* tmpl, int m, int32_t npad, const int64_t* ids, int64_t n_ids) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ids) return;
    const int64_t e = ids ? ids[t] : t;
    for (int j = 0; j < kStateFixed + m; ++j) state[j * (int64_t)npad + e] = tmpl[j * (int64_t)npad + e];
}

// ----------------------------------------------------------------------------- actions

template <typename T>
__global__ void k_gen_actions(T* out, int m, int32_t npad, int64_t n_valid, int64_t env_off, int64_t rows,
                              int64_t row_stride, int64_t row_offset, uint64_t seed) {
    const int64_t env = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = blockIdx.y;
    if (env >= npad || row >= rows) return;
    T* o = out + row * row_stride + env;
    if (env >= n_valid) {
        for (int i = 0; i < m; ++i) o[i * (int64_t)npad] = (T)0;
        return;
    }
    const uint64_t g = (uint64_t)(env_off + env);
    for (int b = 0; b < m; b += 4) {
        uint32_t c[4] = {(uint32_t)g, (uint32_t)(row_offset + row), (uint32_t)(b / 4), 0u};
        philox4x32_10(c, (uint32_t)seed, kStreamAction << 24);
        for (int w = 0; w < 4 && b + w < m; ++w) {
            o[(b + w) * (int64_t)npad] = (T)action_from_word(c[w]);
        }
    }
}

// Sets the device step counter (a kernel rather than a copy, so that it can sit inside a
// captured graph and needs no host synchronisation).
__global__ void k_set_counter(DevMisc* misc, int slot, int64_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        misc->t[slot] = t;
        prepare_next_slot(misc, slot);
    }
}

// ----------------------------------------------------------------------------- launchers

hipError_t launch_set_counter(DevMisc* misc, int slot, int64_t t, hipStream_t s) {
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, s, misc, slot, t);
    return hipGetLastError();
}

hipError_t launch_class_setup(const ClassDesc64* d_in, ClassT<float>* d_f, ClassT<double>* d_d, int n, double dt,
                              uint32_t flags, hipStream_t s) {
    hipLaunchKernelGGL(k_class_setup, dim3((n + 63) / 64), dim3(64), 0, s, d_in, d_f, d_d, n, dt, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_env_setup(ParamPtrs p, int64_t env_off, int64_t n, int32_t npad, const ClassDesc64* d_cls,
                            int cls_index, double dt, T* rec_seg, int32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_env_setup<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, env_off, n, npad,
                       d_cls, cls_index, dt, rec_seg, err);
    return hipGetLastError();
}

__global__ void k_clear_word(int32_t* w) { *w = 0; }

hipError_t launch_clear_word(int32_t* w, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_check_params(ParamPtrs p, int64_t env_off, int64_t n, const ClassDesc64* d_cls, int cls_index,
                               int32_t* err, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_params, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, env_off, n, d_cls,
                       cls_index, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_padding(T* state_seg, T* rec_seg, int m, int32_t npad, int64_t first, hipStream_t s,
                               int rec_len) {
    const int64_t n = npad - first;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_padding<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, state_seg, rec_seg, m,
                       npad, first, rec_len);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reset_seeded(T* state_seg, int m, int32_t npad, int64_t env_off, int64_t n_local,
                               const int64_t* d_local_ids, int64_t n_ids, uint64_t seed, hipStream_t s) {
    if (n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_seeded<T>, dim3((unsigned)((n_ids + 255) / 256)), dim3(256), 0, s, state_seg, m,
                       npad, env_off, n_local, d_local_ids, n_ids, seed);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reset_copy(T* state_seg, const T* tmpl_seg, int m, int32_t npad, const int64_t* d_local_ids,
                             int64_t n_ids, hipStream_t s) {
    if (n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_copy<T>, dim3((unsigned)((n_ids + 255) / 256)), dim3(256), 0, s, state_seg, tmpl_seg,
                       m, npad, d_local_ids, n_ids);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_actions(T* out_seg, int m, int32_t npad, int64_t n_valid, int64_t env_off, int64_t rows,
                              int64_t row_stride, int64_t row_offset, uint64_t seed, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_actions<T>, dim3((unsigned)((npad + 255) / 256), (unsigned)rows), dim3(256), 0, s,
                       out_seg, m, npad, n_valid, env_off, rows, row_stride, row_offset, seed);
    return hipGetLastError();
}

#define MGX_INSTANTIATE(T)                                                                                          \
    template hipError_t launch_env_setup<T>(ParamPtrs, int64_t, int64_t, int32_t, const ClassDesc64*, int, double,   \
                                            T*, int32_t*, hipStream_t);                                               \
    template hipError_t launch_init_padding<T>(T*, T*, int, int32_t, int64_t, hipStream_t, int);                    \
    template hipError_t launch_reset_seeded<T>(T*, int, int32_t, int64_t, int64_t, const int64_t*, int64_t, uint64_t, \
                                               hipStream_t);                                                          \
    template hipError_t launch_reset_copy<T>(T*, const T*, int, int32_t, const int64_t*, int64_t, hipStream_t);     \
    template hipError_t launch_gen_actions<T>(T*, int, int32_t, int64_t, int64_t, int64_t, int64_t, int64_t,        \
                                              uint64_t, hipStream_t);

MGX_INSTANTIATE(float)
MGX_INSTANTIATE(double)

}  // namespace mgx

