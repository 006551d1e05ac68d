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

// ----------------------------------------------------------------------------- step

// K steps of every environment of one class segment; state in registers throughout.
// kShaped: the class has dead zones or direction-dependent gains; kFins: it has fins;
// kPayload: its centre of gravity is off the body origin (fin and payload classes take the
// shaped propeller body too). Each is a separate instantiation (chosen
// on the host from the class) rather than a branch in one kernel, so that the plain
// body's register allocation does not pay for the others.
template <typename T, int M, bool kOut, bool kSingle, bool kShaped, bool kFins, bool kPayload>
__global__ void __launch_bounds__(256) k_step(StepLaunch<T> L) {
    const StepArgs& A = L.a;
    const int tid = threadIdx.x;
    const int64_t env = (int64_t)blockIdx.x * blockDim.x + tid;
    float st[kStats];
#pragma unroll
    for (int j = 0; j < kStats; ++j) st[j] = 0.0f;
    if constexpr (kSingle) {
        // Every lane runs (lanes past the segment on its last slot, without storing), so the
        // loads sit outside any branch; the step reads the counter itself, and the counter
        // update of slot wr comes after the environment work, so that no store precedes
        // (and may alias) the state and record loads. (Done that way in the K-step form, the
        // 16-step launch measured slower: 12.05 against 11.55 us.)
        int64_t t0 = 0;
        env_steps<T, M, kOut, kShaped, kSingle, kFins, kPayload>(A, L.cls, env, 0, A.K, st, &t0);
        if (blockIdx.x == 0 && tid == 0) {
            if (A.advance) A.misc->t[A.wr] = t0 + A.advance;
            prepare_next_slot(A.misc, A.wr);
        }
    } else {
        const int64_t t0 = A.misc->t[A.rd];
        if (blockIdx.x == 0 && tid == 0) {
            if (A.advance) A.misc->t[A.wr] = t0 + A.advance;
            prepare_next_slot(A.misc, A.wr);  // the next launch may be a persistent one
        }
        if (env < A.npad) env_steps<T, M, kOut, kShaped, kSingle, kFins, kPayload>(A, L.cls, env, t0, A.K, st);
    }
    if (!A.partials) return;
    // Statistics: block partials, then the last block to finish reduces them in order.
    __shared__ float red[256 / kWave][kStats];
    __shared__ int is_last;
    block_reduce_stats(st, red, A.partials + (int64_t)blockIdx.x * kStats);
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = atomicAdd(&A.misc->done[A.class_index], 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (tid < kStats) final_reduce_stats(A.partials, gridDim.x, tid, A.stats);
        if (tid == 0) atomicExch(&A.misc->done[A.class_index], 0u);
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

template <typename T, int M, bool kShaped, bool kFins, bool kPayload = false>
static void launch_step_body(const StepLaunch<T>& L, unsigned grid, int block, bool out, bool single,
                             hipStream_t s) {
    if (out)
        hipLaunchKernelGGL((k_step<T, M, true, false, kShaped, kFins, kPayload>), dim3(grid), dim3(block), 0, s, L);
    else if (single)
        hipLaunchKernelGGL((k_step<T, M, false, true, kShaped, kFins, kPayload>), dim3(grid), dim3(block), 0, s, L);
    else
        hipLaunchKernelGGL((k_step<T, M, false, false, kShaped, kFins, kPayload>), dim3(grid), dim3(block), 0, s, L);
}

// Five bodies: plain; shaped propellers; fins (with shaped propellers); payload (with
// shaped propellers); payload with fins and shaped propellers, the most general one. The
// payload body without fins keeps the fin geometry out of its registers.
template <typename T, int M>
static void launch_step_m(const StepLaunch<T>& L, unsigned grid, int block, bool out, bool single, bool shaped,
                          bool fins, bool payload, hipStream_t s) {
    if (payload && fins)
        launch_step_body<T, M, true, true, true>(L, grid, block, out, single, s);
    else if (payload)
        launch_step_body<T, M, true, false, true>(L, grid, block, out, single, s);
    else if (fins)
        launch_step_body<T, M, true, true>(L, grid, block, out, single, s);
    else if (shaped)
        launch_step_body<T, M, true, false>(L, grid, block, out, single, s);
    else
        launch_step_body<T, M, false, false>(L, grid, block, out, single, s);
}

#define MGX_STEP_CASE(MM)                                                     \
    case MM:                                                                  \
        launch_step_m<T, MM>(L, grid, block, out, single, shaped, fins, payload, s);   \
        break;

template <typename T>
hipError_t launch_step(const StepLaunch<T>& L, int m, int block, hipStream_t s) {
    const unsigned grid = (unsigned)((L.a.npad + block - 1) / block);
    const bool out = L.a.traj != nullptr || L.a.forces != nullptr;
    const bool single = L.a.K == 1;
    const bool shaped = L.cls.shaped != 0;
    const bool fins = L.cls.fin_mask != 0;
    const bool payload = L.cls.payload != 0;
    switch (m) {
        MGX_STEP_CASE(1)
        MGX_STEP_CASE(2)
        MGX_STEP_CASE(3)
        MGX_STEP_CASE(4)
        MGX_STEP_CASE(5)
        MGX_STEP_CASE(6)
        MGX_STEP_CASE(7)
        MGX_STEP_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
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
                                              uint64_t, hipStream_t);                                                 \
    template hipError_t launch_step<T>(const StepLaunch<T>&, int, int, hipStream_t);

MGX_INSTANTIATE(float)
MGX_INSTANTIATE(double)

}  // namespace mgx

// Per-wave phase times of the last step launch (diagnostic builds; see g_wave_ts).
extern "C" mgx_status mgx_diag_wave_times(uint64_t* out, int64_t n_waves) {
#ifdef MGX_WAVE_TIMESTAMPS
    if (!out || n_waves < 1 || n_waves > mgx::kWaveTsMax) return mgx::fail(MGX_E_INVALID, "n_waves outside [1, 65536]");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(out, HIP_SYMBOL(mgx::g_wave_ts), sizeof(uint64_t) * 4 * n_waves);
    if (e != hipSuccess) return mgx::fail(MGX_E_DEVICE, "wave times: %s", hipGetErrorString(e));
    return MGX_OK;
#else
    (void)out;
    (void)n_waves;
    return mgx::fail(MGX_E_STATE, "built without MGX_WAVE_TIMESTAMPS");
#endif
}
