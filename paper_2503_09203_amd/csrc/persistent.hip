// Persistent heterogeneous launch: every vehicle class of a batch advanced by one kernel.
//
// Each block copies every class's constants and segment descriptor into LDS once. Wave w
// of the grid then runs tile w of the table (heaviest class first), and waves that finish
// pull the tiles beyond the grid from a device counter. The first round takes no atomic:
// every wave incrementing one counter at launch serialises on that address (about 13 ns
// each, so a thousand waves would start over 13 us). A tile belongs to one class, so the
// thruster count is uniform per wave and the `switch` over m selects a fully unrolled step
// body without divergence. The counter is double-buffered like the step counter: block 0
// clears the slot the next launch will use, so no end-of-launch handshake is needed.
// A batch with no shaped-thrust class runs an instantiation without the shaped body:
// holding both, the kernel needs more than the 256 registers that two waves per SIMD
// allow, and spills 50 of them to scratch memory.
#include <hip/hip_runtime.h>

#include "env_loop.hpp"
#include "kernels.hpp"

namespace mgx {

__device__ __forceinline__ float rfl(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ double rfl(double x) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// Class constants of thruster count M, from LDS into scalar registers (the values are
// uniform across the wave; only the fields the step body reads are moved).
template <typename T, int M>
__device__ __forceinline__ ClassT<T> class_to_sgpr(const ClassT<T>& L) {
    ClassT<T> C;
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int i = 0; i < M; ++i) C.Bk[j][i] = rfl(L.Bk[j][i]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        C.alpha[i] = rfl(L.alpha[i]);
        C.dz[i] = rfl(L.dz[i]);
        C.rev[i] = rfl(L.rev[i]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        C.inertia[j] = rfl(L.inertia[j]);
        C.rb[j] = rfl(L.rb[j]);
    }
    C.g0 = rfl(L.g0);
    C.dt = rfl(L.dt);
    C.inv_dt = rfl(L.inv_dt);
    C.half_dt = rfl(L.half_dt);
    C.m = M;
    C.flags = __builtin_amdgcn_readfirstlane(L.flags);
    C.shaped = __builtin_amdgcn_readfirstlane(L.shaped);
    return C;
}

template <typename T, int M, bool kShapedBody>
__device__ __forceinline__ void run_tile(const StepArgs& A, const ClassT<T>& L, bool shaped, int64_t env, int64_t t0,
                                         int K, float st[kStats]) {
    const ClassT<T> C = class_to_sgpr<T, M>(L);
    if (kShapedBody && shaped)
        env_steps<T, M, false, true>(A, C, env, t0, K, st);
    else
        env_steps<T, M, false, false>(A, C, env, t0, K, st);
}

template <typename T, bool kShapedBody>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_persistent(PersistArgs P) {
    __shared__ ClassT<T> lds_cls[16];
    __shared__ SegDesc lds_seg[16];
    {
        const uint32_t* src = (const uint32_t*)P.cls;
        uint32_t* dst = (uint32_t*)lds_cls;
        const int nw = P.n_classes * (int)(sizeof(ClassT<T>) / 4);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
        const uint32_t* src2 = (const uint32_t*)P.segs;
        uint32_t* dst2 = (uint32_t*)lds_seg;
        const int nw2 = P.n_classes * (int)(sizeof(SegDesc) / 4);
        for (int i = threadIdx.x; i < nw2; i += blockDim.x) dst2[i] = src2[i];
    }
    const int64_t t0 = P.misc->t[P.rd];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (P.advance) P.misc->t[P.wr] = t0 + P.advance;
        prepare_next_slot(P.misc, P.wr);
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t n_waves = gridDim.x * (blockDim.x / kWave);

    uint32_t tile = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    for (;; tile = 0xFFFFFFFFu) {
        if (tile == 0xFFFFFFFFu) {
            uint32_t i = 0;
            if (lane == 0) i = atomicAdd(&P.misc->work[P.rd], 1u);
            tile = n_waves + __builtin_amdgcn_readfirstlane(__shfl(i, 0, kWave));
        }
        if (tile >= (uint32_t)P.n_tiles) break;
        const int c = __builtin_amdgcn_readfirstlane(P.tiles[2 * tile]);
        const int env0 = __builtin_amdgcn_readfirstlane(P.tiles[2 * tile + 1]);
        const SegDesc& sd = lds_seg[c];
        StepArgs A;
        A.state = sd.state;
        A.rec = sd.rec;
        A.actions = (const T*)P.actions + sd.act_off;
        A.row_stride = P.row_stride;
        A.n_rows = P.n_rows;
        A.row0 = P.row0;
        A.hold = P.hold;
        A.K = P.K;
        A.npad = sd.npad;
        A.nvalid = sd.nvalid;
        A.misc = P.misc;
        A.class_index = c;
        A.advance = 0;
        A.rd = P.rd;
        A.wr = P.wr;
        A.t_hint = -1;
        A.row_hint = 0;
        A.traj = nullptr;
        A.traj_stride = 0;
        A.forces = nullptr;
        A.force_stride = 0;
        A.partials = P.tile_partials;
        A.stats = nullptr;
        const ClassT<T>& C = lds_cls[c];
        const bool shaped = sd.shaped != 0;
        const int64_t env = env0 + lane;
        float st[kStats];
#pragma unroll
        for (int j = 0; j < kStats; ++j) st[j] = 0.0f;
        switch (sd.m) {
            case 1: run_tile<T, 1, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 2: run_tile<T, 2, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 3: run_tile<T, 3, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 4: run_tile<T, 4, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 5: run_tile<T, 5, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 6: run_tile<T, 6, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            case 7: run_tile<T, 7, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
            default: run_tile<T, 8, kShapedBody>(A, C, shaped, env, t0, P.K, st); break;
        }
        if (P.tile_partials) {
#pragma unroll
            for (int j = 0; j < kStats; ++j) {
                const float v = is_max_slot(j) ? wave_max(st[j]) : wave_sum(st[j]);
                if (lane == j) P.tile_partials[(int64_t)tile * kStats + j] = v;
            }
        }
    }

    if (!P.tile_partials) return;
    // Statistics: the last wave to finish reduces the tile records per class, in table order.
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&P.misc->exits[P.rd], 1u);
    prev = __builtin_amdgcn_readfirstlane(__shfl(prev, 0, kWave));
    if (prev != n_waves - 1) return;
    __threadfence();
    if (lane < kStats) {
        const int j = lane;
        for (int c = 0; c < P.n_classes; ++c) {
            double acc = 0.0;
            for (int t = 0; t < P.n_tiles; ++t) {
                if (P.tiles[2 * t] != c) continue;
                const double v = (double)__hip_atomic_load(&P.tile_partials[(int64_t)t * kStats + j], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                acc = is_max_slot(j) ? fmax(acc, v) : acc + v;
            }
            P.stats[c * kStats + j] = acc;
        }
    }
}

template <typename T>
hipError_t launch_persistent(const PersistArgs& P, int grid, int block, hipStream_t s) {
    if (P.any_shaped)
        hipLaunchKernelGGL((k_persistent<T, true>), dim3(grid), dim3(block), 0, s, P);
    else
        hipLaunchKernelGGL((k_persistent<T, false>), dim3(grid), dim3(block), 0, s, P);
    return hipGetLastError();
}

// Float only: in double the per-class bodies do not fit the register budget of two waves
// per SIMD, and double batches use the per-class launches.
template hipError_t launch_persistent<float>(const PersistArgs&, int, int, hipStream_t);

}  // namespace mgx
