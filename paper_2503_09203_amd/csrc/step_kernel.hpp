// The step kernel and its launchers, shared by the translation units that instantiate it
// per element type (the step kernels are most of the build's compile time).
#pragma once
#include <hip/hip_runtime.h>

#include "env_loop.hpp"
#include "kernels.hpp"

namespace mgx {

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
    // The single-step instantiation fetches the action row the host expects beside the
    // state; a one-step launch without that expectation (in a graph replayed from another
    // step than it was captured at) runs the K-step one, which reads the counter first.
    const bool single = L.a.K == 1 && L.a.t_hint >= 0;
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

}  // namespace mgx
