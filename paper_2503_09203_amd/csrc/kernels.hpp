// Internal interface between the host runtime and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step.hpp"

namespace mgx {

constexpr int kStats = 8;  // per-class statistics slots
enum StatSlot : int {
    kStNonFinite = 0,
    kStRenorm = 1,
    kStMaxSpeed = 2,
    kStSumSpeed = 3,
    kStMaxRate = 4,
    kStSumRate = 5,
    kStSumKin = 6,
    kStMaxDrift = 7
};

// Raw class description as given by the caller, double precision.
struct ClassDesc64 {
    int32_t m, pad;
    double r[kMaxThr][3], e[kMaxThr][3], k[kMaxThr], tau[kMaxThr], dz[kMaxThr];
    double k_rev[kMaxThr], reaction[kMaxThr];
    int32_t kind[kMaxThr];  // 0 propeller, 1 fin
    double span[kMaxThr][3], fin_max[kMaxThr], fin_lift[kMaxThr], fin_drag0[kMaxThr], fin_drag[kMaxThr];
    double inertia[3], rb[3], g0;
    double rg[3];  // payload: centre of gravity from the body origin
};

// True when the class carries a payload (centre of gravity off the body origin).
__host__ __device__ inline bool has_payload(const ClassDesc64& d) {
    return d.rg[0] != 0.0 || d.rg[1] != 0.0 || d.rg[2] != 0.0;
}

constexpr int32_t kActFin = 1;

// Reverse thrust gain over forward gain of thruster i (1 when the reverse gain is unset).
__host__ __device__ inline double reverse_ratio(const ClassDesc64& d, int i) {
    return (d.k_rev[i] > 0.0 && d.k_rev[i] != d.k[i]) ? d.k_rev[i] / d.k[i] : 1.0;
}

// True when some thruster has a dead zone or a direction-dependent gain: such classes run
// the shaped-thrust instantiation of the step body.
__host__ __device__ inline bool shaped_thrust(const ClassDesc64& d) {
    bool s = false;
    for (int i = 0; i < d.m && i < kMaxThr; ++i)
        s = s || (d.kind[i] != kActFin && (d.dz[i] > 0.0 || reverse_ratio(d, i) != 1.0));
    return s;
}

// Bit i set when actuator i is a fin.
__host__ __device__ inline uint32_t fin_mask_of(const ClassDesc64& d) {
    uint32_t mask = 0;
    for (int i = 0; i < d.m && i < kMaxThr; ++i)
        if (d.kind[i] == kActFin) mask |= 1u << i;
    return mask;
}

// Device bookkeeping of a batch. The step counter is double-buffered: a launch reads
// slot rd and (if it moves the counter) its first block writes slot wr = 1 - rd, so the
// counter advances with one plain store and no completion handshake. `done` counts
// finished blocks per class for the statistics reduction only.
struct DevMisc {
    int64_t t[2];
    int32_t err;
    int32_t pad;
    uint32_t done[16];
    uint32_t work[2];   // persistent launches: tiles handed out past the first round (slot rd)
    uint32_t exits[2];  // persistent launch with statistics: waves finished
};

// Run by one thread of every launch that reads slot rd: clears the counters of slot wr for
// the launch after it.
__device__ __forceinline__ void prepare_next_slot(DevMisc* m, int wr) {
    m->work[wr] = 0u;
    m->exits[wr] = 0u;
}

// One class segment as the persistent kernel sees it.
struct SegDesc {
    void* state;
    const void* rec;
    int64_t act_off;   // elements from the start of an action row
    int32_t npad, nvalid, m, shaped;
};

// Arguments of the persistent heterogeneous kernel (all classes, one launch).
struct PersistArgs {
    const SegDesc* segs;
    const void* cls;       // ClassT<T>[n_classes], staged into LDS by every block
    const int32_t* tiles;  // (class, first env) pairs, heaviest class first
    int32_t n_classes, n_tiles;
    const void* actions;
    int64_t row_stride, n_rows, row0;
    int32_t hold, K;
    DevMisc* misc;
    int32_t rd, wr, advance;
    int32_t n_heavy;       // tiles [0, n_heavy) go first to the first wave on each SIMD
    uint32_t* simd_rank;   // [kSimdKeys] arrival table, or null
    float* tile_partials;  // [n_tiles][kStats] or null
    double* stats;         // [16][kStats]
};

// Arguments of the step kernel for one class segment.
struct StepArgs {
    void* state;          // class segment base, [13+m][npad]
    const void* rec;      // class segment base, [30][npad]
    const void* actions;  // buffer base + class action offset; row r at actions + r*row_stride
    int64_t row_stride, n_rows, row0;
    int32_t hold, K;
    int32_t npad, nvalid;
    DevMisc* misc;
    int32_t class_index;
    int32_t advance;      // 0, or K: block 0 writes t[wr] = t[rd] + K
    int32_t rd, wr;       // step-counter slots
    void* traj;           // class segment base within step row 0, or null
    int64_t traj_stride;  // elements per step row
    void* forces;         // class segment base within step row 0, or null
    int64_t force_stride;
    float* partials;      // [gridDim.x][kStats] or null (no statistics)
    double* stats;        // [kStats] of this class, written by the last block
};

template <typename T>
struct StepLaunch {
    StepArgs a;
    ClassT<T> cls;
};

// Differentiable rollout, one class segment.
struct AdjArgs {
    void* state;           // class segment, [13+m][npad]
    const void* rec;       // [30][npad]
    const void* actions;   // buffer + class action offset
    int64_t row_stride, n_rows, row0;
    int32_t hold, H, ckpt, npad;
    int64_t t0;            // global step at the start of the rollout
    void* ckpt_buf;        // class segment within each checkpoint row; row stride ckpt_stride
    int64_t ckpt_stride;   // elements per checkpoint row (state_elems)
    void* seg_buf;         // recompute buffer, same layout, ckpt rows
    void* pos;             // class segment within a position row (3 x npad); row stride pos_stride
    int64_t pos_stride;
    void* dactions;        // class segment within an action row (m x npad), or null
    void* dparams;         // class segment [18][npad], or null
    DevMisc* misc;
    int32_t rd, wr, advance, pad;
};

// Host-side launchers (kernels.hip).
hipError_t launch_set_counter(DevMisc* misc, int slot, int64_t t, hipStream_t s);
hipError_t launch_class_setup(const ClassDesc64* d_in, ClassT<float>* d_f, ClassT<double>* d_d, int n,
                              double dt, uint32_t flags, hipStream_t s);
// Per-environment parameter arrays (double, over the global env id, DOF-major rows).
struct ParamPtrs {
    const double *mass, *added, *dlin, *dquad, *buoy, *current;
    int64_t n_total;
};

template <typename T>
hipError_t launch_env_setup(ParamPtrs p, int64_t env_off, int64_t n, int32_t npad, const ClassDesc64* d_cls,
                            int cls_index, double dt, T* rec_seg, hipStream_t s);
template <typename T>
hipError_t launch_reset_seeded(T* state_seg, int m, int32_t npad, int64_t env_off, int64_t n_local,
                               const int64_t* d_local_ids, int64_t n_ids, uint64_t seed, hipStream_t s);
template <typename T>
hipError_t launch_reset_copy(T* state_seg, const T* tmpl_seg, int m, int32_t npad, const int64_t* d_local_ids,
                             int64_t n_ids, hipStream_t s);
template <typename T>
hipError_t launch_init_padding(T* state_seg, T* rec_seg, int m, int32_t npad, int64_t nvalid, hipStream_t s,
                               int rec_len = kRecLen);
template <typename T>
hipError_t launch_gen_actions(T* out_seg, int m, int32_t npad, int64_t n_valid, int64_t env_off, int64_t rows,
                              int64_t row_stride, int64_t row_offset, uint64_t seed, hipStream_t s);
template <typename T>
hipError_t launch_step(const StepLaunch<T>& L, int m, int block, hipStream_t s);
template <typename T>
hipError_t launch_persistent(const PersistArgs& P, int grid, int block, hipStream_t s);
template <typename T>
hipError_t launch_rollout_fwd(const AdjArgs& A, const ClassT<T>& C, int m, bool shaped, hipStream_t s);
template <typename T>
hipError_t launch_rollout_bwd(const AdjArgs& A, const ClassT<T>& C, int m, bool shaped, hipStream_t s);

}  // namespace mgx
