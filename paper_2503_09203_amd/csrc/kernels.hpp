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

// Class constants in double, derived from the caller's description, and their single
// rounding to float: thruster layout columns scaled by the gains (with the shaft torque),
// lag factors, fin plane bases and gains, inertia, centre of buoyancy and of gravity.
__host__ __device__ inline void class_setup_one(const ClassDesc64& d, double dt, uint32_t flags, ClassT<double>& D,
                                                ClassT<float>& F) {
    const int shaped = shaped_thrust(d) ? 1 : 0;
    const uint32_t fins = fin_mask_of(d);
    for (int i = 0; i < kMaxThr; ++i) {
        for (int j = 0; j < 3; ++j) D.fin_r[i][j] = D.fin_c[i][j] = D.fin_n[i][j] = 0.0;
        D.fin_max[i] = D.fin_kl[i] = D.fin_kd0[i] = D.fin_kd[i] = 0.0;
        if (i < d.m && ((fins >> i) & 1u)) {
            // fin: no layout column; the plane's basis from the span and the chord at zero
            // deflection (the chord's span component dropped)
            for (int j = 0; j < 6; ++j) D.Bk[j][i] = 0.0;
            double sl = sqrt(d.span[i][0] * d.span[i][0] + d.span[i][1] * d.span[i][1] + d.span[i][2] * d.span[i][2]);
            double s[3] = {d.span[i][0] / sl, d.span[i][1] / sl, d.span[i][2] / sl};
            double es = d.e[i][0] * s[0] + d.e[i][1] * s[1] + d.e[i][2] * s[2];
            double c[3] = {d.e[i][0] - es * s[0], d.e[i][1] - es * s[1], d.e[i][2] - es * s[2]};
            double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            for (int j = 0; j < 3; ++j) c[j] /= cl;
            const double nn[3] = {s[1] * c[2] - s[2] * c[1], s[2] * c[0] - s[0] * c[2], s[0] * c[1] - s[1] * c[0]};
            for (int j = 0; j < 3; ++j) {
                D.fin_r[i][j] = d.r[i][j];
                D.fin_c[i][j] = c[j];
                D.fin_n[i][j] = nn[j];
            }
            D.fin_max[i] = d.fin_max[i];
            D.fin_kl[i] = d.fin_lift[i];
            D.fin_kd0[i] = d.fin_drag0[i];
            D.fin_kd[i] = d.fin_drag[i];
            double tau = d.tau[i];
            D.alpha[i] = tau > 0.0 ? ((flags & kFlagLagEuler) ? dt / tau : 1.0 - exp(-dt / tau)) : 1.0;
            D.dz[i] = 0.0;
            D.rev[i] = 1.0;
        } else if (i < d.m) {
            double len = sqrt(d.e[i][0] * d.e[i][0] + d.e[i][1] * d.e[i][1] + d.e[i][2] * d.e[i][2]);
            double e[3] = {d.e[i][0] / len, d.e[i][1] / len, d.e[i][2] / len};
            const double* r = d.r[i];
            const double k = d.k[i];
            D.Bk[0][i] = k * e[0];
            D.Bk[1][i] = k * e[1];
            D.Bk[2][i] = k * e[2];
            // moment about the CoG plus the shaft torque c_i about the thrust axis
            const double c = d.reaction[i];
            D.Bk[3][i] = k * ((r[1] * e[2] - r[2] * e[1]) + c * e[0]);
            D.Bk[4][i] = k * ((r[2] * e[0] - r[0] * e[2]) + c * e[1]);
            D.Bk[5][i] = k * ((r[0] * e[1] - r[1] * e[0]) + c * e[2]);
            double tau = d.tau[i];
            D.alpha[i] = tau > 0.0 ? ((flags & kFlagLagEuler) ? dt / tau : 1.0 - exp(-dt / tau)) : 1.0;
            D.dz[i] = d.dz[i];
            D.rev[i] = reverse_ratio(d, i);
        } else {
            for (int j = 0; j < 6; ++j) D.Bk[j][i] = 0.0;
            D.alpha[i] = 0.0;
            D.dz[i] = 0.0;
            D.rev[i] = 1.0;
        }
    }
    for (int j = 0; j < 3; ++j) {
        D.inertia[j] = d.inertia[j];
        D.rb[j] = d.rb[j];
    }
    D.g0 = d.g0;
    D.dt = dt;
    D.inv_dt = 1.0 / dt;
    D.half_dt = 0.5 * dt;
    D.m = d.m;
    D.flags = flags;
    D.shaped = shaped;
    D.pad2 = 0;
    D.fin_mask = fins;
    D.pad3 = 0;
    for (int j = 0; j < 3; ++j) D.rg[j] = d.rg[j];
    D.payload = has_payload(d) ? 1 : 0;
    D.pad4 = 0;
    for (int i = 0; i < kMaxThr; ++i) {
        for (int j = 0; j < 6; ++j) F.Bk[j][i] = (float)D.Bk[j][i];
        F.alpha[i] = (float)D.alpha[i];
        F.dz[i] = (float)D.dz[i];
        F.rev[i] = (float)D.rev[i];
        for (int j = 0; j < 3; ++j) {
            F.fin_r[i][j] = (float)D.fin_r[i][j];
            F.fin_c[i][j] = (float)D.fin_c[i][j];
            F.fin_n[i][j] = (float)D.fin_n[i][j];
        }
        F.fin_max[i] = (float)D.fin_max[i];
        F.fin_kl[i] = (float)D.fin_kl[i];
        F.fin_kd0[i] = (float)D.fin_kd0[i];
        F.fin_kd[i] = (float)D.fin_kd[i];
    }
    for (int j = 0; j < 3; ++j) {
        F.inertia[j] = (float)D.inertia[j];
        F.rb[j] = (float)D.rb[j];
    }
    F.g0 = (float)D.g0;
    F.dt = (float)D.dt;
    F.inv_dt = (float)D.inv_dt;
    F.half_dt = (float)D.half_dt;
    F.m = D.m;
    F.flags = flags;
    F.shaped = shaped;
    F.pad2 = 0;
    F.fin_mask = fins;
    F.pad3 = 0;
    for (int j = 0; j < 3; ++j) F.rg[j] = (float)D.rg[j];
    F.payload = D.payload;
    F.pad4 = 0;
}

// Bits of DevMisc::err, the batch's device error word (read by mgx_batch_check).
constexpr int32_t kErrActionRow = 1;  // a step met an action row outside its buffer
constexpr int32_t kErrParam = 2;      // a record was built from a non-finite or out-of-range value
constexpr int32_t kErrNotSpd = 4;     // M_RB + M_A of some environment is not positive definite

// Device bookkeeping of a batch. The step counter is double-buffered: a launch reads
// slot rd and (if it moves the counter) its first block writes slot wr = 1 - rd, so the
// counter advances with one plain store and no completion handshake. `done` counts
// finished blocks per class for the statistics reduction only.
struct DevMisc {
    int64_t t[2];
    int32_t err;        // kErr* bits, sticky until the batch is destroyed
    int32_t check;      // kErr* bits of the last parameter check (mgx_batch_set_params)
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
    int32_t any_shaped;    // some class has dead zones or reverse gains: the kernel with both bodies
    uint32_t* simd_rank;   // [kSimdKeys] arrival table, or null
    float* tile_partials;  // [n_tiles][kStats] or null
    double* stats;         // [16][kStats]
};

// Arguments of the step kernel for one class segment.
// The first 64 bytes hold what the single-step form needs before its loads (one scalar
// cache line, fetched in the kernel's first batch of argument loads).
struct StepArgs {
    void* state;          // class segment base, [13+m][npad]
    const void* rec;      // class segment base, [30][npad]
    const void* actions;  // buffer base + class action offset; row r at actions + r*row_stride
    int64_t row_stride;
    // The step count the host expects the launch to start at (-1: none) and the action row
    // it names, which lies in the buffer (the host drops a hint whose row does not). The
    // single-step form fetches that row beside the state and confirms it against the
    // device counter afterwards, so the row's fetch does not wait for the counter's; a
    // one-step launch without a hint runs the K-step form, which reads the counter first.
    int64_t row_hint, t_hint;
    DevMisc* misc;
    int32_t npad, nvalid;
    int32_t rd, wr;       // step-counter slots
    int32_t hold, K;
    int64_t n_rows, row0;
    int32_t class_index;
    int32_t advance;      // 0, or K: block 0 writes t[wr] = t[rd] + K
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
    // Recompute buffer (states of two segments) and tape (the kTapeLen forward quantities of
    // their steps and the actions' clip mask), both private to the reverse sweep and blocked
    // by 64-environment tile:
    // [tile][2 x ckpt rows][field][64 lanes], so the fields of one step of one tile lie 256 B
    // apart and a wave reaches them from one address with immediate offsets.
    void* seg_buf;         // class block, (13+m) fields per row
    void* tape_buf;        // class block, kTapeLen + 1 fields per row
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
                            int cls_index, double dt, T* rec_seg, int32_t* err, hipStream_t s);
// Sets one device word to 0 (a kernel, not a memset node).
hipError_t launch_clear_word(int32_t* w, hipStream_t s);
// Checks the parameters of environments [env_off, env_off + n) as a record build would,
// without writing a record: ORs kErrParam / kErrNotSpd into *err.
hipError_t launch_check_params(ParamPtrs p, int64_t env_off, int64_t n, const ClassDesc64* d_cls, int cls_index,
                               int32_t* err, hipStream_t s);
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
