// Differentiable rollout: forward pass with checkpoints, and the reverse sweep with
// per-segment recomputation. One environment per lane; the adjoint state and the parameter
// adjoints stay in registers for the whole sweep.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>

#include "adjoint.hpp"
#include "env_loop.hpp"
#include "kernels.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"

namespace mgx {

template <typename T>
__device__ __forceinline__ void load_env(const T* Rc, int64_t np, int64_t e, EnvT<T>& E) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        E.dtMinv[j] = Rc[(kRecDtMinv + j) * np + e];
        E.A[j] = Rc[(kRecAdded + j) * np + e];
        E.dL[j] = Rc[(kRecDlin + j) * np + e];
        E.dQ[j] = Rc[(kRecDquad + j) * np + e];
    }
    E.mass = Rc[kRecMass * np + e];
    E.wmb = Rc[kRecWmB * np + e];
    E.buoy = Rc[kRecBuoy * np + e];
#pragma unroll
    for (int j = 0; j < 3; ++j) E.Vc[j] = Rc[(kRecCurrent + j) * np + e];
}

// Row of the action buffer used by a step (rows validated on the host), and its phase
// within the hold interval, moved one step at a time (no division in the step loops).
struct RowCursor {
    int64_t row;
    int32_t phase, hold;
    __device__ RowCursor(const AdjArgs& A, int64_t t) : hold(A.hold) {
        const int64_t q = floor_div(t, (int64_t)A.hold);
        row = q - A.row0;
        phase = (int32_t)(t - q * A.hold);
    }
    __device__ int64_t next_row() const { return phase + 1 == hold ? row + 1 : row; }
    __device__ int64_t prev_row() const { return phase == 0 ? row - 1 : row; }
    __device__ void advance() {
        if (++phase == hold) {
            phase = 0;
            ++row;
        }
    }
    __device__ void retreat() {
        if (phase == 0) {
            phase = hold - 1;
            --row;
        } else {
            --phase;
        }
    }
};

// Tape of one step: field f of environment e at row + f * field + e (fields: fd[0..M-1] at
// 0.., R at kMaxThr, vc, F, c, sh, dc, dsh, nq, g).
template <typename T, int M>
__device__ __forceinline__ void store_tape(T* row, int64_t field, int64_t e, const VjpTape<T>& tp) {
    T* o = row + e;
#pragma unroll
    for (int i = 0; i < M; ++i) o[i * field] = tp.fd[i];
    o += kMaxThr * field;
#pragma unroll
    for (int j = 0; j < 9; ++j) o[j * field] = tp.R[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) o[(9 + j) * field] = tp.vc[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) o[(12 + j) * field] = tp.F[j];
    o[18 * field] = tp.c;
    o[19 * field] = tp.sh;
    o[20 * field] = tp.dc;
    o[21 * field] = tp.dsh;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[(22 + j) * field] = tp.nq[j];
    o[26 * field] = tp.g;
}

template <typename T, int M>
__device__ __forceinline__ void load_tape(const T* row, int64_t field, int64_t e, VjpTape<T>& tp) {
    const T* o = row + e;
#pragma unroll
    for (int i = 0; i < M; ++i) tp.fd[i] = o[i * field];
    o += kMaxThr * field;
#pragma unroll
    for (int j = 0; j < 9; ++j) tp.R[j] = o[j * field];
#pragma unroll
    for (int j = 0; j < 3; ++j) tp.vc[j] = o[(9 + j) * field];
#pragma unroll
    for (int j = 0; j < 6; ++j) tp.F[j] = o[(12 + j) * field];
    tp.c = o[18 * field];
    tp.sh = o[19 * field];
    tp.dc = o[20 * field];
    tp.dsh = o[21 * field];
#pragma unroll
    for (int j = 0; j < 4; ++j) tp.nq[j] = o[(22 + j) * field];
    tp.g = o[26 * field];
}

// Fields of a tape row: the step's forward quantities, then the mask of the actions that the
// clip to [-1, 1] passes through (bit i for actuator i, held as a value of T): the reverse
// sweep needs no action values of its own.
constexpr int kTapeFields = kTapeLen + 1;

template <typename T, int M>
__device__ __forceinline__ void load_action(const AdjArgs& A, int64_t row, int64_t e, T raw[M]) {
    const T* src = (const T*)A.actions + row * A.row_stride + e;
#pragma unroll
    for (int i = 0; i < M; ++i) raw[i] = src[i * (int64_t)A.npad];
}

// Row k of segment `seg` in a tile's block of the recompute buffer (states) and of the tape,
// both [tile][2 x ckpt rows][field][64 lanes]; consecutive segments alternate between the
// two halves of a block.
template <typename T, int M>
__device__ __forceinline__ T* seg_row_of(const AdjArgs& A, int64_t tile, int seg, int k) {
    constexpr int kRow = (kStateFixed + M) * kWave;
    return (T*)A.seg_buf + (tile * 2 * A.ckpt + (seg & 1) * A.ckpt + (k - seg * A.ckpt)) * kRow;
}
template <typename T>
__device__ __forceinline__ T* tape_row_of(const AdjArgs& A, int64_t tile, int seg, int k) {
    constexpr int kRow = kTapeFields * kWave;
    return (T*)A.tape_buf + (tile * 2 * A.ckpt + (seg & 1) * A.ckpt + (k - seg * A.ckpt)) * kRow;
}

// Segment `seg` (steps k0 .. k1 - 1) run from its checkpoint the way the reverse sweep needs
// it: each step's state before the step into the recompute buffer, and its forward
// quantities and the actions' clip mask into the tape. Used by the forward pass for the last
// segment and by the backward for the others; the actions of step k + 1 are in flight while
// step k runs.
template <typename T, int M, bool kShaped>
__device__ __forceinline__ void recompute_segment(const AdjArgs& A, const ClassT<T>& C, const EnvT<T>& E,
                                                  const T IA2[3], const T Brb[3], int64_t e, int lane, int seg) {
    const int k0 = seg * A.ckpt;
    const int k1 = (k0 + A.ckpt < A.H) ? k0 + A.ckpt : A.H;
    const int64_t tile = e / kWave;
    StateT<T, M> s;
    load_state<T, M>((const T*)A.ckpt_buf + (int64_t)seg * A.ckpt_stride, A.npad, e, s);
    RowCursor rc(A, A.t0 + k0);
    T a[M], nxt[M];
    load_action<T, M>(A, rc.row, e, nxt);
    for (int k = k0; k < k1; ++k) {
        uint32_t pass = 0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            pass |= (nxt[i] > T(-1) && nxt[i] < T(1)) ? 1u << i : 0u;
            a[i] = clip1(nxt[i]);
        }
        load_action<T, M>(A, k + 1 < k1 ? rc.next_row() : rc.row, e, nxt);
        rc.advance();
        store_state<T, M>(seg_row_of<T, M>(A, tile, seg, k), kWave, lane, s);
        VjpTape<T> tp;
        step_body<T, M, false, kShaped, false, false, false, true>(C, E, IA2, Brb, s, a, nullptr, nullptr, &tp);
        T* tr = tape_row_of<T>(A, tile, seg, k);
        store_tape<T, M>(tr, kWave, lane, tp);
        tr[kTapeLen * kWave + lane] = T(pass);
    }
}

// Forward pass with checkpoints. Two waves per 64-environment tile (block of 128): wave 0
// runs every step, storing the checkpoints and the positions; once it has stored the last
// segment's checkpoint (block barrier), wave 1 runs that segment again as the backward's
// recomputation would, into the recompute buffer and the tape, while wave 0 finishes it. The
// backward then sweeps the last segment at once instead of first waiting for its
// recomputation. The grid covers the padded segment exactly, so both waves reach the barrier.
template <typename T, int M, bool kShaped>
__global__ void __launch_bounds__(128) k_rollout_fwd(AdjArgs A, ClassT<T> Cs) {
    const int role = threadIdx.x / kWave;  // 0: the rollout, 1: the last segment's tape
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t e = (int64_t)blockIdx.x * kWave + lane;
    const ClassT<T> C = class_in_vgpr<T, M>(Cs);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (A.advance) A.misc->t[A.wr] = A.t0 + A.advance;
        prepare_next_slot(A.misc, A.wr);
    }
    const int64_t np = A.npad;
    EnvT<T> E;
    load_env<T>((const T*)A.rec, np, e, E);
    set_amc(E, C.flags);
    T IA2[3], Brb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        IA2[j] = C.inertia[j] + E.A[3 + j];
        Brb[j] = E.buoy * C.rb[j];
    }
    T* ck = (T*)A.ckpt_buf;
    const int seg_last = (A.H - 1) / A.ckpt, k_last = seg_last * A.ckpt;
    if (role == 1) {
        __syncthreads();
        recompute_segment<T, M, kShaped>(A, C, E, IA2, Brb, e, lane, seg_last);
        return;
    }
    T* pos = (T*)A.pos;
    StateT<T, M> s;
    load_state<T, M>((const T*)A.state, np, e, s);
    // The action row of step k + 1 is in flight while step k runs (with per-step actions a
    // load issued right before its use would leave every step waiting on memory).
    RowCursor rc(A, A.t0);
    T a[M], nxt[M];
    load_action<T, M>(A, rc.row, e, nxt);
    auto step = [&](int k) {
#pragma unroll
        for (int i = 0; i < M; ++i) a[i] = clip1(nxt[i]);
        load_action<T, M>(A, k + 1 < A.H ? rc.next_row() : rc.row, e, nxt);
        rc.advance();
        step_body<T, M, false, kShaped>(C, E, IA2, Brb, s, a);
#pragma unroll
        for (int j = 0; j < 3; ++j) pos[(int64_t)k * A.pos_stride + j * np + e] = s.p[j];
    };
    for (int k = 0; k < k_last; ++k) {
        if (k % A.ckpt == 0) store_state<T, M>(ck + (int64_t)(k / A.ckpt) * A.ckpt_stride, np, e, s);
        step(k);
    }
    store_state<T, M>(ck + (int64_t)seg_last * A.ckpt_stride, np, e, s);
    __syncthreads();
    for (int k = k_last; k < A.H; ++k) step(k);
    store_state<T, M>((T*)A.state, np, e, s);
}

// Reverse sweep with per-segment recomputation. Two waves per 64-environment tile (block of
// 128): wave 1 recomputes segment s - 1 from its checkpoint into one half of the segment
// buffer while wave 0 sweeps segment s backwards from the other half, so recomputation
// overlaps the sweep; the block barrier after each segment hands the halves over. The last
// segment is in its half already (the forward pass stored it). The grid covers the padded
// segment exactly, so both waves reach every barrier.
template <typename T, int M, bool kShaped>
__global__ void __launch_bounds__(128) k_rollout_bwd(AdjArgs A, ClassT<T> Cs) {
    const int role = threadIdx.x / kWave;  // 0: sweep, 1: recompute
    const int64_t e = (int64_t)blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const ClassT<T> C = class_in_vgpr<T, M>(Cs);
    const int64_t np = A.npad;
    EnvT<T> E;
    load_env<T>((const T*)A.rec, np, e, E);
    set_amc(E, C.flags);
    T IA2[3], Brb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        IA2[j] = C.inertia[j] + E.A[3 + j];
        Brb[j] = E.buoy * C.rb[j];
    }
    // this tile's blocks of the recompute buffer and the tape (the layout of seg_row_of and
    // tape_row_of, with the tile's base hoisted); within a row, field f of lane l at
    // f * kWave + l
    constexpr int kSegRow = (kStateFixed + M) * kWave, kTapeRow = kTapeFields * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    T* sg = (T*)A.seg_buf + (int64_t)blockIdx.x * 2 * A.ckpt * kSegRow;
    T* tb = (T*)A.tape_buf + (int64_t)blockIdx.x * 2 * A.ckpt * kTapeRow;
    const int nseg = (A.H + A.ckpt - 1) / A.ckpt;
    auto seg_row = [&](int seg, int k) { return sg + ((seg & 1) * A.ckpt + (k - seg * A.ckpt)) * kSegRow; };
    auto tape_row = [&](int seg, int k) { return tb + ((seg & 1) * A.ckpt + (k - seg * A.ckpt)) * kTapeRow; };

    // the forward pass stored the last segment's states and tape
    if (role == 1) {
        for (int seg = nseg - 1; seg >= 0; --seg) {
            if (seg > 0) recompute_segment<T, M, kShaped>(A, C, E, IA2, Brb, e, lane, seg - 1);
            __syncthreads();
        }
        return;
    }

    const T* dpos = (const T*)A.pos;
    T* dact = (T*)A.dactions;
    StateT<T, M> xb;
#pragma unroll
    for (int j = 0; j < 3; ++j) xb.p[j] = T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) xb.q[j] = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) xb.nu[j] = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) xb.n[i] = T(0);
    T gdL[6], gdQ[6], gA[6], gDt[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) gdL[j] = gdQ[j] = gA[j] = gDt[j] = T(0);
    int64_t row_cur = -1;
    T arow[M];
#pragma unroll
    for (int i = 0; i < M; ++i) arow[i] = T(0);

    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int k0 = seg * A.ckpt;
        const int k1 = (k0 + A.ckpt < A.H) ? k0 + A.ckpt : A.H;
        // The stored state, tape and position adjoint of step k - 1 are fetched while
        // step k runs (at k0 the fetch repeats step k0), into the other of two buffers: the
        // loop takes two steps per turn, so no step copies its fetched values into the ones
        // it works on (a copy per value and step when one buffer was refilled).
        struct Buf {
            StateT<T, M> s;
            VjpTape<T> tp;
            T dp[3], pass;
        };
        Buf b0, b1;
        auto fetch = [&](Buf& b, int k) {
            load_state<T, M>(seg_row(seg, k), kWave, lane, b.s);
            const T* tr = tape_row(seg, k);
            load_tape<T, M>(tr, kWave, lane, b.tp);
            b.pass = tr[kTapeLen * kWave + lane];
#pragma unroll
            for (int j = 0; j < 3; ++j) b.dp[j] = dpos[(int64_t)k * A.pos_stride + j * np + e];
        };
        RowCursor rb(A, A.t0 + k1 - 1);
        // step k from buffer `cur`, fetching step k - 1 into `nxt`
        auto reverse_step = [&](Buf& cur, Buf& nxt, int k) {
            T ab[M];
#pragma unroll
            for (int j = 0; j < 3; ++j) xb.p[j] += cur.dp[j];
            const int64_t r = rb.row;
            fetch(nxt, k > k0 ? k - 1 : k0);
            rb.retreat();
            vjp_reverse<T, M, kShaped>(C, E, IA2, Brb, cur.s, cur.tp, xb, ab, gdL, gdQ, gA, gDt);
            if (r != row_cur) {
                if (row_cur >= 0 && dact) {
#pragma unroll
                    for (int i = 0; i < M; ++i) dact[row_cur * A.row_stride + i * np + e] = arow[i];
                }
                row_cur = r;
#pragma unroll
                for (int i = 0; i < M; ++i) arow[i] = T(0);
            }
            const uint32_t pass = (uint32_t)cur.pass;
#pragma unroll
            for (int i = 0; i < M; ++i) arow[i] += ((pass >> i) & 1u) ? ab[i] : T(0);
        };
        fetch(b0, k1 - 1);
        for (int k = k1 - 1;;) {
            reverse_step(b0, b1, k);
            if (--k < k0) break;
            reverse_step(b1, b0, k);
            if (--k < k0) break;
        }
        __syncthreads();
    }
    if (row_cur >= 0 && dact) {
#pragma unroll
        for (int i = 0; i < M; ++i) dact[row_cur * A.row_stride + i * np + e] = arow[i];
    }
    if (A.dparams) {
        T* gp = (T*)A.dparams;
        const T inv_dt = C.inv_dt;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            gp[j * np + e] = gdL[j];
            gp[(6 + j) * np + e] = gdQ[j];
            // dt M^-1 = dt / (M_RB + M_A): d/dM_A = -(dt M^-1)^2 / dt
            gp[(12 + j) * np + e] = gA[j] - gDt[j] * E.dtMinv[j] * E.dtMinv[j] * inv_dt;
        }
    }
}

#define MGX_ADJ_CASE(MM)                                                                                         \
    case MM:                                                                                                     \
        if (shaped)                                                                                              \
            hipLaunchKernelGGL((KERNEL<T, MM, true>), dim3(grid), dim3(block), 0, s, A, C);                      \
        else                                                                                                     \
            hipLaunchKernelGGL((KERNEL<T, MM, false>), dim3(grid), dim3(block), 0, s, A, C);                     \
        break;

#define MGX_ADJ_SWITCH          \
    switch (m) {                \
        MGX_ADJ_CASE(1)         \
        MGX_ADJ_CASE(2)         \
        MGX_ADJ_CASE(3)         \
        MGX_ADJ_CASE(4)         \
        MGX_ADJ_CASE(5)         \
        MGX_ADJ_CASE(6)         \
        MGX_ADJ_CASE(7)         \
        MGX_ADJ_CASE(8)         \
        default:                \
            return hipErrorInvalidValue; \
    }

template <typename T>
hipError_t launch_rollout_fwd(const AdjArgs& A, const ClassT<T>& C, int m, bool shaped, hipStream_t s) {
    // one block of two waves per 64-environment tile (npad is a multiple of 64): a few
    // thousand environments are a few tiles per class, each on a compute unit of its own
    // (blocks of several tiles packed them onto fewer units, sharing their issue and memory
    // pipelines: 0.180 against 0.171 ms at 8192 x 256 with 8 thrusters)
    if (A.npad % kWave != 0) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(A.npad / kWave), block = 2 * kWave;
#define KERNEL k_rollout_fwd
    MGX_ADJ_SWITCH
#undef KERNEL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rollout_bwd(const AdjArgs& A, const ClassT<T>& C, int m, bool shaped, hipStream_t s) {
    // one block of two waves per 64-environment tile; npad is a multiple of 64
    if (A.npad % kWave != 0) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(A.npad / kWave), block = 2 * kWave;
#define KERNEL k_rollout_bwd
    MGX_ADJ_SWITCH
#undef KERNEL
    return hipGetLastError();
}

template hipError_t launch_rollout_fwd<float>(const AdjArgs&, const ClassT<float>&, int, bool, hipStream_t);
template hipError_t launch_rollout_fwd<double>(const AdjArgs&, const ClassT<double>&, int, bool, hipStream_t);
template hipError_t launch_rollout_bwd<float>(const AdjArgs&, const ClassT<float>&, int, bool, hipStream_t);
template hipError_t launch_rollout_bwd<double>(const AdjArgs&, const ClassT<double>&, int, bool, hipStream_t);

}  // namespace mgx

using namespace mgx;

static bool class_shaped(const mgx_batch* b, int c) { return shaped_thrust(to_desc64(b->cls[c])); }

static AdjArgs adj_args(mgx_batch* b, int c) {
    const size_t P = (size_t)b->prec;
    AdjArgs A;
    std::memset(&A, 0, sizeof A);
    A.state = b->seg_state(c);
    A.rec = b->seg_rec(c);
    A.actions = (const char*)b->ro_actions + P * b->act_off[c];
    A.row_stride = b->row_elems;
    A.n_rows = b->ro_n_rows;
    A.row0 = b->ro_row0;
    A.hold = b->ro_hold;
    A.H = b->ro_H;
    A.ckpt = b->ro_ckpt;
    A.npad = (int32_t)b->npad[c];
    A.t0 = b->ro_t0;
    A.ckpt_buf = (char*)b->ro_ckpt_mem + P * b->state_off[c];
    A.ckpt_stride = b->state_elems;
    // tile-blocked: a class's block follows the blocks of the classes before it
    A.seg_buf = (char*)b->ro_seg_mem + P * (size_t)2 * b->ro_ckpt * b->state_off[c];
    A.tape_buf = (char*)b->ro_tape_mem + P * (size_t)2 * b->ro_ckpt * kTapeFields * b->pad_off[c];
    A.pos_stride = 3 * b->npad_total;
    A.misc = b->d_misc;
    return A;
}

// The static scratch of the allocation-free forward pass: one array per GPU (each device
// holds its own copy at its own address), its address taken once per device with that
// device current. The generation counts static forward passes per device, so a backward
// pass can tell that a later one has overwritten its checkpoints.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
uint64_t g_scratch_gen[kMaxScratchDevices] = {};
}  // namespace

// Address of this device's scratch array (the array's name is only a host-side stand-in).
static mgx_status scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(MGX_E_INVALID, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        hipDevice_guard g(dev);
        if (!g.ok()) return hip_fail(nullptr, g.err(), "hipSetDevice");
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MGX_OK;
}

static mgx_status rollout_forward(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                  int32_t H, int32_t ckpt_every, void* pos_out, bool use_static) {
    if (!b) return fail(MGX_E_INVALID, "batch is NULL");
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params has not been called");
    if (!actions || !pos_out) return fail(MGX_E_INVALID, "actions / pos_out is NULL");
    for (int c = 0; c < b->n_classes; ++c) {
        if (b->h_class_f[c].fin_mask != 0)
            return fail(MGX_E_INVALID, "class %d has fins: the adjoint covers propeller classes only", c);
        if (b->h_class_f[c].payload != 0)
            return fail(MGX_E_INVALID, "class %d has a payload: the adjoint covers classes without one", c);
    }
    if (H < 1 || H > (1 << 20)) return fail(MGX_E_INVALID, "H=%d outside [1, 2^20]", H);
    if (ckpt_every < 1 || ckpt_every > 4096) return fail(MGX_E_INVALID, "ckpt_every=%d outside [1, 4096]", ckpt_every);
    if (hold < 1 || n_rows < 1) return fail(MGX_E_INVALID, "hold, n_rows must be >= 1");
    mgx_status v = validate_rows(b, b->host_t, n_rows, row0, hold, H);
    if (v != MGX_OK) return v;
    hipDevice_guard guard(b->device);
    const int64_t nck = (H + ckpt_every - 1) / ckpt_every;
    const size_t P = (size_t)b->prec;
    const size_t ck_bytes = P * (size_t)nck * b->state_elems, seg_bytes = P * (size_t)2 * ckpt_every * b->state_elems;
    const size_t tape_bytes = P * (size_t)2 * ckpt_every * kTapeFields * b->npad_total;
    void* ck_mem = nullptr;
    void* seg_mem = nullptr;
    void* tape_mem = nullptr;
    uint64_t gen = 0;
    if (use_static) {
        const size_t ck_aligned = (ck_bytes + 255) / 256 * 256, seg_aligned = (seg_bytes + 255) / 256 * 256;
        if (ck_aligned + seg_aligned + tape_bytes > kScratchBytes)
            return fail(MGX_E_INVALID, "the rollout needs %zu bytes of checkpoints and segment scratch; the static "
                        "scratch holds %zu", ck_aligned + seg_aligned + tape_bytes, kScratchBytes);
        void* base = nullptr;
        mgx_status st = scratch_address(b->device, &base);
        if (st != MGX_OK) return st;
        ck_mem = base;
        seg_mem = (char*)base + ck_aligned;
        tape_mem = (char*)base + ck_aligned + seg_aligned;
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        gen = ++g_scratch_gen[b->device];
    } else {
        if (ck_bytes > b->ckpt_bytes) {
            b->dev_free(b->d_ckpt);
            b->d_ckpt = nullptr;
            b->ckpt_bytes = 0;
            hipError_t e;
            b->d_ckpt = b->dev_alloc(ck_bytes, &e);
            if (e != hipSuccess) return hip_fail(nullptr, e, "hipMalloc(checkpoints)");
            b->ckpt_bytes = ck_bytes;
        }
        if (seg_bytes > b->seg_bytes) {
            b->dev_free(b->d_seg);
            b->d_seg = nullptr;
            b->seg_bytes = 0;
            hipError_t e;
            b->d_seg = b->dev_alloc(seg_bytes, &e);
            if (e != hipSuccess) return hip_fail(nullptr, e, "hipMalloc(segment scratch)");
            b->seg_bytes = seg_bytes;
        }
        if (tape_bytes > b->tape_bytes) {
            b->dev_free(b->d_tape);
            b->d_tape = nullptr;
            b->tape_bytes = 0;
            hipError_t e;
            b->d_tape = b->dev_alloc(tape_bytes, &e);
            if (e != hipSuccess) return hip_fail(nullptr, e, "hipMalloc(segment tape)");
            b->tape_bytes = tape_bytes;
        }
        ck_mem = b->d_ckpt;
        seg_mem = b->d_seg;
        tape_mem = b->d_tape;
    }
    b->ro_ckpt_mem = ck_mem;
    b->ro_seg_mem = seg_mem;
    b->ro_tape_mem = tape_mem;
    b->ro_static_gen = gen;
    b->ro_actions = actions;
    b->ro_n_rows = n_rows;
    b->ro_row0 = row0;
    b->ro_hold = hold;
    b->ro_H = H;
    b->ro_ckpt = ckpt_every;
    b->ro_t0 = b->host_t;
    b->ro_valid = false;
    for (int c = 0; c < b->n_classes; ++c) {
        AdjArgs A = adj_args(b, c);
        A.pos = (char*)pos_out + P * 3 * b->pad_off[c];
        A.rd = b->slot;
        A.wr = 1 - b->slot;
        A.advance = (c == b->n_classes - 1) ? H : 0;
        hipError_t e;
        if (b->prec == MGX_FP32)
            e = launch_rollout_fwd<float>(A, b->h_class_f[c], b->m[c], class_shaped(b, c), b->stream);
        else
            e = launch_rollout_fwd<double>(A, b->h_class_d[c], b->m[c], class_shaped(b, c), b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "rollout forward launch");
    }
    b->slot = 1 - b->slot;
    b->host_t += H;
    b->ro_valid = true;
    return MGX_OK;
}

extern "C" mgx_status mgx_rollout_forward(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                          int32_t H, int32_t ckpt_every, void* pos_out) {
    return rollout_forward(b, actions, n_rows, row0, hold, H, ckpt_every, pos_out, false);
}

extern "C" mgx_status mgx_rollout_forward_static(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0,
                                                 int32_t hold, int32_t H, int32_t ckpt_every, void* pos_out) {
    return rollout_forward(b, actions, n_rows, row0, hold, H, ckpt_every, pos_out, true);
}

extern "C" mgx_status mgx_rollout_backward(mgx_batch* b, const void* dpos, void* dactions, void* dparams) {
    if (!b) return fail(MGX_E_INVALID, "batch is NULL");
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!b->ro_valid) return fail(MGX_E_STATE, "no forward rollout recorded");
    if (!dpos) return fail(MGX_E_INVALID, "dpos is NULL");
    if (b->ro_static_gen) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_gen[b->device] != b->ro_static_gen)
            return fail(MGX_E_STATE, "a later mgx_rollout_forward_static on this GPU overwrote the checkpoints");
    }
    hipDevice_guard guard(b->device);
    const size_t P = (size_t)b->prec;
    for (int c = 0; c < b->n_classes; ++c) {
        AdjArgs A = adj_args(b, c);
        A.pos = (char*)dpos + P * 3 * b->pad_off[c];
        A.dactions = dactions ? (char*)dactions + P * b->act_off[c] : nullptr;
        A.dparams = dparams ? (char*)dparams + P * 18 * b->pad_off[c] : nullptr;
        hipError_t e;
        if (b->prec == MGX_FP32)
            e = launch_rollout_bwd<float>(A, b->h_class_f[c], b->m[c], class_shaped(b, c), b->stream);
        else
            e = launch_rollout_bwd<double>(A, b->h_class_d[c], b->m[c], class_shaped(b, c), b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "rollout backward launch");
    }
    return MGX_OK;
}

// ----------------------------------------------------------------------------- host check

template <int M>
static void host_vjp(const ClassT<double>& C, const EnvT<double>& E, const double* state, const double* a,
                     const double* xbar_in, double* state_out, double* xbar_out, double* abar, double* gp) {
    double IA2[3], Brb[3];
    for (int j = 0; j < 3; ++j) {
        IA2[j] = C.inertia[j] + E.A[3 + j];
        Brb[j] = E.buoy * C.rb[j];
    }
    StateT<double, M> s, s1, xb;
    auto unpack = [](const double* x, StateT<double, M>& o) {
        for (int j = 0; j < 3; ++j) o.p[j] = x[j];
        for (int j = 0; j < 4; ++j) o.q[j] = x[3 + j];
        for (int j = 0; j < 6; ++j) o.nu[j] = x[7 + j];
        for (int i = 0; i < M; ++i) o.n[i] = x[13 + i];
    };
    auto pack = [](const StateT<double, M>& o, double* x) {
        for (int j = 0; j < 3; ++j) x[j] = o.p[j];
        for (int j = 0; j < 4; ++j) x[3 + j] = o.q[j];
        for (int j = 0; j < 6; ++j) x[7 + j] = o.nu[j];
        for (int i = 0; i < M; ++i) x[13 + i] = o.n[i];
    };
    unpack(state, s);
    s1 = s;
    double ac[M];
    for (int i = 0; i < M; ++i) ac[i] = clip1(a[i]);
    if (C.shaped)
        step_body<double, M, false, true>(C, E, IA2, Brb, s1, ac);
    else
        step_body<double, M, false, false>(C, E, IA2, Brb, s1, ac);
    pack(s1, state_out);
    unpack(xbar_in, xb);
    double gdL[6] = {0}, gdQ[6] = {0}, gA[6] = {0}, gDt[6] = {0};
    if (C.shaped)
        step_vjp<double, M, true>(C, E, IA2, Brb, s, ac, xb, abar, gdL, gdQ, gA, gDt);
    else
        step_vjp<double, M, false>(C, E, IA2, Brb, s, ac, xb, abar, gdL, gdQ, gA, gDt);
    pack(xb, xbar_out);
    for (int j = 0; j < 6; ++j) {
        gp[j] = gdL[j];
        gp[6 + j] = gdQ[j];
        gp[12 + j] = gA[j];
        gp[18 + j] = gDt[j];
    }
}

extern "C" mgx_status mgx_host_step_vjp(int32_t m, uint32_t batch_flags, const double* cls, const double* rec,
                                        const double* state, const double* actions, const double* xbar_in,
                                        double* state_out, double* xbar_out, double* abar_out, double* gparams_out) {
    if (m < 1 || m > 8) return fail(MGX_E_INVALID, "m=%d outside [1,8]", m);
    if (!cls || !rec || !state || !actions || !xbar_in || !state_out || !xbar_out || !abar_out || !gparams_out)
        return fail(MGX_E_INVALID, "NULL argument");
    ClassT<double> C;
    std::memset(&C, 0, sizeof C);
    const double* c = cls;
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < kMaxThr; ++i) C.Bk[j][i] = *c++;
    for (int i = 0; i < kMaxThr; ++i) C.alpha[i] = *c++;
    int shaped = 0;
    for (int i = 0; i < kMaxThr; ++i) {
        C.dz[i] = *c++;
        shaped |= (i < m && C.dz[i] > 0.0);
    }
    for (int j = 0; j < 3; ++j) C.inertia[j] = *c++;
    for (int j = 0; j < 3; ++j) C.rb[j] = *c++;
    C.g0 = *c++;
    C.dt = *c++;
    for (int i = 0; i < kMaxThr; ++i) {
        C.rev[i] = *c++;
        shaped |= (i < m && C.rev[i] != 1.0);
    }
    C.inv_dt = 1.0 / C.dt;
    C.half_dt = 0.5 * C.dt;
    C.m = m;
    C.flags = batch_flags;
    C.shaped = shaped;
    EnvT<double> E;
    for (int j = 0; j < 6; ++j) {
        E.dtMinv[j] = rec[kRecDtMinv + j];
        E.A[j] = rec[kRecAdded + j];
        E.dL[j] = rec[kRecDlin + j];
        E.dQ[j] = rec[kRecDquad + j];
    }
    E.mass = rec[kRecMass];
    E.wmb = rec[kRecWmB];
    E.buoy = rec[kRecBuoy];
    for (int j = 0; j < 3; ++j) E.Vc[j] = rec[kRecCurrent + j];
    set_amc(E, C.flags);
    switch (m) {
        case 1: host_vjp<1>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 2: host_vjp<2>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 3: host_vjp<3>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 4: host_vjp<4>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 5: host_vjp<5>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 6: host_vjp<6>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        case 7: host_vjp<7>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
        default: host_vjp<8>(C, E, state, actions, xbar_in, state_out, xbar_out, abar_out, gparams_out); break;
    }
    return MGX_OK;
}
