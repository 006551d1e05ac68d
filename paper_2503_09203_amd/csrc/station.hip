// Station-keeping task on top of the step (Sec. IV-B): per task step, every environment
// advances under its held command, then its observation, reward and termination are
// formed in the same kernel, and an environment whose episode ended starts the next one
// at once (its state and target drawn again), so the batch never leaves the device
// between policy calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "env_loop.hpp"
#include "kernels.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"

namespace mgx {

constexpr uint32_t kStreamTask = 8u;

struct StationConsts {
    double box, tilt0, v0;                                // episode start draws
    double inv_sigma, w_att, w_act_m, d_max, cos_tilt;    // reward (w_act / m) and termination
    int32_t max_steps, substeps;
    uint64_t seed;
};

template <typename T>
// The first 64 bytes hold what the step kernel's loads need (one scalar cache line).
struct StationArgs {
    T* state;
    const T* rec;
    const T* act;        // command rows, class segment: row k at act + k * act_stride
    T* tgt;              // [7][npad]: p*, q*
    int32_t* ep;         // [npad] episode index
    int32_t* et;         // [npad] steps taken in the episode
    int32_t npad, nvalid;
    uint8_t* restart;    // [npad] 1 where an episode started during the launch
    T* obs;              // per step [13+m][npad], row k at obs + k * obs_stride
    T* final_obs;        // the same or NULL; written for lanes whose episode ended
    T* reward;           // per step [npad], row k at reward + k * flag_stride
    uint8_t* term;       // per step [npad], likewise
    uint8_t* trunc;      // per step [npad], likewise
    int64_t act_stride, obs_stride, flag_stride;
    int32_t n_steps;     // task steps in this launch
    int64_t env_off;
    StationConsts P;
};

template <typename T>
struct StationLaunch {
    StationArgs<T> a;
    ClassT<T> cls;
};

// Episode start of global env g, episode k, in double: target p*, q* (a pure yaw) and the
// start attitude q0 = q_z(yaw) q_y(pitch) q_x(roll) with velocities nu0; p = 0, n = 0.
__device__ void episode_draw(const StationConsts& P, uint64_t g, uint32_t k, double tgt[7], double q0[4],
                             double nu0[6]) {
    double u[14];
    for (int j = 0; j < 7; ++j) {
        uint32_t c[4] = {(uint32_t)g, k, (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)P.seed, kStreamTask << 24);
        u[2 * j] = u53(c[0], c[1]);
        u[2 * j + 1] = u53(c[2], c[3]);
    }
    for (int j = 0; j < 3; ++j) tgt[j] = P.box * (2.0 * u[j] - 1.0);
    const double ht = 0.5 * (M_PI * (2.0 * u[3] - 1.0));
    tgt[3] = cos(ht);
    tgt[4] = 0.0;
    tgt[5] = 0.0;
    tgt[6] = sin(ht);
    const double hy = 0.5 * (M_PI * (2.0 * u[4] - 1.0));
    const double hr = 0.5 * (P.tilt0 * (2.0 * u[5] - 1.0));
    const double hp = 0.5 * (P.tilt0 * (2.0 * u[6] - 1.0));
    const double cy = cos(hy), sy = sin(hy), cp = cos(hp), sp = sin(hp), cr = cos(hr), sr = sin(hr);
    q0[0] = cy * cp * cr + sy * sp * sr;
    q0[1] = cy * cp * sr - sy * sp * cr;
    q0[2] = cy * sp * cr + sy * cp * sr;
    q0[3] = sy * cp * cr - cy * sp * sr;
    for (int j = 0; j < 6; ++j) nu0[j] = P.v0 * (2.0 * u[7 + j] - 1.0);
}

template <typename T, int M>
__device__ __forceinline__ void start_state(const StationConsts& P, uint64_t g, uint32_t k, StateT<T, M>& s,
                                            T tg[7]) {
    double t[7], q0[4], nu0[6];
    episode_draw(P, g, k, t, q0, nu0);
#pragma unroll
    for (int j = 0; j < 7; ++j) tg[j] = (T)t[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) s.p[j] = T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) s.q[j] = (T)q0[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) s.nu[j] = (T)nu0[j];
#pragma unroll
    for (int i = 0; i < M; ++i) s.n[i] = T(0);
}

// Attitude error q*^-1 q, scalar part made >= 0.
template <typename T>
__device__ __forceinline__ void attitude_error(const T q[4], const T t[4], T e[4]) {
    e[0] = t[0] * q[0] + t[1] * q[1] + t[2] * q[2] + t[3] * q[3];
    e[1] = t[0] * q[1] - t[1] * q[0] - t[2] * q[3] + t[3] * q[2];
    e[2] = t[0] * q[2] + t[1] * q[3] - t[2] * q[0] - t[3] * q[1];
    e[3] = t[0] * q[3] - t[1] * q[2] + t[2] * q[1] - t[3] * q[0];
    if (e[0] < T(0)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] = -e[j];
    }
}

// Observation in the state's layout: R(q)^T (p* - p), the attitude error, nu, n.
template <typename T, int M>
__device__ __forceinline__ void write_obs(T* O, int64_t np, int64_t env, const StateT<T, M>& s, const T tg[7]) {
    const T d0 = tg[0] - s.p[0], d1 = tg[1] - s.p[1], d2 = tg[2] - s.p[2];
    const T w = s.q[0], x = s.q[1], y = s.q[2], z = s.q[3];
    // columns of R(q)
    const T r00 = T(1) - T(2) * (y * y + z * z), r10 = T(2) * (x * y + w * z), r20 = T(2) * (x * z - w * y);
    const T r01 = T(2) * (x * y - w * z), r11 = T(1) - T(2) * (x * x + z * z), r21 = T(2) * (y * z + w * x);
    const T r02 = T(2) * (x * z + w * y), r12 = T(2) * (y * z - w * x), r22 = T(1) - T(2) * (x * x + y * y);
    O[0 * np + env] = r00 * d0 + r10 * d1 + r20 * d2;
    O[1 * np + env] = r01 * d0 + r11 * d1 + r21 * d2;
    O[2 * np + env] = r02 * d0 + r12 * d1 + r22 * d2;
    T e[4];
    attitude_error(s.q, tg + 3, e);
#pragma unroll
    for (int j = 0; j < 4; ++j) O[(3 + j) * np + env] = e[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) O[(7 + j) * np + env] = s.nu[j];
#pragma unroll
    for (int i = 0; i < M; ++i) O[(kStateFixed + i) * np + env] = s.n[i];
}

__device__ __forceinline__ float exp_(float x) { return expf(x); }
__device__ __forceinline__ double exp_(double x) { return exp(x); }

// Episode 0 of every valid slot; observations of every slot.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_station_start(StationArgs<T> A) {
    const int64_t env = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (env >= A.npad) return;
    const int64_t np = A.npad;
    StateT<T, M> s;
    T tg[7];
    if (env < A.nvalid) {
        start_state<T, M>(A.P, (uint64_t)(A.env_off + env), 0u, s, tg);
        store_state<T, M>(A.state, np, env, s);
#pragma unroll
        for (int j = 0; j < 7; ++j) A.tgt[j * np + env] = tg[j];
    } else {
        load_state<T, M>(A.state, np, env, s);
#pragma unroll
        for (int j = 0; j < 7; ++j) tg[j] = A.tgt[j * np + env];
    }
    A.ep[env] = 0;
    A.et[env] = 0;
    A.restart[env] = env < A.nvalid ? 1 : 0;
    if (A.obs) write_obs<T, M>(A.obs, np, env, s, tg);
}

// Restarts of the lanes in `need` (a mask over the wave), one lane at a time with its draw
// spread over the wave: lane j < 7 runs generator call j, lanes 1..4 each take one sine and
// cosine, and lane shuffles bring the values to the restarting lane. The arithmetic is
// that of episode_draw, value for value. A step ends few episodes per wave, and each then
// costs a few hundred instructions of the wave instead of the draw's serial chain of about
// a thousand (seven generator calls, eight double-precision sines and cosines), which
// would hold the whole wave, and so the launch, at one wave per SIMD.
constexpr int kSpreadRestarts = 3;

template <typename T, int M>
__device__ __forceinline__ void restart_spread(const StationConsts& P, uint64_t need, uint32_t g, uint32_t k,
                                               StateT<T, M>& s, T tg[7]) {
    const int lane = __lane_id();
    while (need) {
        const int src = __ffsll((unsigned long long)need) - 1;
        need &= need - 1;
        uint32_t c[4] = {__shfl(g, src), __shfl(k, src), (uint32_t)(lane < 7 ? lane : 0), 0u};
        philox4x32_10(c, (uint32_t)P.seed, kStreamTask << 24);
        const double a = 2.0 * u53(c[0], c[1]) - 1.0;  // 2 u[2j] - 1 on lane j
        const double b = 2.0 * u53(c[2], c[3]) - 1.0;  // 2 u[2j+1] - 1
        const double b2 = __shfl(b, 2);
        // half-angles: target yaw (u3), yaw (u4), pitch (u6), roll (u5)
        const double ang = lane == 1   ? 0.5 * (M_PI * b)
                           : lane == 2 ? 0.5 * (M_PI * a)
                           : lane == 3 ? 0.5 * (P.tilt0 * a)
                                       : 0.5 * (P.tilt0 * b2);
        const double cs = cos(ang), sn = sin(ang);
        const double scale = lane < 2 ? P.box : P.v0;  // target position on lanes 0-1, velocities on 3-6
        const double xa = scale * a, xb = scale * b;
        const double px = __shfl(xa, 0), py = __shfl(xb, 0), pz = __shfl(xa, 1);
        const double ct = __shfl(cs, 1), st = __shfl(sn, 1);
        const double cy = __shfl(cs, 2), sy = __shfl(sn, 2), cp = __shfl(cs, 3), sp = __shfl(sn, 3);
        const double cr = __shfl(cs, 4), sr = __shfl(sn, 4);
        const double v[6] = {__shfl(xb, 3), __shfl(xa, 4), __shfl(xb, 4), __shfl(xa, 5), __shfl(xb, 5), __shfl(xa, 6)};
        if (lane == src) {
            tg[0] = (T)px;
            tg[1] = (T)py;
            tg[2] = (T)pz;
            tg[3] = (T)ct;
            tg[4] = T(0);
            tg[5] = T(0);
            tg[6] = (T)st;
#pragma unroll
            for (int j = 0; j < 3; ++j) s.p[j] = T(0);
            s.q[0] = (T)(cy * cp * cr + sy * sp * sr);
            s.q[1] = (T)(cy * cp * sr - sy * sp * cr);
            s.q[2] = (T)(cy * sp * cr + sy * cp * sr);
            s.q[3] = (T)(sy * cp * cr - cy * sp * sr);
#pragma unroll
            for (int j = 0; j < 6; ++j) s.nu[j] = (T)v[j];
#pragma unroll
            for (int i = 0; i < M; ++i) s.n[i] = T(0);
        }
    }
}

// n_steps task steps of one class segment in one launch: the state, record and target stay
// in registers from step to step, the next command row is fetched during the current step,
// and each step's observation, reward and flags go to their own output row. kMulti = false
// is the one-step form (a Gym step), compiled without the loop.
template <typename T, int M, bool kShaped, bool kFins, bool kPayload, bool kMulti>
__global__ void __launch_bounds__(256) k_station_step(StationLaunch<T> L) {
    const StationArgs<T>& A = L.a;
    const int64_t env = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = A.npad;
    // Every lane loads everything, with no branch ahead of its loads: lanes past the segment
    // (whole waves) at its last slot, padding slots as they are (they hold a valid state,
    // parameter set and command). Behind a branch on the kernel arguments, each group of
    // loads waited for another argument fetch; a one-step launch took about 8 us.
    // Every lane also takes the steps (the commands' loads otherwise moved behind the branch
    // that left padding lanes out): padding lanes store and report nothing and never end an
    // episode (they stay in the wave for the restarts); lanes past the segment write nothing.
    const bool live = env < np;
    const bool valid = env < A.nvalid;
    const int64_t el = live ? env : np - 1;
    StateT<T, M> s;
    load_state<T, M>(A.state, np, el, s);
    // classes with fins carry the attitude's low-order words through the launch (float)
    constexpr bool kComp = kFins && std::is_same<T, float>::value;
    StateLo<T> lo;
#pragma unroll
    for (int j = 0; j < 4; ++j) lo.q[j] = T(0);
    T tg[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) tg[j] = A.tgt[j * np + el];
    const ClassT<T> C = class_in_vgpr<T, M, kFins>(L.cls);
    EnvT<T> E;
    T IA2[3], Brb[3];
    bool restarted = false;
    T nxt[M];
    load_record<T, kPayload>(A.rec, np, el, C.flags, E);
    int32_t ep = A.ep[el];
    int32_t et = A.et[el];
#pragma unroll
    for (int i = 0; i < M; ++i) nxt[i] = A.act[i * np + el];
    env_prologue<T, kPayload>(C, E, IA2, Brb);
    const int32_t n_steps = kMulti ? A.n_steps : 1;
    for (int32_t k = 0; k < n_steps; ++k) {
        T r = T(0);
        bool term = false, trunc = false;
        {
            T a[M];
#pragma unroll
            for (int i = 0; i < M; ++i) a[i] = clip1(nxt[i]);
            if constexpr (kMulti) {
                // the next row, clamped to the last (a load guarded per step would make the
                // compiler wait for it before the step)
                const T* an = A.act + (int64_t)(k + 1 < n_steps ? k + 1 : k) * A.act_stride + el;
#pragma unroll
                for (int i = 0; i < M; ++i) nxt[i] = an[i * np];
            }
            // substeps >= 1 (checked at creation): the first step is unconditional, so no
            // branch on the argument stands between the record's loads and their use
            int j = 0;
            do {
                step_body<T, M, false, kShaped, kFins, kPayload, kComp>(C, E, IA2, Brb, s, a, nullptr, &lo);
            } while (++j < A.P.substeps);
            float st[kStats];  // launch statistics are not kept by the task
            renorm_attitude<T, M>(s, st);

            // reward and termination on the state the transition ends in
            bool fin = true;
#pragma unroll
            for (int j = 0; j < 3; ++j) fin &= finite_(s.p[j]);
#pragma unroll
            for (int j = 0; j < 4; ++j) fin &= finite_(s.q[j]);
#pragma unroll
            for (int j = 0; j < 6; ++j) fin &= finite_(s.nu[j]);
#pragma unroll
            for (int i = 0; i < M; ++i) fin &= finite_(s.n[i]);
            const T d0 = tg[0] - s.p[0], d1 = tg[1] - s.p[1], d2 = tg[2] - s.p[2];
            const T d = sqrt_(d0 * d0 + d1 * d1 + d2 * d2);
            T e[4];
            attitude_error(s.q, tg + 3, e);
            T a2 = T(0);
#pragma unroll
            for (int i = 0; i < M; ++i) a2 += a[i] * a[i];
            const T up = T(1) - T(2) * (s.q[1] * s.q[1] + s.q[2] * s.q[2]);
            r = exp_(-d * (T)A.P.inv_sigma) - (T)A.P.w_att * (T(1) - e[0] * e[0]) - (T)A.P.w_act_m * a2;
            term = valid && (!fin || d > (T)A.P.d_max || up < (T)A.P.cos_tilt);
            if (!fin || !valid) r = T(0);
            et += valid ? 1 : 0;
            trunc = valid && et >= A.P.max_steps;
        }
        const bool done = term || trunc;
        if (done) {
            if (A.final_obs) write_obs<T, M>(A.final_obs + (int64_t)k * A.obs_stride, np, env, s, tg);
            ++ep;
            et = 0;
            restarted = true;
#pragma unroll
            for (int j = 0; j < 4; ++j) lo.q[j] = T(0);
        }
        const uint64_t need = __ballot(done);
        if (need) {
            if (__popcll(need) <= kSpreadRestarts)
                restart_spread<T, M>(A.P, need, (uint32_t)(A.env_off + env), (uint32_t)ep, s, tg);
            else if (done)
                start_state<T, M>(A.P, (uint64_t)(A.env_off + env), (uint32_t)ep, s, tg);
        }
        if (live) {
            write_obs<T, M>(A.obs + (int64_t)k * A.obs_stride, np, env, s, tg);
            const int64_t fo = (int64_t)k * A.flag_stride + env;
            A.reward[fo] = r;
            A.term[fo] = term ? 1 : 0;
            A.trunc[fo] = trunc ? 1 : 0;
        }
    }
    if (valid) {
        store_state<T, M>(A.state, np, env, s);
        if (restarted) {
#pragma unroll
            for (int j = 0; j < 7; ++j) A.tgt[j * np + env] = tg[j];
        }
        A.ep[env] = ep;
        A.et[env] = et;
    }
    if (live) A.restart[env] = restarted ? 1 : 0;
}

template <typename T, int M, bool kMulti>
static void launch_station_body(const StationLaunch<T>& L, bool shaped, bool fins, bool payload, hipStream_t s) {
    const dim3 grid((unsigned)((L.a.npad + 255) / 256)), block(256);
    if (payload && fins)
        hipLaunchKernelGGL((k_station_step<T, M, true, true, true, kMulti>), grid, block, 0, s, L);
    else if (payload)
        hipLaunchKernelGGL((k_station_step<T, M, true, false, true, kMulti>), grid, block, 0, s, L);
    else if (fins)
        hipLaunchKernelGGL((k_station_step<T, M, true, true, false, kMulti>), grid, block, 0, s, L);
    else if (shaped)
        hipLaunchKernelGGL((k_station_step<T, M, true, false, false, kMulti>), grid, block, 0, s, L);
    else
        hipLaunchKernelGGL((k_station_step<T, M, false, false, false, kMulti>), grid, block, 0, s, L);
}

template <typename T, int M>
static void launch_station_m(const StationLaunch<T>& L, bool shaped, bool fins, bool payload, hipStream_t s) {
    if (L.a.n_steps > 1)
        launch_station_body<T, M, true>(L, shaped, fins, payload, s);
    else
        launch_station_body<T, M, false>(L, shaped, fins, payload, s);
}

template <typename T>
static hipError_t launch_station(const StationLaunch<T>& L, int m, hipStream_t s) {
    const bool shaped = L.cls.shaped != 0, fins = L.cls.fin_mask != 0, payload = L.cls.payload != 0;
    switch (m) {
        case 1: launch_station_m<T, 1>(L, shaped, fins, payload, s); break;
        case 2: launch_station_m<T, 2>(L, shaped, fins, payload, s); break;
        case 3: launch_station_m<T, 3>(L, shaped, fins, payload, s); break;
        case 4: launch_station_m<T, 4>(L, shaped, fins, payload, s); break;
        case 5: launch_station_m<T, 5>(L, shaped, fins, payload, s); break;
        case 6: launch_station_m<T, 6>(L, shaped, fins, payload, s); break;
        case 7: launch_station_m<T, 7>(L, shaped, fins, payload, s); break;
        case 8: launch_station_m<T, 8>(L, shaped, fins, payload, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_start(const StationArgs<T>& A, int m, hipStream_t s) {
    const dim3 grid((unsigned)((A.npad + 255) / 256)), block(256);
    switch (m) {
        case 1: hipLaunchKernelGGL((k_station_start<T, 1>), grid, block, 0, s, A); break;
        case 2: hipLaunchKernelGGL((k_station_start<T, 2>), grid, block, 0, s, A); break;
        case 3: hipLaunchKernelGGL((k_station_start<T, 3>), grid, block, 0, s, A); break;
        case 4: hipLaunchKernelGGL((k_station_start<T, 4>), grid, block, 0, s, A); break;
        case 5: hipLaunchKernelGGL((k_station_start<T, 5>), grid, block, 0, s, A); break;
        case 6: hipLaunchKernelGGL((k_station_start<T, 6>), grid, block, 0, s, A); break;
        case 7: hipLaunchKernelGGL((k_station_start<T, 7>), grid, block, 0, s, A); break;
        case 8: hipLaunchKernelGGL((k_station_start<T, 8>), grid, block, 0, s, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mgx

using namespace mgx;

struct mgx_station {
    mgx_batch* batch = nullptr;
    mgx_station_desc desc{};
    StationConsts P{};
    void* d_tgt = nullptr;       // [7][npad] per class segment, at 7 * pad_off[c]
    int32_t* d_ep = nullptr;     // [npad_total]
    int32_t* d_et = nullptr;     // [npad_total]
    uint8_t* d_restart = nullptr;  // [npad_total]: an episode started in the last reset or step call
    bool started = false;
};

#define HIP_TRY_ST(b, call)                                       \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((b), e_, #call);    \
    } while (0)

static void free_station(mgx_station* s) {
    if (s->d_tgt) (void)hipFree(s->d_tgt);
    if (s->d_ep) (void)hipFree(s->d_ep);
    if (s->d_et) (void)hipFree(s->d_et);
    if (s->d_restart) (void)hipFree(s->d_restart);
    s->d_tgt = nullptr;
    s->d_ep = s->d_et = nullptr;
    s->d_restart = nullptr;
}

template <typename T>
static StationArgs<T> station_args(mgx_station* st, int c) {
    mgx_batch* b = st->batch;
    StationArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.state = (T*)b->seg_state(c);
    a.rec = (const T*)b->seg_rec(c);
    a.tgt = (T*)st->d_tgt + 7 * b->pad_off[c];
    a.ep = st->d_ep + b->pad_off[c];
    a.et = st->d_et + b->pad_off[c];
    a.restart = st->d_restart + b->pad_off[c];
    a.npad = (int32_t)b->npad[c];
    a.nvalid = (int32_t)b->n[c];
    a.env_off = b->env_off[c];
    a.P = st->P;
    a.P.w_act_m = st->desc.w_act / b->m[c];
    return a;
}

extern "C" mgx_status mgx_station_create(mgx_batch* b, const mgx_station_desc* d, mgx_station** out) {
    if (!b || !d || !out) return fail(MGX_E_INVALID, "NULL argument");
    *out = nullptr;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    const double pi = M_PI;
    if (!(d->target_box >= 0 && d->target_box <= 1e4)) return fail(MGX_E_INVALID, "target_box outside [0, 1e4]");
    if (!(d->tilt0 >= 0 && d->tilt0 <= pi / 2)) return fail(MGX_E_INVALID, "tilt0 outside [0, pi/2]");
    if (!(d->v0 >= 0 && d->v0 <= 100)) return fail(MGX_E_INVALID, "v0 outside [0, 100]");
    if (!(d->sigma_p > 0 && std::isfinite(d->sigma_p))) return fail(MGX_E_INVALID, "sigma_p must be > 0");
    if (!(d->w_att >= 0 && std::isfinite(d->w_att)) || !(d->w_act >= 0 && std::isfinite(d->w_act)))
        return fail(MGX_E_INVALID, "w_att and w_act must be finite and >= 0");
    if (!(d->d_max > 0)) return fail(MGX_E_INVALID, "d_max must be > 0");
    if (!(d->tilt_max > 0 && d->tilt_max <= pi)) return fail(MGX_E_INVALID, "tilt_max outside (0, pi]");
    if (d->max_steps < 1) return fail(MGX_E_INVALID, "max_steps must be >= 1");
    if (d->substeps < 1 || d->substeps > 1000) return fail(MGX_E_INVALID, "substeps outside [1, 1000]");
    hipDevice_guard g(b->device);
    mgx_station* s = new (std::nothrow) mgx_station();
    if (!s) return fail(MGX_E_NOMEM, "host allocation");
    s->batch = b;
    s->desc = *d;
    s->P.box = d->target_box;
    s->P.tilt0 = d->tilt0;
    s->P.v0 = d->v0;
    s->P.inv_sigma = 1.0 / d->sigma_p;
    s->P.w_att = d->w_att;
    s->P.d_max = d->d_max;
    s->P.cos_tilt = std::cos(d->tilt_max);
    s->P.max_steps = d->max_steps;
    s->P.substeps = d->substeps;
    const size_t P = (size_t)b->prec, N = (size_t)b->npad_total;
    hipError_t e = hipMalloc(&s->d_tgt, 7 * N * P);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_ep, N * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_et, N * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_restart, N);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_restart, 0, N, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_tgt, 0, 7 * N * P, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_ep, 0, N * sizeof(int32_t), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_et, 0, N * sizeof(int32_t), b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        free_station(s);
        delete s;
        return e == hipErrorOutOfMemory ? fail(MGX_E_NOMEM, "station buffers") : hip_fail(b, e, "station buffers");
    }
    ++b->n_stations;
    *out = s;
    return MGX_OK;
}

extern "C" mgx_status mgx_station_destroy(mgx_station* s) {
    if (!s) return MGX_OK;
    mgx_batch* b = s->batch;
    hipDevice_guard g(b->device);
    (void)hipStreamSynchronize(b->stream);
    free_station(s);
    --b->n_stations;
    delete s;
    return MGX_OK;
}

extern "C" mgx_status mgx_station_reset(mgx_station* s, uint64_t seed, void* obs) {
    if (!s) return fail(MGX_E_INVALID, "station is NULL");
    mgx_batch* b = s->batch;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    hipDevice_guard g(b->device);
    s->P.seed = seed;
    const size_t P = (size_t)b->prec;
    for (int c = 0; c < b->n_classes; ++c) {
        hipError_t e;
        if (b->prec == MGX_FP32) {
            StationArgs<float> a = station_args<float>(s, c);
            a.obs = obs ? (float*)((char*)obs + P * b->state_off[c]) : nullptr;
            e = launch_start<float>(a, b->m[c], b->stream);
        } else {
            StationArgs<double> a = station_args<double>(s, c);
            a.obs = obs ? (double*)((char*)obs + P * b->state_off[c]) : nullptr;
            e = launch_start<double>(a, b->m[c], b->stream);
        }
        if (e != hipSuccess) return hip_fail(b, e, "station start launch");
    }
    s->started = true;
    return MGX_OK;
}

extern "C" mgx_status mgx_station_step(mgx_station* s, const void* actions, int32_t n_steps, void* obs, void* reward,
                                       uint8_t* terminated, uint8_t* truncated, void* final_obs) {
    if (!s) return fail(MGX_E_INVALID, "station is NULL");
    mgx_batch* b = s->batch;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!b->params_set) return fail(MGX_E_STATE, "mgx_batch_set_params has not been called");
    if (!s->started) return fail(MGX_E_STATE, "mgx_station_reset has not been called");
    if (!actions || !obs || !reward || !terminated || !truncated)
        return fail(MGX_E_INVALID, "actions, obs, reward, terminated and truncated are required");
    if (n_steps < 1) return fail(MGX_E_INVALID, "n_steps must be >= 1");
    hipDevice_guard g(b->device);
    const size_t P = (size_t)b->prec;
    for (int c = 0; c < b->n_classes; ++c) {
        const int64_t so = b->state_off[c], po = b->pad_off[c];
        hipError_t e;
        if (b->prec == MGX_FP32) {
            StationLaunch<float> L{station_args<float>(s, c), b->h_class_f[c]};
            L.a.act = (const float*)((const char*)actions + P * b->act_off[c]);
            L.a.obs = (float*)obs + so;
            L.a.final_obs = final_obs ? (float*)final_obs + so : nullptr;
            L.a.reward = (float*)reward + po;
            L.a.term = terminated + po;
            L.a.trunc = truncated + po;
            L.a.act_stride = b->row_elems;
            L.a.obs_stride = b->state_elems;
            L.a.flag_stride = b->npad_total;
            L.a.n_steps = n_steps;
            e = launch_station<float>(L, b->m[c], b->stream);
        } else {
            StationLaunch<double> L{station_args<double>(s, c), b->h_class_d[c]};
            L.a.act = (const double*)((const char*)actions + P * b->act_off[c]);
            L.a.obs = (double*)obs + so;
            L.a.final_obs = final_obs ? (double*)final_obs + so : nullptr;
            L.a.reward = (double*)reward + po;
            L.a.term = terminated + po;
            L.a.trunc = truncated + po;
            L.a.act_stride = b->row_elems;
            L.a.obs_stride = b->state_elems;
            L.a.flag_stride = b->npad_total;
            L.a.n_steps = n_steps;
            e = launch_station<double>(L, b->m[c], b->stream);
        }
        if (e != hipSuccess) return hip_fail(b, e, "station step launch");
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_station_episodes(mgx_station* s, int32_t* episode, int32_t* steps) {
    if (!s || !episode || !steps) return fail(MGX_E_INVALID, "NULL argument");
    mgx_batch* b = s->batch;
    hipDevice_guard g(b->device);
    std::vector<int32_t> ep((size_t)b->npad_total), et((size_t)b->npad_total);
    HIP_TRY_ST(b, hipMemcpyAsync(ep.data(), s->d_ep, sizeof(int32_t) * ep.size(), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY_ST(b, hipMemcpyAsync(et.data(), s->d_et, sizeof(int32_t) * et.size(), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY_ST(b, hipStreamSynchronize(b->stream));
    for (int c = 0; c < b->n_classes; ++c)
        for (int64_t i = 0; i < b->n[c]; ++i) {
            episode[b->env_off[c] + i] = ep[(size_t)(b->pad_off[c] + i)];
            steps[b->env_off[c] + i] = et[(size_t)(b->pad_off[c] + i)];
        }
    return MGX_OK;
}

extern "C" mgx_status mgx_station_resample(mgx_station* s, const mgx_dr_spec* spec, const double* nominal,
                                           uint64_t seed) {
    if (!s) return fail(MGX_E_INVALID, "station is NULL");
    mgx_batch* b = s->batch;
    if (b->faulted) return fail(MGX_E_STATE, "batch faulted by an earlier device error");
    if (!s->started) return fail(MGX_E_STATE, "mgx_station_reset has not been called");
    return resample_masked(b, spec, nominal, s->d_restart, s->d_ep, seed);
}
