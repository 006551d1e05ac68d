// Continuous-batching server: a scheduler thread, a device arena sized to the memory
// budget, and one persistent launch per iteration over the tiles of every active request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>

#include <sys/prctl.h>
#include <vector>

#include "env_loop.hpp"
#include "kernels.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"

namespace mgx {

// One 64-environment tile of one session for one iteration.
struct ServeTile {
    float* state;        // session segment [13+m][npad]
    const float* rec;    // [30][npad]
    int64_t t0;          // session step at the start of this iteration
    uint64_t seed;       // the session's action stream
    const float* act;    // the request's commands [rows][m][nvalid], or null (generated from seed)
    int64_t act_row0;    // hold interval of the request's row 0
    int32_t npad, env0, steps, hold;
    int32_t cls, nvalid, pad0, pad1;
};

struct ServeArgs {
    const ServeTile* tiles;
    const ClassT<float>* cls;
    int32_t n_tiles, n_classes;
    DevMisc* misc;
    int32_t rd, wr;
};

// Commands of one hold interval for session-local env e, row r (the generator of
// mgx_gen_actions).
template <int M>
__device__ __forceinline__ void session_actions(uint64_t seed, int64_t e, int64_t r, float a[M]) {
#pragma unroll
    for (int b = 0; b < M; b += 4) {
        uint32_t c[4] = {(uint32_t)e, (uint32_t)r, (uint32_t)(b / 4), 0u};
        philox4x32_10(c, (uint32_t)seed, kStreamAction << 24);
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (b + w < M) a[b + w] = action_from_word(c[w]);
    }
}

// Commands of hold interval `row`: the request's own (clipped to [-1, 1]; padded lanes 0),
// or the session's generated stream.
template <int M>
__device__ __forceinline__ void tile_actions(const ServeTile& T, int64_t e, int64_t row, float a[M]) {
    if (T.act) {
        const int64_t n = T.nvalid;
        const float* src = T.act + (row - T.act_row0) * M * n + e;
#pragma unroll
        for (int i = 0; i < M; ++i) a[i] = e < n ? clip1(src[i * n]) : 0.0f;
    } else {
        session_actions<M>(T.seed, e, row, a);
    }
}

template <int M, bool kShaped>
__device__ __forceinline__ void serve_env(const ServeTile& T, const ClassT<float>& Cs, int64_t e) {
    const ClassT<float> C = class_in_vgpr<float, M>(Cs);
    const int64_t np = T.npad;
    float* S = T.state;
    const float* Rc = T.rec;
    StateT<float, M> s;
#pragma unroll
    for (int j = 0; j < 3; ++j) s.p[j] = S[j * np + e];
#pragma unroll
    for (int j = 0; j < 4; ++j) s.q[j] = S[(3 + j) * np + e];
#pragma unroll
    for (int j = 0; j < 6; ++j) s.nu[j] = S[(7 + j) * np + e];
#pragma unroll
    for (int i = 0; i < M; ++i) s.n[i] = S[(kStateFixed + i) * np + e];
    EnvT<float> E;
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
    set_amc(E, C.flags);
    float IA2[3], Brb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        IA2[j] = C.inertia[j] + E.A[3 + j];
        Brb[j] = E.buoy * C.rb[j];
    }
    const int64_t hold = T.hold;
    int64_t row = T.t0 / hold;
    int phase = (int)(T.t0 - row * hold);
    float a[M];
    tile_actions<M>(T, e, row, a);
    for (int k = 0; k < T.steps; ++k) {
        step_body<float, M, false, kShaped>(C, E, IA2, Brb, s, a);
        if (++phase == hold) {
            phase = 0;
            ++row;
            if (k + 1 < T.steps) tile_actions<M>(T, e, row, a);   // no row past the last step
        }
    }
    {
        float n2 = fma_(s.q[3], s.q[3], fma_(s.q[2], s.q[2], fma_(s.q[1], s.q[1], s.q[0] * s.q[0])));
        if (abs_(n2 - 1.0f) > 1e-6f) {
            double qd[4] = {(double)s.q[0], (double)s.q[1], (double)s.q[2], (double)s.q[3]};
            double inv = 1.0 / sqrt(qd[0] * qd[0] + qd[1] * qd[1] + qd[2] * qd[2] + qd[3] * qd[3]);
#pragma unroll
            for (int j = 0; j < 4; ++j) s.q[j] = (float)(qd[j] * inv);
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) S[j * np + e] = s.p[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) S[(3 + j) * np + e] = s.q[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) S[(7 + j) * np + e] = s.nu[j];
#pragma unroll
    for (int i = 0; i < M; ++i) S[(kStateFixed + i) * np + e] = s.n[i];
}

__device__ __forceinline__ float rfl_f(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }

template <int M>
__device__ __forceinline__ void serve_tile(const ServeTile& T, const ClassT<float>& L, int64_t e) {
    ClassT<float> C;
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int i = 0; i < M; ++i) C.Bk[j][i] = rfl_f(L.Bk[j][i]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        C.alpha[i] = rfl_f(L.alpha[i]);
        C.dz[i] = rfl_f(L.dz[i]);
        C.rev[i] = rfl_f(L.rev[i]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        C.inertia[j] = rfl_f(L.inertia[j]);
        C.rb[j] = rfl_f(L.rb[j]);
    }
    C.g0 = rfl_f(L.g0);
    C.dt = rfl_f(L.dt);
    C.inv_dt = rfl_f(L.inv_dt);
    C.half_dt = rfl_f(L.half_dt);
    C.m = M;
    C.flags = __builtin_amdgcn_readfirstlane(L.flags);
    C.shaped = __builtin_amdgcn_readfirstlane(L.shaped);
    if (C.shaped)
        serve_env<M, true>(T, C, e);
    else
        serve_env<M, false>(T, C, e);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_serve(ServeArgs P) {
    __shared__ ClassT<float> lds_cls[16];
    {
        const uint32_t* src = (const uint32_t*)P.cls;
        uint32_t* dst = (uint32_t*)lds_cls;
        const int nw = P.n_classes * (int)(sizeof(ClassT<float>) / 4);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        prepare_next_slot(P.misc, P.wr);
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t n_waves = gridDim.x * (blockDim.x / kWave);
    // Wave w runs tile w; tiles beyond the grid come from the counter (as in the
    // persistent step kernel, so that the launch does not start behind one atomic).
    uint32_t tile = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    for (;; tile = 0xFFFFFFFFu) {
        if (tile == 0xFFFFFFFFu) {
            uint32_t i = 0;
            if (lane == 0) i = atomicAdd(&P.misc->work[P.rd], 1u);
            tile = n_waves + __builtin_amdgcn_readfirstlane(__shfl(i, 0, kWave));
        }
        if (tile >= (uint32_t)P.n_tiles) break;
        const ServeTile T = P.tiles[tile];
        const int c = __builtin_amdgcn_readfirstlane(T.cls);
        const ClassT<float>& L = lds_cls[c];
        const int64_t e = T.env0 + lane;
        switch (L.m) {
            case 1: serve_tile<1>(T, L, e); break;
            case 2: serve_tile<2>(T, L, e); break;
            case 3: serve_tile<3>(T, L, e); break;
            case 4: serve_tile<4>(T, L, e); break;
            case 5: serve_tile<5>(T, L, e); break;
            case 6: serve_tile<6>(T, L, e); break;
            case 7: serve_tile<7>(T, L, e); break;
            default: serve_tile<8>(T, L, e); break;
        }
    }
}

// New session: record from the class-nominal parameters, seeded state; padded slots at rest.
__global__ void k_session_init(float* state, float* rec, int m, int64_t n, int64_t npad, const ClassDesc64* cls, int ci,
                               const double* nominal, double dt, uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npad) return;
    if (e < n) {
        const double* p = nominal + 23 * ci;
        // the nominal values are validated at server creation and the server runs no payload
        // class, so M is diagonal with positive entries and the record is always valid
        (void)write_record<float>(cls[ci].inertia, cls[ci].g0, dt, p[0], p + 1, p + 7, p + 13, p[19], p + 20, rec,
                                  npad, e);
        seeded_state<float>((uint64_t)e, seed, m, state, npad, e);
    } else {
        for (int j = 0; j < kStateFixed + m; ++j) state[j * npad + e] = (j == 3) ? 1.0f : 0.0f;
        for (int j = 0; j < kRecLen; ++j) rec[j * npad + e] = 0.0f;
    }
}

}  // namespace mgx

using namespace mgx;

namespace {

double now_s() {
    using namespace std::chrono;
    static const steady_clock::time_point t0 = steady_clock::now();
    return duration<double>(steady_clock::now() - t0).count();
}

// First-fit allocator over [0, size), 256-byte granules, coalescing frees.
class Arena {
   public:
    void init(size_t size) {
        free_.clear();
        free_[0] = size;
        size_ = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Session {
    int cls = 0, m = 0;
    int64_t n = 0, npad = 0;
    size_t off = 0, bytes = 0;
    int64_t t_sched = 0;   // steps enqueued on the device
    uint64_t seed = 0;
    int32_t hold = 1;
    bool keep = false;
    bool busy = false;     // a request is attached
    int readers = 0;       // host copies of the state in progress: no request is admitted meanwhile
};

struct Req {
    mgx_request r;
    int state = 0;         // 0 queued, 1 running, 2 done, 3 cancelled, 4 failed
    int64_t session = -1;
    int64_t steps_done = 0, steps_sched = 0;
    double t_arr = 0, t_admit = 0, t_done = 0;
    bool cancel = false;
    bool needs_init = false;      // new session: record and state still to be written
    int64_t act_row0 = 0;         // caller commands: hold interval of their row 0
    hipEvent_t last_ev = nullptr;  // event of the iteration holding this request's latest chunk
};

struct Iter {
    int lane = 0;                  // stream of the pool it runs on
    hipEvent_t ev = nullptr;
    std::vector<std::pair<int64_t, int32_t>> work;  // (request, steps)
};

// One stream of the pool, with its own work counter and tile buffers, so that iterations
// on different streams may run concurrently.
struct Lane {
    hipStream_t stream = nullptr;
    DevMisc* misc = nullptr;
    int slot = 0;
    ServeTile* h_tiles = nullptr;
    ServeTile* d_tiles = nullptr;
    bool busy = false;
};

constexpr int kMaxTiles = 1 << 18;

}  // namespace

struct mgx_server {
    mgx_server_desc d;
    int device = 0, n_cu = 256;
    hipStream_t stream = nullptr;  // set-up work
    std::vector<Lane> lanes;
    void* arena_mem = nullptr;
    Arena arena;
    ClassDesc64* d_classdesc = nullptr;
    ClassT<float>* d_class = nullptr;
    ClassT<double>* d_class_d = nullptr;
    ClassT<float> h_class[MGX_MAX_CLASSES];
    double* d_nominal = nullptr;
    int next_lane = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false;
    std::deque<int64_t> pending;
    std::vector<int64_t> active;
    std::map<int64_t, Req> reqs;
    std::map<int64_t, Session> sessions;
    std::vector<Iter> inflight;
    std::vector<double> latencies;
    int64_t next_req = 0, next_session = 0;
    int64_t n_submitted = 0, n_completed = 0, n_cancelled = 0, env_steps = 0, iterations = 0;
    double t_create = 0;
    bool failed = false;

    size_t session_bytes(int cls, int64_t n) const {
        const int64_t npad = (n + kWave - 1) / kWave * kWave;
        const int m = h_class[cls].m;
        return (size_t)4 * npad * (kStateFixed + m + kRecLen);
    }
    void loop();
    void admit_locked();
    bool launch_locked();
    void complete_locked(Iter& it);
    void free_session_locked(int64_t sid);
};

void mgx_server::free_session_locked(int64_t sid) {
    auto it = sessions.find(sid);
    if (it == sessions.end()) return;
    arena.release(it->second.off, it->second.bytes);
    sessions.erase(it);
}

void mgx_server::admit_locked() {
    const bool fifo = (d.serve_flags & MGX_SERVE_FIFO) != 0;
    for (auto it = pending.begin(); it != pending.end();) {
        if ((int)active.size() >= (fifo ? 1 : d.max_active)) break;
        Req& q = reqs[*it];
        if (q.cancel) {
            q.state = 3;
            q.t_done = now_s();
            ++n_cancelled;
            it = pending.erase(it);
            done_cv.notify_all();
            continue;
        }
        int64_t sid = q.r.session;
        auto fail_request = [&]() {
            q.state = 4;
            q.t_done = now_s();
            it = pending.erase(it);
            done_cv.notify_all();
        };
        if (sid >= 0) {
            auto s = sessions.find(sid);
            if (s == sessions.end()) {
                fail_request();
                continue;
            }
            if (s->second.busy || s->second.readers > 0) {
                if (fifo) break;
                ++it;
                continue;
            }
        }
        // caller commands must cover every hold interval the request's steps touch, from the
        // session's current step on
        const int64_t t_start = sid >= 0 ? sessions[sid].t_sched : 0;
        const int64_t hold = sid >= 0 ? sessions[sid].hold : q.r.hold;
        if (q.r.actions && (t_start + q.r.horizon - 1) / hold - t_start / hold + 1 > q.r.action_rows) {
            fail_request();
            continue;
        }
        if (sid >= 0) {
            Session& S = sessions[sid];
            S.busy = true;
            S.keep = S.keep || q.r.keep;
        } else {
            const size_t bytes = session_bytes(q.r.class_index, q.r.n_envs);
            size_t off = 0;
            if (!arena.alloc(bytes, &off)) {
                if (fifo) break;
                ++it;  // first fit: a smaller request further back may fit
                continue;
            }
            sid = next_session++;
            Session S;
            S.cls = q.r.class_index;
            S.m = h_class[S.cls].m;
            S.n = q.r.n_envs;
            S.npad = (S.n + kWave - 1) / kWave * kWave;
            S.off = off;
            S.bytes = bytes;
            S.seed = q.r.seed;
            S.hold = q.r.hold;
            S.keep = q.r.keep != 0;
            S.busy = true;
            q.needs_init = true;
            sessions[sid] = S;
        }
        q.act_row0 = t_start / hold;
        q.session = sid;
        q.state = 1;
        q.t_admit = now_s();
        active.push_back(*it);
        it = pending.erase(it);
    }
}

bool mgx_server::launch_locked() {
    const bool fifo = (d.serve_flags & MGX_SERVE_FIFO) != 0;
    int li = -1;
    for (int k = 0; k < (int)lanes.size(); ++k) {
        const int c = (next_lane + k) % (int)lanes.size();
        if (!lanes[c].busy) {
            li = c;
            break;
        }
    }
    if (li < 0) return false;
    Lane& L = lanes[li];
    Iter iter;
    iter.lane = li;
    ServeTile* ht = L.h_tiles;
    int n = 0;
    std::vector<int64_t> picked;
    for (int64_t rid : active) {
        Req& q = reqs[rid];
        if (q.cancel || q.steps_sched >= q.r.horizon) continue;
        Session& S = sessions[q.session];
        const int64_t remaining = q.r.horizon - q.steps_sched;
        const int64_t cap = (fifo || d.chunk_steps <= 0) ? remaining : std::min<int64_t>(remaining, d.chunk_steps);
        const int32_t steps = (int32_t)cap;
        const int ntile = (int)(S.npad / kWave);
        if (n + ntile > kMaxTiles) break;
        float* base = (float*)((char*)arena_mem + S.off);
        float* rec = base + (size_t)(kStateFixed + S.m) * S.npad;
        if (q.needs_init) {
            hipLaunchKernelGGL(k_session_init, dim3((unsigned)((S.npad + 255) / 256)), dim3(256), 0, L.stream, base, rec,
                               S.m, S.n, S.npad, d_classdesc, S.cls, d_nominal, d.dt, S.seed);
            if (hipGetLastError() != hipSuccess) failed = true;
            q.needs_init = false;
        } else if (q.last_ev) {
            // the previous chunk of this request runs on another stream: order after it
            if (hipStreamWaitEvent(L.stream, q.last_ev, 0) != hipSuccess) failed = true;
        }
        for (int t = 0; t < ntile; ++t) {
            ServeTile& T = ht[n++];
            T.state = base;
            T.rec = rec;
            T.t0 = S.t_sched;
            T.seed = S.seed;
            T.act = q.r.actions;
            T.act_row0 = q.act_row0;
            T.npad = (int32_t)S.npad;
            T.env0 = t * kWave;
            T.steps = steps;
            T.hold = S.hold;
            T.cls = S.cls;
            T.nvalid = (int32_t)S.n;
            T.pad0 = T.pad1 = 0;
        }
        S.t_sched += steps;
        q.steps_sched += steps;
        iter.work.push_back({rid, steps});
        picked.push_back(rid);
    }
    if (n == 0) return false;
    hipError_t e = hipMemcpyAsync(L.d_tiles, ht, sizeof(ServeTile) * n, hipMemcpyHostToDevice, L.stream);
    ServeArgs P;
    P.tiles = L.d_tiles;
    P.cls = d_class;
    P.n_tiles = n;
    P.n_classes = d.n_classes;
    P.misc = L.misc;
    P.rd = L.slot;
    P.wr = 1 - L.slot;
    L.slot = 1 - L.slot;
    const int grid = std::min((n + 3) / 4, n_cu * 2);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_serve, dim3(grid), dim3(256), 0, L.stream, P);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&iter.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(iter.ev, L.stream);
    if (e != hipSuccess) {
        failed = true;
        return false;
    }
    for (int64_t rid : picked) reqs[rid].last_ev = iter.ev;
    L.busy = true;
    next_lane = (li + 1) % (int)lanes.size();
    ++iterations;
    inflight.push_back(std::move(iter));
    return true;
}

void mgx_server::complete_locked(Iter& it) {
    const double t = now_s();
    for (auto& w : it.work) {
        Req& q = reqs[w.first];
        q.steps_done += w.second;
        Session& S = sessions[q.session];
        env_steps += (int64_t)w.second * S.n;
        if (q.steps_done >= q.r.horizon || (q.cancel && q.steps_done >= q.steps_sched)) {
            q.state = q.cancel && q.steps_done < q.r.horizon ? 3 : 2;
            q.t_done = t;
            if (q.state == 2) {
                ++n_completed;
                latencies.push_back(t - q.t_arr);
            } else {
                ++n_cancelled;
            }
            S.busy = false;
            if (!S.keep) free_session_locked(q.session);
            active.erase(std::remove(active.begin(), active.end(), w.first), active.end());
        }
    }
    for (auto& w : it.work) {
        Req& q = reqs[w.first];
        if (q.last_ev == it.ev) q.last_ev = nullptr;
    }
    lanes[it.lane].busy = false;
    (void)hipEventDestroy(it.ev);
    done_cv.notify_all();
}

void mgx_server::loop() {
    (void)hipSetDevice(device);
    // Completions are found by polling events; with the default 50 us timer slack a short
    // timed wait would oversleep by that much on every request.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        for (size_t i = 0; i < inflight.size();) {
            hipError_t q = hipEventQuery(inflight[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (q != hipSuccess) failed = true;
            complete_locked(inflight[i]);
            inflight.erase(inflight.begin() + (long)i);
            progress = true;
        }
        // cancelled requests with nothing in flight leave immediately
        for (auto it = active.begin(); it != active.end();) {
            Req& q = reqs[*it];
            if (q.cancel && q.steps_done >= q.steps_sched) {
                q.state = 3;
                q.t_done = now_s();
                ++n_cancelled;
                Session& S = sessions[q.session];
                S.busy = false;
                if (!S.keep) free_session_locked(q.session);
                it = active.erase(it);
                done_cv.notify_all();
                progress = true;
            } else {
                ++it;
            }
        }
        if (!failed) admit_locked();
        if (!failed && launch_locked()) progress = true;
        if (stop && pending.empty() && active.empty() && inflight.empty()) break;
        if (failed && inflight.empty()) {
            for (auto& kv : reqs)
                if (kv.second.state < 2) kv.second.state = 4;
            done_cv.notify_all();
            if (stop) break;
        }
        if (!progress) cv.wait_for(lk, std::chrono::microseconds(inflight.empty() ? 500 : 5));
    }
}

extern "C" double mgx_server_now(void) { return now_s(); }

extern "C" mgx_status mgx_server_create(const mgx_server_desc* d, mgx_server** out) {
    if (!d || !out) return fail(MGX_E_INVALID, "NULL argument");
    *out = nullptr;
    if (d->n_classes < 1 || d->n_classes > MGX_MAX_CLASSES || !d->class_ids || !d->nominal)
        return fail(MGX_E_INVALID, "n_classes in [1,16] with class_ids and nominal parameters");
    if (!(d->dt > 0) || d->chunk_steps < 0 || d->max_active < 1 || d->budget_bytes < 4096 || d->streams < 0 ||
        d->streams > 16)
        return fail(MGX_E_INVALID, "dt > 0, chunk_steps >= 0, max_active >= 1, budget >= 4096 bytes, streams in [0, 16]");
    if (d->batch_flags & ~(MGX_FLAG_NO_AMC | MGX_FLAG_LAG_EULER)) return fail(MGX_E_INVALID, "unknown batch flag");
    std::vector<ClassDesc64> d64(MGX_MAX_CLASSES);
    for (int c = 0; c < d->n_classes; ++c) {
        mgx_class_desc cd;
        if (!get_class(d->class_ids[c], &cd)) return fail(MGX_E_INVALID, "class id %d unknown", d->class_ids[c]);
        if (fin_mask_of(to_desc64(cd)) != 0)
            return fail(MGX_E_INVALID, "class %d has fins: the server runs propeller classes only", c);
        if (has_payload(to_desc64(cd)))
            return fail(MGX_E_INVALID, "class %d has a payload: the server runs classes without one", c);
        d64[c] = to_desc64(cd);
        const double* p = d->nominal + 23 * c;
        if (!(p[0] > 0) || !std::isfinite(p[0])) return fail(MGX_E_INVALID, "nominal mass of class %d must be > 0", c);
        for (int j = 1; j < 23; ++j)
            if (!std::isfinite(p[j]) || (j < 20 && !(p[j] >= 0)))
                return fail(MGX_E_INVALID, "nominal value %d of class %d must be finite%s", j, c,
                            j < 20 ? " and >= 0" : "");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(MGX_E_DEVICE, "no HIP device visible");
    mgx_server* s = new (std::nothrow) mgx_server();
    if (!s) return fail(MGX_E_NOMEM, "host allocation");
    s->d = *d;
    s->device = d->device;
    if (s->device < 0) (void)hipGetDevice(&s->device);
    hipDevice_guard g(s->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->device) == hipSuccess && prop.multiProcessorCount > 0)
        s->n_cu = prop.multiProcessorCount;
    auto cleanup = [s]() {
        for (Lane& L : s->lanes) {
            if (L.h_tiles) (void)hipHostFree(L.h_tiles);
            if (L.d_tiles) (void)hipFree(L.d_tiles);
            if (L.misc) (void)hipFree(L.misc);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        void* ps[] = {s->arena_mem, s->d_classdesc, s->d_class, s->d_class_d, s->d_nominal};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
    };
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s->arena_mem, (size_t)d->budget_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_classdesc, sizeof(ClassDesc64) * MGX_MAX_CLASSES);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_class, sizeof(ClassT<float>) * MGX_MAX_CLASSES);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_class_d, sizeof(ClassT<double>) * MGX_MAX_CLASSES);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_nominal, sizeof(double) * 23 * d->n_classes);
    const int n_lanes = (d->serve_flags & MGX_SERVE_FIFO) ? 1 : (d->streams > 0 ? d->streams : 4);
    s->lanes.resize(n_lanes);
    for (int i = 0; i < n_lanes && e == hipSuccess; ++i) {
        Lane& L = s->lanes[i];
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc((void**)&L.misc, sizeof(DevMisc));
        if (e == hipSuccess) e = hipMemset(L.misc, 0, sizeof(DevMisc));
        if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_tiles, sizeof(ServeTile) * kMaxTiles, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_tiles, sizeof(ServeTile) * kMaxTiles);
    }
    if (e == hipSuccess) e = hipMemcpy(s->d_classdesc, d64.data(), sizeof(ClassDesc64) * MGX_MAX_CLASSES, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->d_nominal, d->nominal, sizeof(double) * 23 * d->n_classes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_class_setup(s->d_classdesc, s->d_class, s->d_class_d, d->n_classes, d->dt,
                                                d->batch_flags, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_class, s->d_class, sizeof(ClassT<float>) * MGX_MAX_CLASSES, hipMemcpyDeviceToHost,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        g_hip_err = (int32_t)e;
        cleanup();
        return fail(e == hipErrorOutOfMemory ? MGX_E_NOMEM : MGX_E_DEVICE, "server set-up: %s", hipGetErrorString(e));
    }
    // First use of a stream sets up its hardware queue: do it now, not during serving.
    for (Lane& L : s->lanes) {
        if (e != hipSuccess) break;
        ServeArgs P;
        std::memset(&P, 0, sizeof P);
        P.tiles = L.d_tiles;
        P.cls = s->d_class;
        P.n_tiles = 0;
        P.n_classes = d->n_classes;
        P.misc = L.misc;
        P.rd = L.slot;
        P.wr = 1 - L.slot;
        L.slot = 1 - L.slot;
        hipLaunchKernelGGL(k_serve, dim3(1), dim3(256), 0, L.stream, P);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(L.stream);
    }
    if (e != hipSuccess) {
        g_hip_err = (int32_t)e;
        cleanup();
        return fail(MGX_E_DEVICE, "server stream warm-up: %s", hipGetErrorString(e));
    }
    s->arena.init((size_t)d->budget_bytes);
    s->t_create = now_s();
    s->th = std::thread([s]() { s->loop(); });
    *out = s;
    return MGX_OK;
}

extern "C" mgx_status mgx_server_submit(mgx_server* s, const mgx_request* r, int64_t* request_id) {
    if (!s || !r || !request_id) return fail(MGX_E_INVALID, "NULL argument");
    if (r->class_index < 0 || r->class_index >= s->d.n_classes) return fail(MGX_E_INVALID, "class_index out of range");
    if (r->horizon < 1 || r->hold < 1) return fail(MGX_E_INVALID, "horizon and hold must be >= 1");
    if (r->actions && r->action_rows < 1) return fail(MGX_E_INVALID, "action_rows must be >= 1 with actions");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(MGX_E_STATE, "server is stopping");
    if (r->session < 0) {
        if (r->n_envs < 1 || r->n_envs > (int64_t)1 << 26) return fail(MGX_E_INVALID, "n_envs outside [1, 2^26]");
        if (s->session_bytes(r->class_index, r->n_envs) > (size_t)s->d.budget_bytes)
            return fail(MGX_E_BUDGET, "request needs %zu bytes; budget is %lld",
                        s->session_bytes(r->class_index, r->n_envs), (long long)s->d.budget_bytes);
    } else {
        auto it = s->sessions.find(r->session);
        if (it == s->sessions.end()) return fail(MGX_E_INVALID, "session %lld is not resident", (long long)r->session);
        if (it->second.cls != r->class_index)
            return fail(MGX_E_INVALID, "session %lld belongs to class %d", (long long)r->session, it->second.cls);
    }
    const int64_t id = s->next_req++;
    Req q;
    q.r = *r;
    q.t_arr = r->arrival > 0 ? r->arrival : now_s();
    s->reqs[id] = q;
    s->pending.push_back(id);
    ++s->n_submitted;
    *request_id = id;
    s->cv.notify_all();
    return MGX_OK;
}

static void fill_status(const Req& q, mgx_request_status* o) {
    std::memset(o, 0, sizeof *o);
    o->state = q.state;
    o->session = q.session;
    o->steps_done = q.steps_done;
    o->t_arrival = q.t_arr;
    o->t_admit = q.t_admit;
    o->t_done = q.t_done;
}

extern "C" mgx_status mgx_server_poll(mgx_server* s, int64_t id, mgx_request_status* out) {
    if (!s || !out) return fail(MGX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MGX_E_INVALID, "unknown request %lld", (long long)id);
    fill_status(it->second, out);
    return MGX_OK;
}

extern "C" mgx_status mgx_server_wait(mgx_server* s, int64_t id, double timeout_s, mgx_request_status* out) {
    if (!s) return fail(MGX_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MGX_E_INVALID, "unknown request %lld", (long long)id);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (it->second.state < 2) {
        if (s->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && it->second.state < 2) {
            if (out) fill_status(it->second, out);
            return fail(MGX_E_STATE, "request %lld not finished after %.3f s", (long long)id, timeout_s);
        }
    }
    if (out) fill_status(it->second, out);
    return it->second.state == 4 ? fail(MGX_E_DEVICE, "request failed") : MGX_OK;
}

extern "C" mgx_status mgx_server_cancel(mgx_server* s, int64_t id) {
    if (!s) return fail(MGX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MGX_E_INVALID, "unknown request %lld", (long long)id);
    it->second.cancel = true;
    s->cv.notify_all();
    return MGX_OK;
}

extern "C" mgx_status mgx_server_read_state(mgx_server* s, int64_t session, float* out, int64_t capacity) {
    if (!s || !out) return fail(MGX_E_INVALID, "NULL argument");
    Session S;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->sessions.find(session);
        if (it == s->sessions.end()) return fail(MGX_E_INVALID, "session %lld is not resident", (long long)session);
        if (it->second.busy) return fail(MGX_E_STATE, "session %lld has a request in progress", (long long)session);
        S = it->second;
        if (capacity < (int64_t)(kStateFixed + S.m) * S.n)
            return fail(MGX_E_INVALID, "capacity %lld < %lld", (long long)capacity,
                        (long long)((kStateFixed + S.m) * S.n));
        // Not busy: no work on this session is in flight. Marking it read keeps the
        // scheduler from admitting a queued request for it until the copy is done.
        ++it->second.readers;
    }
    const int rows = kStateFixed + S.m;
    hipError_t e = hipSuccess;
    {
        hipDevice_guard g(s->device);
        std::vector<float> tmp((size_t)rows * S.npad);
        e = hipMemcpy(tmp.data(), (char*)s->arena_mem + S.off, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (int j = 0; j < rows; ++j)
                std::memcpy(out + j * S.n, tmp.data() + (size_t)j * S.npad, sizeof(float) * S.n);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        --s->sessions[session].readers;
        s->cv.notify_all();
    }
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipMemcpy(session state)");
    return MGX_OK;
}

extern "C" mgx_status mgx_server_release(mgx_server* s, int64_t session) {
    if (!s) return fail(MGX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end()) return fail(MGX_E_INVALID, "session %lld is not resident", (long long)session);
    if (it->second.busy || it->second.readers > 0)
        return fail(MGX_E_STATE, "session %lld has a request or a read in progress", (long long)session);
    s->free_session_locked(session);
    return MGX_OK;
}

extern "C" mgx_status mgx_server_stats_get(mgx_server* s, mgx_server_stats* o) {
    if (!s || !o) return fail(MGX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(o, 0, sizeof *o);
    o->submitted = s->n_submitted;
    o->completed = s->n_completed;
    o->cancelled = s->n_cancelled;
    o->queued = (int64_t)s->pending.size();
    o->active = (int64_t)s->active.size();
    o->env_steps = s->env_steps;
    o->iterations = s->iterations;
    o->bytes_in_use = (int64_t)s->arena.used();
    o->bytes_peak = (int64_t)s->arena.peak();
    o->budget_bytes = s->d.budget_bytes;
    o->wall = now_s() - s->t_create;
    if (!s->latencies.empty()) {
        std::vector<double> v = s->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double x = p * (double)(v.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - (double)i;
            return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
        };
        o->p50_latency = pct(0.50);
        o->p99_latency = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        o->mean_latency = sum / (double)v.size();
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_server_destroy(mgx_server* s) {
    if (!s) return MGX_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->reqs) kv.second.cancel = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    hipDevice_guard g(s->device);
    (void)hipStreamSynchronize(s->stream);
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.h_tiles) (void)hipHostFree(L.h_tiles);
        if (L.d_tiles) (void)hipFree(L.d_tiles);
        if (L.misc) (void)hipFree(L.misc);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    void* ps[] = {s->arena_mem, s->d_classdesc, s->d_class, s->d_class_d, s->d_nominal};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return MGX_OK;
}
