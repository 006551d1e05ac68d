// Per-environment K-step loop and statistics reductions, shared by the per-class kernel
// and the persistent heterogeneous kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "step.hpp"

namespace mgx {

// ----------------------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32->64-bit
// multiplications by fixed odd constants, the high halves xored with the other counter
// words and the round key; the key advances by two Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
    return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * 0x1.0p-53;
}

constexpr uint32_t kStreamInit = 3u;
constexpr uint32_t kStreamAction = 4u;

// M = M_RB + M_A of a class with a payload (centre of gravity at rg from the body origin):
// [m 1 + A_1, -m S(rg); m S(rg), I_o + A_2] with I_o = I_g + m(|rg|^2 1 - rg rg^T).
__device__ __forceinline__ void payload_mass_matrix(const double inertia[3], const double rg[3], double m,
                                                    const double added[6], double M[6][6]) {
    const double S[3][3] = {{0.0, -rg[2], rg[1]}, {rg[2], 0.0, -rg[0]}, {-rg[1], rg[0], 0.0}};
    const double r2 = rg[0] * rg[0] + rg[1] * rg[1] + rg[2] * rg[2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[i][j] = (i == j) ? m : 0.0;
            M[i][3 + j] = -m * S[i][j];
            M[3 + i][j] = m * S[i][j];
            M[3 + i][3 + j] = ((i == j) ? inertia[i] + m * r2 : 0.0) - m * rg[i] * rg[j];
        }
    for (int j = 0; j < 6; ++j) M[j][j] += added[j];
}

// Cholesky factor L (M = L L^T) in double; false when a pivot is not positive (M is not
// positive definite) or not finite.
__device__ __forceinline__ bool cholesky6(const double M[6][6], double L[6][6]) {
    bool ok = true;
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 6; ++i) L[j][i] = 0.0;
    for (int j = 0; j < 6; ++j) {
        double d = M[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        ok = ok && d > 0.0 && d <= 1.0e300;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = M[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    return ok;
}

// dt M^-1 of a payload class by Cholesky factorisation in double; false (out undefined)
// when M is not positive definite.
__device__ __forceinline__ bool payload_minv(const double inertia[3], const double rg[3], double m,
                                             const double added[6], double dt, double out[6][6]) {
    double M[6][6], L[6][6];
    payload_mass_matrix(inertia, rg, m, added, M);
    if (!cholesky6(M, L)) return false;
    for (int c = 0; c < 6; ++c) {  // column c of M^-1: L y = e_c, then L^T x = y
        double y[6], x[6];
        for (int i = 0; i < 6; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
            y[i] = v / L[i][i];
        }
        for (int i = 5; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 6; ++k) v -= L[k][i] * x[k];
            x[i] = v / L[i][i];
        }
        for (int i = 0; i < 6; ++i) out[i][c] = dt * x[i];
    }
    return true;
}

__device__ __forceinline__ bool finite64(double x) { return x - x == 0.0; }

// Validity of one environment's parameters, as a record build needs them: kErrParam when
// a value is not finite or out of range (mass > 0; added mass, damping, buoyancy >= 0),
// kErrNotSpd when M = M_RB + M_A is not positive definite (diagonal: every M_jj > 0; with a
// payload: every Cholesky pivot > 0). 0 when valid.
__device__ __forceinline__ int32_t params_flags(const double inertia[3], double m, const double added[6],
                                                const double dlin[6], const double dquad[6], double buoy,
                                                const double cur[3], const double* rg) {
    bool ok = finite64(m) && m > 0.0 && finite64(buoy) && buoy >= 0.0;
    bool spd = true;
    for (int j = 0; j < 6; ++j) {
        ok = ok && finite64(added[j]) && finite64(dlin[j]) && dlin[j] >= 0.0 && finite64(dquad[j]) &&
             dquad[j] >= 0.0;
        const double Mjj = (j < 3 ? m : inertia[j - 3]) + added[j];
        spd = spd && Mjj > 0.0;
    }
    for (int j = 0; j < 3; ++j) ok = ok && finite64(cur[j]);
    if (!ok) return kErrParam;
    if (spd && rg && (rg[0] != 0.0 || rg[1] != 0.0 || rg[2] != 0.0)) {
        double M[6][6], L[6][6];
        payload_mass_matrix(inertia, rg, m, added, M);
        spd = cholesky6(M, L);
    }
    return spd ? 0 : kErrNotSpd;
}

// Per-environment record (dt M^-1, m, M_A, d_L, d_Q, W - B, B, V_c), derived in double
// (M = M_RB + M_A with M_RB = diag(m, m, m, I)) and rounded once; column i of a segment.
// With a payload (rg non-null and non-zero) dt M^-1 is the full symmetric inverse: its
// diagonal in the usual rows, the off-diagonal entries in the 15 rows from kRecMinvOff.
// Returns params_flags of the inputs; when they are invalid the dt M^-1 rows hold NaN, so
// the environment's state turns non-finite at its next step instead of running on with an
// undefined inverse.
template <typename T>
__device__ __forceinline__ int32_t write_record(const double inertia[3], double g0, double dt, double m,
                                                const double added[6], const double dlin[6], const double dquad[6],
                                                double buoy, const double cur[3], T* rec, int64_t npad, int64_t i,
                                                const double* rg = nullptr) {
    const int32_t flags = params_flags(inertia, m, added, dlin, dquad, buoy, cur, rg);
    const bool payload = rg && (rg[0] != 0.0 || rg[1] != 0.0 || rg[2] != 0.0);
    const double nan = __builtin_nan("");
    if (payload) {
        double Mi[6][6];
        if (flags || !payload_minv(inertia, rg, m, added, dt, Mi))
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) Mi[a][b] = nan;
        int k = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a + 1; b < 6; ++b, ++k) rec[(kRecMinvOff + k) * npad + i] = (T)(0.5 * (Mi[a][b] + Mi[b][a]));
        for (int j = 0; j < 6; ++j) rec[(kRecDtMinv + j) * npad + i] = (T)Mi[j][j];
    }
    for (int j = 0; j < 6; ++j) {
        const double Mjj = (j < 3 ? m : inertia[j - 3]) + added[j];
        if (!payload) rec[(kRecDtMinv + j) * npad + i] = (T)(flags ? nan : dt / Mjj);
        rec[(kRecAdded + j) * npad + i] = (T)added[j];
        rec[(kRecDlin + j) * npad + i] = (T)dlin[j];
        rec[(kRecDquad + j) * npad + i] = (T)dquad[j];
    }
    rec[kRecMass * npad + i] = (T)m;
    rec[kRecWmB * npad + i] = (T)(m * g0 - buoy);
    rec[kRecBuoy * npad + i] = (T)buoy;
    for (int j = 0; j < 3; ++j) rec[(kRecCurrent + j) * npad + i] = (T)cur[j];
    return flags;
}

// Seeded initial state of global env id g: p = 0, q uniform on S^3 (normalised Gaussian),
// nu ~ N(0, 0.2^2), n = 0; Box-Muller over Philox words, in double, rounded once.
template <typename T>
__device__ __forceinline__ void seeded_state(uint64_t g, uint64_t seed, int m, T* state, int64_t npad, int64_t e) {
    double u[10];
    for (int j = 0; j < 5; ++j) {
        uint32_t c[4] = {(uint32_t)g, 0u, (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)seed, kStreamInit << 24);
        u[2 * j] = u53(c[0], c[1]);
        u[2 * j + 1] = u53(c[2], c[3]);
    }
    double z[10];
    for (int j = 0; j < 5; ++j) {
        double rad = sqrt(-2.0 * log(1.0 - u[2 * j]));
        double ang = 2.0 * M_PI * u[2 * j + 1];
        z[2 * j] = rad * cos(ang);
        z[2 * j + 1] = rad * sin(ang);
    }
    double qn = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3]);
    for (int j = 0; j < 3; ++j) state[j * npad + e] = (T)0;
    for (int j = 0; j < 4; ++j) state[(3 + j) * npad + e] = (T)(z[j] / qn);
    for (int j = 0; j < 6; ++j) state[(7 + j) * npad + e] = (T)(0.2 * z[4 + j]);
    for (int i = 0; i < m; ++i) state[(kStateFixed + i) * npad + e] = (T)0;
}

// Action in [-1, 1) from a generator word: ((w >> 8) - 2^23) 2^-23, exact in float.
__device__ __forceinline__ float action_from_word(uint32_t w) {
    return (float)((int32_t)(w >> 8) - (1 << 23)) * 0x1.0p-23f;
}


__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__host__ __device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

template <typename T>
__device__ __forceinline__ bool finite_(T x) {
    return x == x && abs_(x) <= (T)3.0e38;
}

__device__ __forceinline__ bool is_max_slot(int j) {
    return j == kStMaxSpeed || j == kStMaxRate || j == kStMaxDrift;
}

// Wave then block reduction of per-lane statistics; thread j < kStats writes slot j.
__device__ __forceinline__ void block_reduce_stats(const float st[kStats], float (*red)[kStats], float* out) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
#pragma unroll
    for (int j = 0; j < kStats; ++j) {
        float v = is_max_slot(j) ? wave_max(st[j]) : wave_sum(st[j]);
        if (lane == 0) red[wv][j] = v;
    }
    __syncthreads();
    if (tid < kStats) {
        float v = red[0][tid];
        for (int w = 1; w < (int)blockDim.x / kWave; ++w) v = is_max_slot(tid) ? fmaxf(v, red[w][tid]) : v + red[w][tid];
        out[tid] = v;
    }
}

// Deterministic reduction over n partial records (fixed order), slot j.
__device__ __forceinline__ void final_reduce_stats(const float* partials, unsigned n, int j, double* out) {
    double acc = 0.0;
    for (unsigned b = 0; b < n; ++b) {
        const double v = (double)__hip_atomic_load(&partials[(int64_t)b * kStats + j], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        acc = is_max_slot(j) ? fmax(acc, v) : acc + v;
    }
    out[j] = acc;
}

#ifdef MGX_WAVE_TIMESTAMPS
// Diagnostic builds only: per-wave phase times of the step loop on the 100 MHz real-time
// counter (entry; prologue loads landed; steps done; stores drained), indexed by the wave's
// position in its launch. Every translation unit has its own copy; the step kernels' copy
// is read back by mgx_diag_wave_times.
constexpr int kWaveTsMax = 1 << 16;
static __device__ unsigned long long g_wave_ts[kWaveTsMax][4];
#define MGX_WAVE_TS(var) const unsigned long long var = __builtin_amdgcn_s_memrealtime()
#else
#define MGX_WAVE_TS(var)
#endif

// A wave-uniform value moved to a vector register and hidden from the uniformity analysis,
// so the compiler keeps it there. The allocation columns (6 x m values) would otherwise sit
// in scalar registers, which cannot hold them next to the loop's own scalars for m = 8.
__device__ __forceinline__ float in_vgpr(float x) {
    asm("" : "+v"(x));
    return x;
}
__device__ __forceinline__ double in_vgpr(double x) {
    asm("" : "+v"(x));
    return x;
}
__device__ __forceinline__ int32_t in_vgpr(int32_t x) {
    asm("" : "+v"(x));
    return x;
}

// 64-bit wave-uniform value of lane 0 (the value is the same in every lane)
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A copy of the class constants for the step loop. With more than six thrusters, or with
// fins, the per-actuator arrays (k-scaled layout columns, lag factors, fin geometry and
// gains) move to vector registers; up to six propellers they fit the scalar file next to
// the loop's own scalars and stay there.
template <typename T, int M, bool kFins = false>
__device__ __forceinline__ ClassT<T> class_in_vgpr(const ClassT<T>& Cs) {
    ClassT<T> C = Cs;
    if constexpr (kFins) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                C.fin_r[i][j] = in_vgpr(Cs.fin_r[i][j]);
                C.fin_c[i][j] = in_vgpr(Cs.fin_c[i][j]);
                C.fin_n[i][j] = in_vgpr(Cs.fin_n[i][j]);
            }
            C.fin_max[i] = in_vgpr(Cs.fin_max[i]);
            C.fin_kl[i] = in_vgpr(Cs.fin_kl[i]);
            C.fin_kd0[i] = in_vgpr(Cs.fin_kd0[i]);
            C.fin_kd[i] = in_vgpr(Cs.fin_kd[i]);
        }
    }
    if constexpr (M > 6 || kFins) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
#pragma unroll
            for (int j = 0; j < 6; ++j) C.Bk[j][i] = in_vgpr(Cs.Bk[j][i]);
            C.alpha[i] = in_vgpr(Cs.alpha[i]);
        }
    }
    return C;
}

// State and per-environment record of slot `env` of a segment of np slots.
template <typename T, int M>
__device__ __forceinline__ void load_state(const T* S, int64_t np, int64_t env, StateT<T, M>& s) {
#pragma unroll
    for (int j = 0; j < 3; ++j) s.p[j] = S[j * np + env];
#pragma unroll
    for (int j = 0; j < 4; ++j) s.q[j] = S[(3 + j) * np + env];
#pragma unroll
    for (int j = 0; j < 6; ++j) s.nu[j] = S[(7 + j) * np + env];
#pragma unroll
    for (int i = 0; i < M; ++i) s.n[i] = S[(kStateFixed + i) * np + env];
}

template <typename T, int M>
__device__ __forceinline__ void store_state(T* S, int64_t np, int64_t env, const StateT<T, M>& s) {
#pragma unroll
    for (int j = 0; j < 3; ++j) S[j * np + env] = s.p[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) S[(3 + j) * np + env] = s.q[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) S[(7 + j) * np + env] = s.nu[j];
#pragma unroll
    for (int i = 0; i < M; ++i) S[(kStateFixed + i) * np + env] = s.n[i];
}

template <typename T, bool kPayload>
__device__ __forceinline__ void load_record(const T* Rc, int64_t np, int64_t env, uint32_t flags, EnvT<T>& E) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        E.dtMinv[j] = Rc[(kRecDtMinv + j) * np + env];
        E.A[j] = Rc[(kRecAdded + j) * np + env];
        E.dL[j] = Rc[(kRecDlin + j) * np + env];
        E.dQ[j] = Rc[(kRecDquad + j) * np + env];
    }
    E.mass = Rc[kRecMass * np + env];
    E.wmb = Rc[kRecWmB * np + env];
    E.buoy = Rc[kRecBuoy * np + env];
#pragma unroll
    for (int j = 0; j < 3; ++j) E.Vc[j] = Rc[(kRecCurrent + j) * np + env];
    if constexpr (kPayload) {
#pragma unroll
        for (int k = 0; k < 15; ++k) E.dtMinvOff[k] = Rc[(kRecMinvOff + k) * np + env];
    }
    set_amc(E, flags);
}

// Per-environment constants of the step formed once per launch: I + A_2, B r_b and, with
// a payload, the inertia about the origin plus A_2, m r_g and B r_b - W r_g.
template <typename T, bool kPayload>
__device__ __forceinline__ void env_prologue(const ClassT<T>& C, EnvT<T>& E, T IA2[3], T Brb[3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        IA2[j] = C.inertia[j] + E.A[3 + j];
        Brb[j] = E.buoy * C.rb[j];
    }
    if constexpr (kPayload) {
        // I_o + A_2 = I_g + m(|r_g|^2 1 - r_g r_g^T) + A_2; m r_g; (B r_b - W r_g)
        const T* r = C.rg;
        const T m = E.mass, W = E.mass * C.g0;
        E.IoA[0] = IA2[0] + m * (r[1] * r[1] + r[2] * r[2]);
        E.IoA[1] = IA2[1] + m * (r[0] * r[0] + r[2] * r[2]);
        E.IoA[2] = IA2[2] + m * (r[0] * r[0] + r[1] * r[1]);
        E.IoA[3] = -(m * r[0] * r[1]);
        E.IoA[4] = -(m * r[0] * r[2]);
        E.IoA[5] = -(m * r[1] * r[2]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            E.mrg[j] = m * r[j];
            Brb[j] = fma_(-W, r[j], Brb[j]);
        }
    }
}

// Long-horizon attitude drift check: renormalise in double when | |q|^2 - 1 | > 1e-6,
// recording the drift and whether it renormalised in the launch statistics `st`.
template <typename T, int M>
__device__ __forceinline__ void renorm_attitude(StateT<T, M>& s, float st[kStats]) {
    T n2 = fma_(s.q[3], s.q[3], fma_(s.q[2], s.q[2], fma_(s.q[1], s.q[1], s.q[0] * s.q[0])));
    T drift = abs_(n2 - T(1));
    if (drift > T(1e-6)) {
        double qd[4] = {(double)s.q[0], (double)s.q[1], (double)s.q[2], (double)s.q[3]};
        double inv = 1.0 / sqrt(qd[0] * qd[0] + qd[1] * qd[1] + qd[2] * qd[2] + qd[3] * qd[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j) s.q[j] = (T)(qd[j] * inv);
        st[kStRenorm] = 1.0f;
    }
    st[kStMaxDrift] = (float)drift;
}

// K steps of environment `env` (a slot of the segment described by A) from global step
// t0. Commands are fetched raw one hold interval before use and clipped when their row
// becomes current; all prologue loads are drained once before the loop so that the only
// memory operations in flight inside it are those prefetches.
// kSingle: a launch of exactly one step without outputs (the single-step kernel). Such a
// launch never reaches the next action row, so it does not fetch it. Every lane of its grid
// calls this (env may be past the segment: such a lane works on the last slot and stores
// nothing). It reads the step counter itself and returns it in *t_single (t0 is not used):
// the state and record are loaded first, then the action row the host expected
// (A.row_hint, for step A.t_hint), and the counter last, per lane, so that waiting for the
// earlier loads does not wait for it (vector loads complete in order; a scalar load would
// be waited for with every other scalar load). The step runs on the expected row, and the
// counter is compared only afterwards; a launch that finds another step (which the host's
// own bookkeeping never produces: graphs replayed from another step than their capture's
// run one-step launches without a hint, in the K-step instantiation) runs the step again
// from the loaded state on the row the counter names. Reading the counter first and the
// row after it cost a dependent memory round trip of about half a microsecond per launch.
template <typename T, int M, bool kOut, bool kShaped, bool kSingle = false, bool kFins = false, bool kPayload = false>
__device__ __forceinline__ void env_steps(const StepArgs& A, const ClassT<T>& Cs, int64_t env, int64_t t0, int K,
                                          float st[kStats], int64_t* t_single = nullptr) {
    static_assert(!(kSingle && kOut), "the single-step form has no per-step outputs");
    MGX_WAVE_TS(ts_entry);
    const int64_t np = A.npad;
    const int64_t envl = (kSingle && env >= np) ? np - 1 : env;  // the slot this lane reads
    T* S = (T*)A.state;
    const T* Rc = (const T*)A.rec;
    StateT<T, M> s;
    load_state<T, M>(S, np, envl, s);
    EnvT<T> E;
    load_record<T, kPayload>(Rc, np, envl, Cs.flags, E);
    const ClassT<T> C = class_in_vgpr<T, M, kFins>(Cs);
    // classes with fins carry the attitude's low-order words through the launch (float)
    constexpr bool kComp = kFins && std::is_same<T, float>::value;
    StateLo<T> lo;
#pragma unroll
    for (int j = 0; j < 4; ++j) lo.q[j] = T(0);

    // Action rows, relative to the buffer start, uniform across the wave. Every fetch is
    // issued unconditionally at a row index clamped into the buffer (validity is tracked
    // separately), so each prefetch has a single definition and no copy forces an early wait.
    const int64_t hold = A.hold, nrows = A.n_rows, rstride = A.row_stride;
    const T* abase = (const T*)A.actions + envl;
    auto clamp_row = [nrows](int64_t x) { return x < 0 ? (int64_t)0 : (x >= nrows ? nrows - 1 : x); };
    T cur[M], nxt[M];
    bool bad;
    int phase = 0;
    int64_t r = 0;
    int64_t t_lane = 0;
    if constexpr (kSingle) {
        const T* ph = abase + A.row_hint * rstride;   // inside the buffer (host-checked)
#pragma unroll
        for (int i = 0; i < M; ++i) cur[i] = ph[i * np];
        bad = false;
        t_lane = A.misc->t[A.rd + in_vgpr(0)];         // a vector load, issued last
    } else {
        const int64_t rowa = floor_div(t0, hold);
        phase = (int)(t0 - rowa * hold);
        r = rowa - A.row0;
        bad = (r < 0 || r >= nrows);
        const T* p0 = abase + clamp_row(r) * rstride;
#pragma unroll
        for (int i = 0; i < M; ++i) cur[i] = p0[i * np];
        const T* p1 = abase + clamp_row(r + 1) * rstride;
#pragma unroll
        for (int i = 0; i < M; ++i) nxt[i] = p1[i * np];
        if (hold - phase < K && r + 1 >= nrows) bad = true;
    }
    if constexpr (!kSingle) __builtin_amdgcn_s_waitcnt(0);
    MGX_WAVE_TS(ts_loaded);
#pragma unroll
    for (int i = 0; i < M; ++i) cur[i] = clip1(cur[i]);
    T IA2[3], Brb[3];
    env_prologue<T, kPayload>(C, E, IA2, Brb);
    if constexpr (kSingle) {
        const StateT<T, M> s_in = s;
        step_body<T, M, false, kShaped, kFins, kPayload, kComp>(C, E, IA2, Brb, s, cur, nullptr, &lo);
        const int64_t tc = uniform64(t_lane);
        if (tc != A.t_hint) {
            // not the step the host expected: the row the counter names, through volatile
            // loads (the compiler would otherwise merge them with the expected row's fetch
            // into one fetch placed after the counter's)
            r = floor_div(tc, hold) - A.row0;
            bad = (r < 0 || r >= nrows);
            const volatile T* p0 = abase + clamp_row(r) * rstride;
#pragma unroll
            for (int i = 0; i < M; ++i) cur[i] = clip1((T)p0[i * np]);
            s = s_in;
#pragma unroll
            for (int j = 0; j < 4; ++j) lo.q[j] = T(0);
            step_body<T, M, false, kShaped, kFins, kPayload, kComp>(C, E, IA2, Brb, s, cur, nullptr, &lo);
        }
        *t_single = tc;
    } else {

    // Runs of steps between action-row switches: the inner loop carries only its counter,
    // and the row bookkeeping happens once per hold interval.
    int k = 0;
    while (k < K) {
        const int64_t left = hold - phase;  // steps until the next row switch, >= 1
        const int run = (int64_t)(K - k) < left ? K - k : (int)left;
        for (int j = 0; j < run; ++j, ++k) {
            if constexpr (kOut) {
                T f[kForceLen];
                step_body<T, M, true, kShaped, kFins, kPayload, kComp>(C, E, IA2, Brb, s, cur, f, &lo);
                if (A.forces) {
                    T* fo = (T*)A.forces + k * A.force_stride + env;
#pragma unroll
                    for (int c = 0; c < kForceLen; ++c) fo[c * np] = f[c];
                }
                if (A.traj) {
                    T* to = (T*)A.traj + k * A.traj_stride + env;
#pragma unroll
                    for (int c = 0; c < 3; ++c) to[c * np] = s.p[c];
#pragma unroll
                    for (int c = 0; c < 4; ++c) to[(3 + c) * np] = s.q[c];
#pragma unroll
                    for (int c = 0; c < 6; ++c) to[(7 + c) * np] = s.nu[c];
#pragma unroll
                    for (int i = 0; i < M; ++i) to[(kStateFixed + i) * np] = s.n[i];
                }
            } else {
                step_body<T, M, false, kShaped, kFins, kPayload, kComp>(C, E, IA2, Brb, s, cur, nullptr, &lo);
            }
        }
        phase += run;
        if (phase == hold) {
            phase = 0;
            ++r;
#pragma unroll
            for (int i = 0; i < M; ++i) cur[i] = clip1(nxt[i]);
            const T* pn = abase + clamp_row(r + 1) * rstride;
#pragma unroll
            for (int i = 0; i < M; ++i) nxt[i] = pn[i * np];
            if (k + hold < K && r + 1 >= nrows) bad = true;
        }
    }
    }
    MGX_WAVE_TS(ts_stepped);
    if (bad && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&A.misc->err, kErrActionRow);

    // The same check as renorm_attitude, written out: as a call it changes the register
    // allocation of the fused loop (15 more instructions in the plain K-step kernel).
    {
        T n2 = fma_(s.q[3], s.q[3], fma_(s.q[2], s.q[2], fma_(s.q[1], s.q[1], s.q[0] * s.q[0])));
        T drift = abs_(n2 - T(1));
        if (drift > T(1e-6)) {
            double qd[4] = {(double)s.q[0], (double)s.q[1], (double)s.q[2], (double)s.q[3]};
            double inv = 1.0 / sqrt(qd[0] * qd[0] + qd[1] * qd[1] + qd[2] * qd[2] + qd[3] * qd[3]);
#pragma unroll
            for (int j = 0; j < 4; ++j) s.q[j] = (T)(qd[j] * inv);
            st[kStRenorm] = 1.0f;
        }
        st[kStMaxDrift] = (float)drift;
    }

    if (!kSingle || env < np) store_state<T, M>(S, np, env, s);
#ifdef MGX_WAVE_TIMESTAMPS
    __builtin_amdgcn_s_waitcnt(0);
    MGX_WAVE_TS(ts_stored);
    {
        const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0 && w < kWaveTsMax) {
            g_wave_ts[w][0] = ts_entry;
            g_wave_ts[w][1] = ts_loaded;
            g_wave_ts[w][2] = ts_stepped;
            g_wave_ts[w][3] = ts_stored;
        }
    }
#endif

    if (A.partials) {
        if (env < A.nvalid) {
            bool fin = true;
#pragma unroll
            for (int j = 0; j < 3; ++j) fin &= finite_(s.p[j]);
#pragma unroll
            for (int j = 0; j < 4; ++j) fin &= finite_(s.q[j]);
#pragma unroll
            for (int j = 0; j < 6; ++j) fin &= finite_(s.nu[j]);
#pragma unroll
            for (int i = 0; i < M; ++i) fin &= finite_(s.n[i]);
            if (fin) {
                float sp = (float)sqrt_(s.nu[0] * s.nu[0] + s.nu[1] * s.nu[1] + s.nu[2] * s.nu[2]);
                float rt = (float)sqrt_(s.nu[3] * s.nu[3] + s.nu[4] * s.nu[4] + s.nu[5] * s.nu[5]);
                // nu^T (M_RB + M_A) nu. Diagonal M: (m + A_j) v_j^2 + (I_j + A_{3+j}) w_j^2.
                // With a payload the full M: m |v|^2 + A_1 v.v - 2 v.(m r_g x w) + w^T (I_o + A_2) w.
                const T* v = s.nu;
                const T* w = s.nu + 3;
                T ke = T(0);
                if constexpr (kPayload) {
                    T mrw[3], Iw[3];
                    cross(E.mrg, w, mrw);
                    Iw[0] = fma_(E.IoA[4], w[2], fma_(E.IoA[3], w[1], E.IoA[0] * w[0]));
                    Iw[1] = fma_(E.IoA[5], w[2], fma_(E.IoA[1], w[1], E.IoA[3] * w[0]));
                    Iw[2] = fma_(E.IoA[2], w[2], fma_(E.IoA[5], w[1], E.IoA[4] * w[0]));
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        ke += v[j] * ((E.mass + E.A[j]) * v[j] - T(2) * mrw[j]) + w[j] * Iw[j];
                } else {
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        ke += (E.mass + E.A[j]) * (v[j] * v[j]) + IA2[j] * (w[j] * w[j]);
                }
                st[kStMaxSpeed] = sp;
                st[kStSumSpeed] = sp;
                st[kStMaxRate] = rt;
                st[kStSumRate] = rt;
                st[kStSumKin] = (float)(T(0.5) * ke);
            } else {
                st[kStNonFinite] = 1.0f;
                st[kStMaxDrift] = 0.0f;
                st[kStRenorm] = 0.0f;
            }
        } else {
            st[kStRenorm] = 0.0f;
            st[kStMaxDrift] = 0.0f;
        }
    }
}

}  // namespace mgx
