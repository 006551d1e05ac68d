// One step of the batched underwater-vehicle dynamics for a single environment held in
// registers. Templated on the arithmetic type T (float, double, or a host-side counting
// type that measures the algorithmic cost) and on the thruster count M, so that the
// thruster loops unroll and the per-environment state lives in VGPRs.
//
// Order of the step (MarineGym, arXiv 2503.09203: Sec. III-D for the rotor and thrust
// models, Sec. III-B Eqs. (1)-(3) for the forces, the ocean-current substitution v_r):
//   1. rotor lag        n+ = n + alpha (a - n)            (a already clipped to [-1, 1])
//   2. thrust           f_i = k_i s_i |s_i|, s_i = sgn(n+_i) max(|n+_i| - delta_i, 0);
//                       tau = B f, B columns [e_i ; r_i x e_i] (k_i folded into B at setup)
//   3. kinematics       R(q); g_b = R^T e_z; v_c = R^T V_c; v_r = v - v_c
//   4. forces           Coriolis of rigid body and added mass, damping, restoring, and
//                       the added-mass term of the rotating current projection
//   5. solve            nu+ = nu + (dt M^-1) F,  M = M_RB + M_A (diagonal here)
//   6. pose             p+ = p + dt R v+;  q+ = q (x) exp(dt w+ / 2), renormalised
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

namespace mgx {

constexpr int kMaxThr = 8;
constexpr int kStateFixed = 13;
constexpr int kRecLen = 30;
// Classes with a payload (centre of gravity off the body origin) store the off-diagonal
// entries of the symmetric dt M^-1 in 15 more rows, (0,1), (0,2), ..., (4,5) row by row.
constexpr int kRecMinvOff = 30;
constexpr int kRecLenPayload = 45;
constexpr int kForceLen = 12;
constexpr int kWave = 64;

// Per-environment record fields (component-major rows of the record buffer).
enum RecField : int {
    kRecDtMinv = 0,   // dt / M_jj, j < 6
    kRecMass = 6,     // m
    kRecAdded = 7,    // M_A diagonal, 6
    kRecDlin = 13,    // 6
    kRecDquad = 19,   // 6
    kRecWmB = 25,     // W - B
    kRecBuoy = 26,    // B
    kRecCurrent = 27  // V_c world, 3
};

// Batch flags (mirror of the public header).
constexpr uint32_t kFlagNoAmc = 1u;
constexpr uint32_t kFlagLagEuler = 2u;

// Per-class constants in the batch precision, derived in double on the device.
template <typename T>
struct ClassT {
    T Bk[6][kMaxThr];  // thruster layout columns [e_i; r_i x e_i] scaled by the thrust gain k_i
    T alpha[kMaxThr];  // lag factor
    T dz[kMaxThr];     // dead zone
    T inertia[3];
    T rb[3];
    T g0, dt, inv_dt, half_dt;
    int32_t m;
    uint32_t flags;    // batch flags
    int32_t shaped;    // any dead zone or direction-dependent gain
    int32_t pad2;
    T rev[kMaxThr];    // reverse gain over forward gain (1 when symmetric)
    // Fins (rudders): bit i of fin_mask marks actuator i as a fin (its layout columns are
    // zero). Position, in-plane basis (chord at zero deflection, and span x chord), largest
    // deflection, lift and drag gains.
    uint32_t fin_mask;
    int32_t pad3;
    T fin_r[kMaxThr][3];
    T fin_c[kMaxThr][3];
    T fin_n[kMaxThr][3];
    T fin_max[kMaxThr];
    T fin_kl[kMaxThr];
    T fin_kd0[kMaxThr];
    T fin_kd[kMaxThr];
    // Payload: centre of gravity from the body origin (inertia given about it).
    T rg[3];
    int32_t payload;
    int32_t pad4;
};

template <typename T>
struct EnvT {
    T dtMinv[6];
    T mass;
    T A[6];
    T dL[6];
    T dQ[6];
    T wmb;
    T buoy;
    T Vc[3];
    T Ah[3];  // coefficients of the added-mass current term: A1, or 0 with kFlagNoAmc
    // payload only: off-diagonal dt M^-1, I_o + A_2 (xx, yy, zz, xy, xz, yz), m r_g
    T dtMinvOff[15];
    T IoA[6];
    T mrg[3];
};

// Fills EnvT::Ah from the added mass and the batch flags (once per environment, so that
// the step loop carries no branch on the flag).
template <typename T>
__host__ __device__ __forceinline__ void set_amc(EnvT<T>& E, uint32_t flags) {
#pragma unroll
    for (int j = 0; j < 3; ++j) E.Ah[j] = (flags & kFlagNoAmc) ? T(0) : E.A[j];
}

template <typename T, int M>
struct StateT {
    T p[3];
    T q[4];
    T nu[6];
    T n[M];
};

// Low-order words of the attitude for the compensated update: the quaternion is then the
// unevaluated sum hi + lo of each component, with |lo| <= ulp(hi) / 2. Rounding the
// attitude to float every step turns its direction by about 2^-24 rad per step; on
// trajectories that amplify attitude errors (classes with fins) those turns dominate the
// error after many steps, and carrying the low words through a launch removes them.
template <typename T>
struct StateLo {
    T q[4];
};

// hi + lo += x as an error-free transformation (Knuth's TwoSum of hi and x + lo): the new
// hi is the rounded sum, lo what the rounding dropped.
template <typename T>
__host__ __device__ __forceinline__ void two_sum_acc(T& hi, T& lo, T x) {
    const T y = x + lo;
    const T t = hi + y;
    const T bb = t - hi;
    lo = (hi - (t - bb)) + (y - bb);
    hi = t;
}

// ----------------------------------------------------------------------------- arithmetic

__host__ __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float abs_(float a) { return __builtin_fabsf(a); }
__host__ __device__ __forceinline__ double abs_(double a) { return __builtin_fabs(a); }
__host__ __device__ __forceinline__ float max_(float a, float b) { return __builtin_fmaxf(a, b); }
__host__ __device__ __forceinline__ double max_(double a, double b) { return __builtin_fmax(a, b); }
__host__ __device__ __forceinline__ float copysign_(float a, float b) { return __builtin_copysignf(a, b); }
__host__ __device__ __forceinline__ double copysign_(double a, double b) { return __builtin_copysign(a, b); }
__host__ __device__ __forceinline__ float sqrt_(float a) { return __builtin_sqrtf(a); }
__host__ __device__ __forceinline__ double sqrt_(double a) { return __builtin_sqrt(a); }
// 1/sqrt: the hardware reciprocal square root in float on the device (about 1 ulp), the
// correctly rounded quotient on the host and in double.
__device__ __forceinline__ float rsqrt_(float a) { return __builtin_amdgcn_rsqf(a); }
__host__ __forceinline__ float rsqrt_(float a) { return 1.0f / __builtin_sqrtf(a); }
__host__ __device__ __forceinline__ double rsqrt_(double a) { return 1.0 / __builtin_sqrt(a); }

// True if the predicate holds on any active lane of the wavefront (on the host: itself).
__device__ __forceinline__ bool any_lane(bool p) { return __any(p); }
__host__ __forceinline__ bool any_lane(bool p) { return p; }

// Command clip to [-1, 1] that lets NaN through (a NaN command marks the env non-finite).
template <typename T>
__host__ __device__ __forceinline__ T clip1(T a) {
    return a < T(-1) ? T(-1) : (a > T(1) ? T(1) : a);
}

// Per-lane selection (a vector select on the device).
template <typename T>
__host__ __device__ __forceinline__ T select_(bool c, T a, T b) {
    return c ? a : b;
}

template <typename T>
__host__ __device__ __forceinline__ void cross(const T a[3], const T b[3], T out[3]) {
    out[0] = fma_(a[1], b[2], -(a[2] * b[1]));
    out[1] = fma_(a[2], b[0], -(a[0] * b[2]));
    out[2] = fma_(a[0], b[1], -(a[1] * b[0]));
}

// acc - a x b, component-wise, as two fused multiply-adds per component.
template <typename T>
__host__ __device__ __forceinline__ void sub_cross(const T a[3], const T b[3], T acc[3]) {
    acc[0] = fma_(a[2], b[1], fma_(-a[1], b[2], acc[0]));
    acc[1] = fma_(a[0], b[2], fma_(-a[2], b[0], acc[1]));
    acc[2] = fma_(a[1], b[0], fma_(-a[0], b[1], acc[2]));
}

// sin and cos of a fin deflection. float: Taylor polynomials to x^9 and x^10 (truncation
// below 2e-9 for |x| <= pi/4, the largest deflection a class may declare) with an exact
// fallback when any lane is outside that range; double: the exact functions.
template <typename T>
__host__ __device__ __forceinline__ void sincos_deflection(T x, T& s, T& c) {
    if constexpr (std::is_same<T, double>::value) {
        s = sin(x);
        c = cos(x);
    } else {
        const T x2 = x * x;
        s = x * fma_(fma_(fma_(fma_(x2, T(1.0f / 362880.0f), T(-1.0f / 5040.0f)), x2, T(1.0f / 120.0f)), x2,
                         T(-1.0f / 6.0f)),
                     x2, T(1.0f));
        c = fma_(fma_(fma_(fma_(fma_(x2, T(-1.0f / 3628800.0f), T(1.0f / 40320.0f)), x2, T(-1.0f / 720.0f)), x2,
                           T(1.0f / 24.0f)),
                      x2, T(-0.5f)),
                 x2, T(1.0f));
        const bool big = !(abs_(x) <= T(0.7854f));
        if (__builtin_expect(any_lane(big), 0)) {
            T se, ce;
            if constexpr (std::is_same<T, float>::value) {
                sincosf(x, &se, &ce);
            } else {
                se = sin(x);
                ce = cos(x);
            }
            s = big ? se : s;
            c = big ? ce : c;
        }
    }
}

// Fin (rudder) forces added to tau. Fin i at r_i moves through the water at
// u = v_r + w x r_i; with (u_c, u_n) its components on the fin plane's basis (chord c at
// zero deflection, n = span x c) and delta = delta_max n_i the deflection, the angle of
// attack satisfies |u_p| sin(a) = sin(d) u_c - cos(d) u_n and |u_p| cos(a) = cos(d) u_c +
// sin(d) u_n, so no angle is formed. Lift K_L sin(a)cos(a)|u_p|^2 acts along
// span x u_p / |u_p| = (u_c n - u_n c) / |u_p|, drag (K_D0 + K_D sin^2(a))|u_p|^2 along
// -u_p / |u_p|; the force F acts at r_i, adding [F; r_i x F].
template <typename T, int M>
__host__ __device__ __forceinline__ void add_fin_wrench(const ClassT<T>& C, const T nl[M], const T vr[3],
                                                        const T w[3], T tau[6]) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (!((C.fin_mask >> i) & 1u)) continue;
        const T* r = C.fin_r[i];
        T u[3] = {vr[0], vr[1], vr[2]};
        sub_cross(r, w, u);  // u + w x r = u - r x w
        const T uc = fma_(u[2], C.fin_c[i][2], fma_(u[1], C.fin_c[i][1], u[0] * C.fin_c[i][0]));
        const T un = fma_(u[2], C.fin_n[i][2], fma_(u[1], C.fin_n[i][1], u[0] * C.fin_n[i][0]));
        const T wp2 = fma_(un, un, uc * uc);
        T sd, cd;
        sincos_deflection(C.fin_max[i] * nl[i], sd, cd);
        const T sa = fma_(sd, uc, -(cd * un));  // |u_p| sin(a)
        const T ca = fma_(cd, uc, sd * un);     // |u_p| cos(a)
        const T inv = wp2 > T(0) ? rsqrt_(wp2) : T(0);
        const T kl = C.fin_kl[i] * (sa * ca) * inv;
        const T kd = fma_(C.fin_kd[i], sa * sa, C.fin_kd0[i] * wp2) * inv;
        const T fc = fma_(-kl, un, -(kd * uc));
        const T fn = fma_(kl, uc, -(kd * un));
        T F[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            F[j] = fma_(fc, C.fin_c[i][j], fn * C.fin_n[i][j]);
            tau[j] += F[j];
        }
        T rf[3];
        cross(r, F, rf);
#pragma unroll
        for (int j = 0; j < 3; ++j) tau[3 + j] += rf[j];
    }
}

// Unit-quaternion increment exp(h w) = (cos(phi), sin(phi) w/|w|), phi = h |w|.
// float: even polynomials in phi^2 (truncation below 3e-11 for phi <= 0.05) with an
// exact fallback above; double: the exact form.
template <typename T>
__host__ __device__ __forceinline__ void quat_increment(T h, const T w[3], T& c, T& s) {
    T w2 = fma_(w[2], w[2], fma_(w[1], w[1], w[0] * w[0]));
    if constexpr (std::is_same<T, double>::value) {
        T wn = sqrt_(w2);
        T phi = h * wn;
        c = cos(phi);
        s = wn > 0.0 ? sin(phi) / wn : h;
    } else {
        T phi2 = (h * h) * w2;
        c = fma_(fma_(phi2, T(1.0f / 24.0f), T(-0.5f)), phi2, T(1.0f));
        s = h * fma_(fma_(phi2, T(1.0f / 120.0f), T(-1.0f / 6.0f)), phi2, T(1.0f));
        // the exact form where the series is not accurate enough: evaluated by the whole
        // wavefront when any lane needs it and selected per lane, so the common case is one
        // uniform branch with no execution-mask bookkeeping; marked unlikely, so that the
        // common path falls through and a step takes no branch here
        const bool big = !(phi2 <= T(0.0025f));
        if (__builtin_expect(any_lane(big), 0)) {
            T phi = sqrt_(phi2);
            T sn, cs;
            if constexpr (std::is_same<T, float>::value) {
                sincosf(phi, &sn, &cs);
            } else {
                sn = sin(phi);
                cs = cos(phi);
            }
            const T se = sn * h / phi;
            c = big ? cs : c;
            s = big ? se : s;
        }
    }
}

// The same increment with its scalar part given as c - 1 = -2 sin^2(phi / 2), free of the
// cancellation in 1 - cos(phi), for the compensated attitude update.
template <typename T>
__host__ __device__ __forceinline__ void quat_increment_cm1(T h, const T w[3], T& cm1, T& s) {
    T w2 = fma_(w[2], w[2], fma_(w[1], w[1], w[0] * w[0]));
    if constexpr (std::is_same<T, double>::value) {
        T wn = sqrt_(w2);
        T phi = h * wn;
        T sh = sin(0.5 * phi);
        cm1 = -2.0 * sh * sh;
        s = wn > 0.0 ? sin(phi) / wn : h;
    } else {
        T phi2 = (h * h) * w2;
        cm1 = fma_(phi2, T(1.0f / 24.0f), T(-0.5f)) * phi2;
        s = h * fma_(fma_(phi2, T(1.0f / 120.0f), T(-1.0f / 6.0f)), phi2, T(1.0f));
        const bool big = !(phi2 <= T(0.0025f));
        if (__builtin_expect(any_lane(big), 0)) {
            T phi = sqrt_(phi2);
            T sn, cs;
            if constexpr (std::is_same<T, float>::value) {
                sincosf(T(0.5f) * phi, &sn, &cs);
            } else {
                sn = sin(T(0.5f) * phi);
                cs = cos(T(0.5f) * phi);
            }
            const T ce = T(-2.0f) * (sn * sn);
            const T se = (T(2.0f) * (sn * cs)) * h / phi;
            cm1 = big ? ce : cm1;
            s = big ? se : s;
        }
    }
}

// d/d(phi^2) of the attitude increment (cos(phi), h sin(phi)/phi), phi^2 = h^2 |w|^2,
// matching the branches of quat_increment.
template <typename T>
__host__ __device__ __forceinline__ void quat_increment_d(T h, T phi2, T& dc, T& ds) {
    if constexpr (std::is_same<T, double>::value) {
        if (phi2 < 1e-8) {
            dc = -0.5 + phi2 / 12.0;
            ds = h * (-1.0 / 6.0 + phi2 / 60.0);
        } else {
            const T phi = sqrt_(phi2);
            const T sn = sin(phi), cs = cos(phi);
            dc = -sn / (2.0 * phi);
            ds = h * (phi * cs - sn) / (2.0 * phi * phi2);
        }
    } else {
        if (phi2 <= T(0.0025f)) {
            dc = fma_(phi2, T(1.0f / 12.0f), T(-0.5f));
            ds = h * fma_(phi2, T(1.0f / 60.0f), T(-1.0f / 6.0f));
        } else {
            const T phi = sqrt_(phi2);
            T sn, cs;
            if constexpr (std::is_same<T, float>::value) {
                sincosf(phi, &sn, &cs);
            } else {
                sn = sin(phi);
                cs = cos(phi);
            }
            dc = -sn / (T(2) * phi);
            ds = h * (phi * cs - sn) / (T(2) * phi * phi2);
        }
    }
}

// The forward quantities of one step that its reverse pass needs and that cost more to
// recompute than to keep: thrust derivatives, the rotation, the relative velocity, the
// force, the attitude increment and its derivatives, the unnormalised attitude and its
// renormalisation factor. kTapeLen values per environment and step (fd padded to 8).
constexpr int kTapeLen = kMaxThr + 9 + 3 + 6 + 4 + 4 + 1;

template <typename T>
struct VjpTape {
    T fd[kMaxThr];  // d(thrust / k)/d(lagged rotor state)
    T R[9];         // R(q), row-major
    T vc[3];        // R^T V_c
    T F[6];         // right-hand side of M dnu/dt = F
    T c, sh, dc, dsh;
    T nq[4];        // q (x) dq before renormalisation
    T g;            // renormalisation factor
};

// dnu = (dt M^-1) F with the symmetric dt M^-1 of a payload class: diagonal entries in
// dtMinv, the others (0,1), (0,2), ..., (4,5) in dtMinvOff.
template <typename T>
__host__ __device__ __forceinline__ void payload_solve(const EnvT<T>& E, const T F[6], T dnu[6]) {
    constexpr int kOff[6][6] = {{-1, 0, 1, 2, 3, 4},   {0, -1, 5, 6, 7, 8},    {1, 5, -1, 9, 10, 11},
                                {2, 6, 9, -1, 12, 13}, {3, 7, 10, 12, -1, 14}, {4, 8, 11, 13, 14, -1}};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        T acc = E.dtMinv[i] * F[i];
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (j != i) acc = fma_(E.dtMinvOff[kOff[i][j]], F[j], acc);
        dnu[i] = acc;
    }
}

// One step. `a` holds commands already clipped to [-1, 1]. IA2 = I + A_2 and Brb = B r_b
// are per-environment constants hoisted out of the step loop by the caller. `forces`
// (optional, 12 values) receives the actuator wrench and the hydrodynamic wrench of
// Eq. (3) with d(nu)/dt the solved acceleration.
template <typename T, int M, bool kForces = false, bool kShaped = false, bool kFins = false, bool kPayload = false,
          bool kComp = false, bool kTape = false>
__host__ __device__ __forceinline__ void step_body(const ClassT<T>& C, const EnvT<T>& E, const T IA2[3],
                                                   const T Brb[3], StateT<T, M>& s, const T a[M],
                                                   T* forces = nullptr, StateLo<T>* lo = nullptr,
                                                   VjpTape<T>* tape = nullptr) {
    static_assert(!(kTape && (kFins || kPayload || kComp)), "the tape covers the diagonal propeller body");
    // 1. rotor lag (first-order hold; alpha = 1 is the zero-order rotor)
    T nl[M];
#pragma unroll
    for (int i = 0; i < M; ++i) nl[i] = fma_(C.alpha[i], a[i] - s.n[i], s.n[i]);

    // 2. thrust and thruster layout
    T tau[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if constexpr (kFins) {
            if ((C.fin_mask >> i) & 1u) continue;  // fins push through add_fin_wrench
        }
        T f;  // thrust divided by the forward gain k_i (folded into Bk)
        if constexpr (kShaped) {
            // dead zone, and the reverse gain as a ratio to the forward one
            T mag = max_(abs_(nl[i]) - C.dz[i], T(0));
            const T g = select_(nl[i] < T(0), C.rev[i], T(1));
            f = copysign_(g * (mag * mag), nl[i]);
            if constexpr (kTape) tape->fd[i] = T(2) * g * mag;
        } else {
            f = nl[i] * abs_(nl[i]);
            if constexpr (kTape) tape->fd[i] = T(2) * abs_(nl[i]);
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) tau[j] = fma_(C.Bk[j][i], f, tau[j]);
    }

    // 3. kinematics
    const T qw = s.q[0], qx = s.q[1], qy = s.q[2], qz = s.q[3];
    const T x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
    const T xx = qx * x2, yy = qy * y2, zz = qz * z2;
    const T xy = qx * y2, xz = qx * z2, yz = qy * z2;
    const T wx = qw * x2, wy = qw * y2, wz = qw * z2;
    T R[3][3];
    R[0][0] = T(1) - (yy + zz);
    R[0][1] = xy - wz;
    R[0][2] = xz + wy;
    R[1][0] = xy + wz;
    R[1][1] = T(1) - (xx + zz);
    R[1][2] = yz - wx;
    R[2][0] = xz - wy;
    R[2][1] = yz + wx;
    R[2][2] = T(1) - (xx + yy);
    const T gb[3] = {R[2][0], R[2][1], R[2][2]};
    T vc[3], vr[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        vc[j] = fma_(R[2][j], E.Vc[2], fma_(R[1][j], E.Vc[1], R[0][j] * E.Vc[0]));
        vr[j] = s.nu[j] - vc[j];
    }
    if constexpr (kTape) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            tape->vc[i] = vc[i];
#pragma unroll
            for (int j = 0; j < 3; ++j) tape->R[3 * i + j] = R[i][j];
        }
    }
    const T* v = s.nu;
    const T* w = s.nu + 3;
    if constexpr (kFins) add_fin_wrench<T, M>(C, nl, vr, w, tau);

    // 4. forces, accumulated per degree of freedom into the right-hand side F of
    // M dnu/dt = F (every term evaluated at the step-start velocity)
    T A1vr[3], P[3], L[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A1vr[j] = E.A[j] * vr[j];
        P[j] = fma_(E.mass, v[j], A1vr[j]);
        if constexpr (!kPayload) L[j] = IA2[j] * w[j];
    }
    if constexpr (kPayload) {
        // with the centre of gravity at r_g: m w x (v + w x r_g) in the linear rows, so
        // P gains w x (m r_g); the angular rows use the full I_o + A_2
        sub_cross(E.mrg, w, P);
        // IoA: xx, yy, zz, xy, xz, yz
        L[0] = fma_(E.IoA[4], w[2], fma_(E.IoA[3], w[1], E.IoA[0] * w[0]));
        L[1] = fma_(E.IoA[5], w[2], fma_(E.IoA[1], w[1], E.IoA[3] * w[0]));
        L[2] = fma_(E.IoA[2], w[2], fma_(E.IoA[5], w[1], E.IoA[4] * w[0]));
    }
    T Fl[3], Fa[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fl[j] = fma_(E.wmb, gb[j], tau[j]);  // restoring, linear rows: -(W - B) g_b moved right
        Fa[j] = tau[3 + j];
    }
    // Coriolis, linear rows: m w x v + w x (A1 v_r) = w x (m v + A1 v_r)
    sub_cross(w, P, Fl);
    // angular rows: w x (I w) + w x (A2 w) + v_r x (A1 v_r) = w x ((I + A2) w) + v_r x (A1 v_r)
    sub_cross(w, L, Fa);
    sub_cross(vr, A1vr, Fa);
    if constexpr (kPayload) {
        // payload: m r_g x (w x v) in the angular rows
        T wxv[3];
        cross(w, v, wxv);
        sub_cross(E.mrg, wxv, Fa);
    }
    // restoring, angular rows: B r_b x g_b (with a payload, (B r_b - W r_g) x g_b: the
    // caller folds the weight's moment into Brb)
    sub_cross(Brb, gb, Fa);
    // added-mass term of the rotating current projection: A1 (w x v_c) (coefficients 0
    // when the term is switched off)
    T wvc[3];
    cross(w, vc, wvc);
    // damping on nu_r = (v_r, w): (d_L + d_Q |x|) x per degree of freedom
    T dcl[3], dca[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fl[j] = fma_(-E.Ah[j], wvc[j], Fl[j]);
        dcl[j] = fma_(E.dQ[j], abs_(vr[j]), E.dL[j]);
        dca[j] = fma_(E.dQ[3 + j], abs_(w[j]), E.dL[3 + j]);
        Fl[j] = fma_(-dcl[j], vr[j], Fl[j]);
        Fa[j] = fma_(-dca[j], w[j], Fa[j]);
    }

    if constexpr (kForces) {  // evaluated with the step-start velocity
        // actuator wrench, and the hydrodynamic wrench -M_A d(nu)/dt - C_A nu_r - D nu_r -
        // g_A - (A1 (w x v_c); 0) with d(nu)/dt the solved acceleration
        T cal[3], caa[3], A2w[3], t1[3], t2[3], rmom[3];
        cross(w, A1vr, cal);
#pragma unroll
        for (int j = 0; j < 3; ++j) A2w[j] = E.A[3 + j] * w[j];
        cross(vr, A1vr, t1);
        cross(w, A2w, t2);
        if constexpr (kPayload) {
            T Bb[3] = {E.buoy * C.rb[0], E.buoy * C.rb[1], E.buoy * C.rb[2]};
            cross(Bb, gb, rmom);
        } else {
            cross(Brb, gb, rmom);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) caa[j] = t1[j] + t2[j];
#pragma unroll
        for (int j = 0; j < 6; ++j) forces[j] = tau[j];
        T dnu[6];
        if constexpr (kPayload) {
            const T F6[6] = {Fl[0], Fl[1], Fl[2], Fa[0], Fa[1], Fa[2]};
            payload_solve(E, F6, dnu);
        } else {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                dnu[j] = E.dtMinv[j] * Fl[j];
                dnu[3 + j] = E.dtMinv[3 + j] * Fa[j];
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            forces[6 + j] = -(E.A[j] * dnu[j] * C.inv_dt) - E.Ah[j] * wvc[j] - cal[j] - dcl[j] * vr[j] -
                            E.buoy * gb[j];
            forces[9 + j] = -(E.A[3 + j] * dnu[3 + j] * C.inv_dt) - caa[j] - dca[j] * w[j] - rmom[j];
        }
    }

    if constexpr (kTape) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            tape->F[j] = Fl[j];
            tape->F[3 + j] = Fa[j];
        }
    }

    // 5. acceleration solve and velocity update: diagonal M, or the full symmetric
    // dt M^-1 of a class with a payload
    if constexpr (kPayload) {
        const T F6[6] = {Fl[0], Fl[1], Fl[2], Fa[0], Fa[1], Fa[2]};
        T dnu[6];
        payload_solve(E, F6, dnu);
#pragma unroll
        for (int j = 0; j < 6; ++j) s.nu[j] += dnu[j];
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            s.nu[j] = fma_(E.dtMinv[j], Fl[j], s.nu[j]);
            s.nu[3 + j] = fma_(E.dtMinv[3 + j], Fa[j], s.nu[3 + j]);
        }
    }

    // 6. pose: position with the updated velocity and the step-start attitude
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T rv = fma_(R[j][2], s.nu[2], fma_(R[j][1], s.nu[1], R[j][0] * s.nu[0]));
        s.p[j] = fma_(C.dt, rv, s.p[j]);
    }
    // attitude: body-frame increment on the right
    if constexpr (kComp) {
        // compensated: q (x) dq - q = q (c - 1) + q (x) (0, d) added to q_hi + q_lo, then
        // the Newton step toward |q| = 1 applied as q_hi += q_hi (g - 1)
        T cm1, sh;
        quat_increment_cm1(C.half_dt, s.nu + 3, cm1, sh);
        const T dx = sh * s.nu[3], dy = sh * s.nu[4], dz = sh * s.nu[5];
        const T d0 = fma_(qw, cm1, -fma_(qx, dx, fma_(qy, dy, qz * dz)));
        const T d1 = fma_(qw, dx, fma_(qx, cm1, fma_(qy, dz, -(qz * dy))));
        const T d2 = fma_(qw, dy, fma_(qy, cm1, fma_(qz, dx, -(qx * dz))));
        const T d3 = fma_(qw, dz, fma_(qz, cm1, fma_(qx, dy, -(qy * dx))));
        two_sum_acc(s.q[0], lo->q[0], d0);
        two_sum_acc(s.q[1], lo->q[1], d1);
        two_sum_acc(s.q[2], lo->q[2], d2);
        two_sum_acc(s.q[3], lo->q[3], d3);
        // |q|^2 - 1 with the low words' first-order part
        T n2m1 = fma_(s.q[3], s.q[3], fma_(s.q[2], s.q[2], fma_(s.q[1], s.q[1], fma_(s.q[0], s.q[0], T(-1)))));
        T cr = fma_(s.q[3], lo->q[3], fma_(s.q[2], lo->q[2], fma_(s.q[1], lo->q[1], s.q[0] * lo->q[0])));
        const T gm1 = T(-0.5) * fma_(T(2), cr, n2m1);
#pragma unroll
        for (int j = 0; j < 4; ++j) two_sum_acc(s.q[j], lo->q[j], s.q[j] * gm1);
#pragma unroll
        for (int i = 0; i < M; ++i) s.n[i] = nl[i];
        return;
    }
    T c, sh;
    quat_increment(C.half_dt, s.nu + 3, c, sh);
    const T dx = sh * s.nu[3], dy = sh * s.nu[4], dz = sh * s.nu[5];
    T nq0 = fma_(qw, c, -fma_(qx, dx, fma_(qy, dy, qz * dz)));
    T nq1 = fma_(qw, dx, fma_(qx, c, fma_(qy, dz, -(qz * dy))));
    T nq2 = fma_(qw, dy, fma_(qy, c, fma_(qz, dx, -(qx * dz))));
    T nq3 = fma_(qw, dz, fma_(qz, c, fma_(qx, dy, -(qy * dx))));
    T n2 = fma_(nq3, nq3, fma_(nq2, nq2, fma_(nq1, nq1, nq0 * nq0)));
    T g;
    if constexpr (std::is_same<T, double>::value) {
        g = 1.0 / sqrt_(n2);
    } else {
        g = fma_(T(-0.5f), n2, T(1.5f));  // one Newton step toward 1/|q|
    }
    if constexpr (kTape) {
        const T* w1 = s.nu + 3;
        const T h = C.half_dt;
        const T phi2 = (h * h) * fma_(w1[2], w1[2], fma_(w1[1], w1[1], w1[0] * w1[0]));
        quat_increment_d(h, phi2, tape->dc, tape->dsh);
        tape->c = c;
        tape->sh = sh;
        tape->nq[0] = nq0;
        tape->nq[1] = nq1;
        tape->nq[2] = nq2;
        tape->nq[3] = nq3;
        tape->g = g;
    }
    s.q[0] = nq0 * g;
    s.q[1] = nq1 * g;
    s.q[2] = nq2 * g;
    s.q[3] = nq3 * g;
#pragma unroll
    for (int i = 0; i < M; ++i) s.n[i] = nl[i];
}

}  // namespace mgx
