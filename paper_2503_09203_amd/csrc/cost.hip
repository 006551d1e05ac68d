// Algorithmic cost of one environment-step, measured by running the very step body the
// kernels run on the host with a counting scalar type.
#include <hip/hip_runtime.h>

#include <cmath>

#include "adjoint.hpp"
#include "mgx.h"
#include "runtime_internal.hpp"
#include "step.hpp"

namespace mgx {

struct CostTally {
    double flops = 0, ops = 0;
};
static thread_local CostTally g_tally;

// A double that counts the arithmetic done on it: add/sub/mul 1 flop and 1 op, fused
// multiply-add 2 flops and 1 op, min/max/copysign/select 1 op; negation and absolute
// value are free operand modifiers on the vector ALU.
struct Cnt {
    double v = 0;
    constexpr Cnt() = default;
    constexpr Cnt(double x) : v(x) {}
};
static inline Cnt tally(double v, double fl, double op) {
    g_tally.flops += fl;
    g_tally.ops += op;
    return Cnt(v);
}
static inline Cnt operator+(Cnt a, Cnt b) { return tally(a.v + b.v, 1, 1); }
static inline Cnt operator-(Cnt a, Cnt b) { return tally(a.v - b.v, 1, 1); }
static inline Cnt operator*(Cnt a, Cnt b) { return tally(a.v * b.v, 1, 1); }
static inline Cnt operator/(Cnt a, Cnt b) { return tally(a.v / b.v, 1, 1); }
static inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
static inline Cnt& operator+=(Cnt& a, Cnt b) { return a = a + b; }
static inline Cnt& operator-=(Cnt& a, Cnt b) { return a = a - b; }
static inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
static inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
static inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
static inline Cnt fma_(Cnt a, Cnt b, Cnt c) { return tally(std::fma(a.v, b.v, c.v), 2, 1); }
static inline Cnt abs_(Cnt a) { return Cnt(std::fabs(a.v)); }
static inline Cnt max_(Cnt a, Cnt b) { return tally(std::fmax(a.v, b.v), 0, 1); }
static inline Cnt copysign_(Cnt a, Cnt b) { return tally(std::copysign(a.v, b.v), 0, 1); }
static inline Cnt select_(bool c, Cnt a, Cnt b) { return tally(c ? a.v : b.v, 0, 1); }
static inline Cnt sqrt_(Cnt a) { return tally(std::sqrt(a.v), 1, 1); }
static inline Cnt rsqrt_(Cnt a) { return tally(1.0 / std::sqrt(a.v), 1, 1); }
static inline Cnt sin(Cnt a) { return tally(std::sin(a.v), 1, 1); }
static inline Cnt cos(Cnt a) { return tally(std::cos(a.v), 1, 1); }

template <int M>
static CostTally measure(uint32_t flags, uint32_t fin_mask = 0, bool payload = false) {
    ClassT<Cnt> C;
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < kMaxThr; ++i) C.Bk[j][i] = Cnt(3.0 * (i + 1) + 0.3 * j);
    for (int i = 0; i < kMaxThr; ++i) {
        C.alpha[i] = 0.1;
        C.dz[i] = (flags & MGX_COST_SHAPED) ? 0.05 : 0.0;
        C.rev[i] = (flags & MGX_COST_SHAPED) ? 0.7 : 1.0;
    }
    for (int j = 0; j < 3; ++j) {
        C.inertia[j] = 1.0 + j;
        C.rb[j] = j == 2 ? -0.01 : 0.0;
        C.rg[j] = payload ? 0.01 * (j + 1) : 0.0;
    }
    C.g0 = 9.81;
    C.dt = 0.01;
    C.inv_dt = 100;
    C.half_dt = 0.005;
    C.m = M;
    C.flags = flags & ~MGX_COST_SHAPED;
    C.shaped = (flags & MGX_COST_SHAPED) ? 1 : 0;
    C.fin_mask = fin_mask;
    C.payload = payload ? 1 : 0;
    for (int i = 0; i < kMaxThr; ++i) {
        const double r[3] = {-0.5, 0.1, 0.05}, c[3] = {1, 0, 0}, n[3] = {0, 1, 0};
        for (int j = 0; j < 3; ++j) {
            C.fin_r[i][j] = r[j];
            C.fin_c[i][j] = c[j];
            C.fin_n[i][j] = n[j];
        }
        C.fin_max[i] = 0.4;
        C.fin_kl[i] = 10;
        C.fin_kd0[i] = 0.3;
        C.fin_kd[i] = 5;
    }
    EnvT<Cnt> E;
    for (int j = 0; j < 6; ++j) {
        E.dtMinv[j] = 0.001;
        E.A[j] = 1.0;
        E.dL[j] = 5;
        E.dQ[j] = 20;
    }
    E.mass = 12;
    E.wmb = -1;
    E.buoy = 118;
    for (int j = 0; j < 3; ++j) E.Vc[j] = 0.1 * (j + 1);
    set_amc(E, flags & ~MGX_COST_SHAPED);
    Cnt IA2[3] = {2, 3, 4}, Brb[3] = {0, 0, -1.18};
    StateT<Cnt, M> s;
    for (int j = 0; j < 3; ++j) s.p[j] = 0;
    s.q[0] = 0.9;
    s.q[1] = 0.1;
    s.q[2] = 0.3;
    s.q[3] = -0.2;
    for (int j = 0; j < 6; ++j) s.nu[j] = 0.1 * (j - 2);
    for (int i = 0; i < M; ++i) s.n[i] = 0.1 * i - 0.3;
    Cnt a[M];
    for (int i = 0; i < M; ++i) a[i] = 0.5 - 0.1 * i;
    for (int k = 0; k < 15; ++k) E.dtMinvOff[k] = 1e-5;
    for (int j = 0; j < 6; ++j) E.IoA[j] = j < 3 ? 2.0 + j : 0.01;
    for (int j = 0; j < 3; ++j) E.mrg[j] = 0.1 * (j + 1);
    g_tally = CostTally();
    // classes with fins run the compensated attitude update in float
    StateLo<Cnt> lo;
    for (int j = 0; j < 4; ++j) lo.q[j] = 0.0;
    if (payload && fin_mask)
        step_body<Cnt, M, false, true, true, true, true>(C, E, IA2, Brb, s, a, nullptr, &lo);
    else if (payload)
        step_body<Cnt, M, false, true, false, true>(C, E, IA2, Brb, s, a);
    else if (fin_mask)
        step_body<Cnt, M, false, true, true, false, true>(C, E, IA2, Brb, s, a, nullptr, &lo);
    else if (flags & MGX_COST_SHAPED)
        step_body<Cnt, M, false, true>(C, E, IA2, Brb, s, a);
    else
        step_body<Cnt, M, false>(C, E, IA2, Brb, s, a);
    return g_tally;
}

// The reverse sweep's arithmetic per environment-step: the hand-written vector-Jacobian
// product of the step (its forward recomputation included), counted like the step itself.
template <int M>
static CostTally measure_vjp(uint32_t flags) {
    ClassT<Cnt> C;
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < kMaxThr; ++i) C.Bk[j][i] = Cnt(3.0 * (i + 1) + 0.3 * j);
    for (int i = 0; i < kMaxThr; ++i) {
        C.alpha[i] = 0.1;
        C.dz[i] = (flags & MGX_COST_SHAPED) ? 0.05 : 0.0;
        C.rev[i] = (flags & MGX_COST_SHAPED) ? 0.7 : 1.0;
    }
    for (int j = 0; j < 3; ++j) {
        C.inertia[j] = 1.0 + j;
        C.rb[j] = j == 2 ? -0.01 : 0.0;
        C.rg[j] = 0.0;
    }
    C.g0 = 9.81;
    C.dt = 0.01;
    C.inv_dt = 100;
    C.half_dt = 0.005;
    C.m = M;
    C.flags = flags & ~MGX_COST_SHAPED;
    C.shaped = (flags & MGX_COST_SHAPED) ? 1 : 0;
    C.fin_mask = 0;
    C.payload = 0;
    EnvT<Cnt> E;
    for (int j = 0; j < 6; ++j) {
        E.dtMinv[j] = 0.001;
        E.A[j] = 1.0;
        E.dL[j] = 5;
        E.dQ[j] = 20;
    }
    E.mass = 12;
    E.wmb = -1;
    E.buoy = 118;
    for (int j = 0; j < 3; ++j) E.Vc[j] = 0.1 * (j + 1);
    set_amc(E, flags & ~MGX_COST_SHAPED);
    Cnt IA2[3] = {2, 3, 4}, Brb[3] = {0, 0, -1.18};
    StateT<Cnt, M> s, xb;
    for (int j = 0; j < 3; ++j) s.p[j] = 0, xb.p[j] = 0.3;
    s.q[0] = 0.9;
    s.q[1] = 0.1;
    s.q[2] = 0.3;
    s.q[3] = -0.2;
    for (int j = 0; j < 4; ++j) xb.q[j] = 0.1 * j;
    for (int j = 0; j < 6; ++j) s.nu[j] = 0.1 * (j - 2), xb.nu[j] = 0.2;
    for (int i = 0; i < M; ++i) s.n[i] = 0.1 * i - 0.3, xb.n[i] = 0.05;
    Cnt a[M], ab[M], gdL[6], gdQ[6], gA[6], gDt[6];
    for (int i = 0; i < M; ++i) a[i] = 0.5 - 0.1 * i;
    for (int j = 0; j < 6; ++j) gdL[j] = gdQ[j] = gA[j] = gDt[j] = 0.0;
    // the forward quantities come from the tape the recomputation writes: only the reverse
    // part is the sweep's own work
    VjpTape<Cnt> tp;
    if (flags & MGX_COST_SHAPED)
        vjp_forward<Cnt, M, true>(C, E, IA2, Brb, s, a, tp);
    else
        vjp_forward<Cnt, M, false>(C, E, IA2, Brb, s, a, tp);
    g_tally = CostTally();
    if (flags & MGX_COST_SHAPED)
        vjp_reverse<Cnt, M, true>(C, E, IA2, Brb, s, tp, xb, ab, gdL, gdQ, gA, gDt);
    else
        vjp_reverse<Cnt, M, false>(C, E, IA2, Brb, s, tp, xb, ab, gdL, gdQ, gA, gDt);
    return g_tally;
}

}  // namespace mgx

extern "C" mgx_status mgx_vjp_cost(int32_t m, uint32_t batch_flags, double* flops, double* valu_ops) {
    using namespace mgx;
    if (!flops || !valu_ops) return fail(MGX_E_INVALID, "NULL argument");
    CostTally t;
    switch (m) {
        case 1: t = measure_vjp<1>(batch_flags); break;
        case 2: t = measure_vjp<2>(batch_flags); break;
        case 3: t = measure_vjp<3>(batch_flags); break;
        case 4: t = measure_vjp<4>(batch_flags); break;
        case 5: t = measure_vjp<5>(batch_flags); break;
        case 6: t = measure_vjp<6>(batch_flags); break;
        case 7: t = measure_vjp<7>(batch_flags); break;
        case 8: t = measure_vjp<8>(batch_flags); break;
        default: return fail(MGX_E_INVALID, "m=%d outside [1,8]", m);
    }
    *flops = t.flops;
    *valu_ops = t.ops;
    return MGX_OK;
}

extern "C" mgx_status mgx_step_cost(int32_t m, uint32_t batch_flags, double* flops, double* valu_ops) {
    using namespace mgx;
    if (!flops || !valu_ops) return fail(MGX_E_INVALID, "NULL argument");
    CostTally t;
    switch (m) {
        case 1: t = measure<1>(batch_flags); break;
        case 2: t = measure<2>(batch_flags); break;
        case 3: t = measure<3>(batch_flags); break;
        case 4: t = measure<4>(batch_flags); break;
        case 5: t = measure<5>(batch_flags); break;
        case 6: t = measure<6>(batch_flags); break;
        case 7: t = measure<7>(batch_flags); break;
        case 8: t = measure<8>(batch_flags); break;
        default: return fail(MGX_E_INVALID, "m=%d outside [1,8]", m);
    }
    *flops = t.flops;
    *valu_ops = t.ops;
    return MGX_OK;
}

extern "C" mgx_status mgx_class_step_cost(int32_t class_id, uint32_t batch_flags, double* flops, double* valu_ops) {
    using namespace mgx;
    if (!flops || !valu_ops) return fail(MGX_E_INVALID, "NULL argument");
    if (batch_flags & MGX_COST_SHAPED) return fail(MGX_E_INVALID, "MGX_COST_SHAPED is taken from the class");
    mgx_class_desc cd;
    if (!get_class(class_id, &cd)) return fail(MGX_E_INVALID, "class id %d unknown", class_id);
    const ClassDesc64 d = to_desc64(cd);
    const uint32_t fins = fin_mask_of(d);
    const bool pl = has_payload(d);
    const uint32_t f = batch_flags | (shaped_thrust(d) ? MGX_COST_SHAPED : 0u);
    CostTally t;
    switch (cd.m) {
        case 1: t = measure<1>(f, fins, pl); break;
        case 2: t = measure<2>(f, fins, pl); break;
        case 3: t = measure<3>(f, fins, pl); break;
        case 4: t = measure<4>(f, fins, pl); break;
        case 5: t = measure<5>(f, fins, pl); break;
        case 6: t = measure<6>(f, fins, pl); break;
        case 7: t = measure<7>(f, fins, pl); break;
        default: t = measure<8>(f, fins, pl); break;
    }
    *flops = t.flops;
    *valu_ops = t.ops;
    return MGX_OK;
}
