// Vector-Jacobian product of one step of the batched underwater-vehicle dynamics (the
// step_body of step.hpp), written out by hand in reverse order of the forward pass.
//
// Given the state before the step, the clipped commands, and the adjoint of the state
// after the step, it returns the adjoint of the state before the step and of the
// commands, and accumulates the adjoints of the per-environment damping (d_L, d_Q), of the
// added-mass diagonal through the Coriolis and current terms (direct part), and of
// dt M^-1 (chained to the added mass by the caller).
#pragma once

#include "step.hpp"

namespace mgx {

template <typename T>
__host__ __device__ __forceinline__ void qmul(const T a[4], const T b[4], T o[4]) {
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] + a[2] * b[0] + a[3] * b[1] - a[1] * b[3];
    o[3] = a[0] * b[3] + a[3] * b[0] + a[1] * b[2] - a[2] * b[1];
}

template <typename T>
__host__ __device__ __forceinline__ void cross_bar(const T x[3], const T y[3], const T zb[3], T xb[3], T yb[3]) {
    // z = x cross y:  xb += y cross zb,  yb += zb cross x
    T t[3];
    cross(y, zb, t);
    xb[0] += t[0];
    xb[1] += t[1];
    xb[2] += t[2];
    cross(zb, x, t);
    yb[0] += t[0];
    yb[1] += t[1];
    yb[2] += t[2];
}

// Forward part of the vector-Jacobian product: the step's quantities from the state before
// it and the clipped commands.
template <typename T, int M, bool kShaped = false>
__host__ __device__ __forceinline__ void vjp_forward(const ClassT<T>& C, const EnvT<T>& E, const T IA2[3],
                                                     const T Brb[3], const StateT<T, M>& s, const T a[M],
                                                     VjpTape<T>& tp) {
#pragma clang fp contract(fast)
    T tau[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const T nl = fma_(C.alpha[i], a[i] - s.n[i], s.n[i]);
        T f;
        if constexpr (kShaped) {
            const T mag = max_(abs_(nl) - C.dz[i], T(0));
            const T g = select_(nl < T(0), C.rev[i], T(1));
            f = copysign_(g * (mag * mag), nl);
            tp.fd[i] = T(2) * g * mag;
        } else {
            f = nl * abs_(nl);
            tp.fd[i] = T(2) * abs_(nl);
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) tau[j] = fma_(C.Bk[j][i], f, tau[j]);
    }
    const T qw = s.q[0], qx = s.q[1], qy = s.q[2], qz = s.q[3];
    const T x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
    const T xx = qx * x2, yy = qy * y2, zz = qz * z2;
    const T xy = qx * y2, xz = qx * z2, yz = qy * z2;
    const T wx = qw * x2, wy = qw * y2, wz = qw * z2;
    T* R = tp.R;
    R[0] = T(1) - (yy + zz);
    R[1] = xy - wz;
    R[2] = xz + wy;
    R[3] = xy + wz;
    R[4] = T(1) - (xx + zz);
    R[5] = yz - wx;
    R[6] = xz - wy;
    R[7] = yz + wx;
    R[8] = T(1) - (xx + yy);
    const T gb[3] = {R[6], R[7], R[8]};
    T* vc = tp.vc;
    T vr[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        vc[j] = fma_(R[6 + j], E.Vc[2], fma_(R[3 + j], E.Vc[1], R[j] * E.Vc[0]));
        vr[j] = s.nu[j] - vc[j];
    }
    const T* v = s.nu;
    const T* w = s.nu + 3;
    T A1vr[3], P[3], L[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A1vr[j] = E.A[j] * vr[j];
        P[j] = fma_(E.mass, v[j], A1vr[j]);
        L[j] = IA2[j] * w[j];
    }
    T cor_lin[3], cor_ang[3], t1[3];
    cross(w, P, cor_lin);
    cross(w, L, cor_ang);
    cross(vr, A1vr, t1);
#pragma unroll
    for (int j = 0; j < 3; ++j) cor_ang[j] = cor_ang[j] + t1[j];
    const bool amc = !(C.flags & kFlagNoAmc);
    T hA[3] = {T(0), T(0), T(0)};
    if (amc) {
        T wvc[3];
        cross(w, vc, wvc);
#pragma unroll
        for (int j = 0; j < 3; ++j) hA[j] = E.A[j] * wvc[j];
    }
    T damp[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        damp[j] = fma_(E.dQ[j], abs_(vr[j]), E.dL[j]) * vr[j];
        damp[3 + j] = fma_(E.dQ[3 + j], abs_(w[j]), E.dL[3 + j]) * w[j];
    }
    T rmom[3];
    cross(Brb, gb, rmom);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        tp.F[j] = fma_(E.wmb, gb[j], tau[j] - cor_lin[j] - damp[j] - hA[j]);
        tp.F[3 + j] = tau[3 + j] - cor_ang[j] - damp[3 + j] - rmom[j];
    }
    T w1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) w1[j] = s.nu[3 + j] + E.dtMinv[3 + j] * tp.F[3 + j];
    const T h = C.half_dt;
    const T w2 = fma_(w1[2], w1[2], fma_(w1[1], w1[1], w1[0] * w1[0]));
    quat_increment(h, w1, tp.c, tp.sh);
    const T phi2 = (h * h) * w2;
    quat_increment_d(h, phi2, tp.dc, tp.dsh);
    const T c = tp.c, sh = tp.sh;
    const T d1 = sh * w1[0], d2 = sh * w1[1], d3 = sh * w1[2];
    tp.nq[0] = fma_(qw, c, -fma_(qx, d1, fma_(qy, d2, qz * d3)));
    tp.nq[1] = fma_(qw, d1, fma_(qx, c, fma_(qy, d3, -(qz * d2))));
    tp.nq[2] = fma_(qw, d2, fma_(qy, c, fma_(qz, d1, -(qx * d3))));
    tp.nq[3] = fma_(qw, d3, fma_(qz, c, fma_(qx, d2, -(qy * d1))));
    const T n2 = fma_(tp.nq[3], tp.nq[3], fma_(tp.nq[2], tp.nq[2], fma_(tp.nq[1], tp.nq[1], tp.nq[0] * tp.nq[0])));
    if constexpr (std::is_same<T, double>::value) {
        tp.g = 1.0 / sqrt_(n2);
    } else {
        tp.g = fma_(T(-0.5f), n2, T(1.5f));
    }
}

// Reverse part: given the state before the step, its tape and the adjoint of the state
// after the step, the adjoint of the state before it and of the commands, accumulating the
// parameter adjoints. The cheap forward quantities are formed again from the state and the
// tape.
template <typename T, int M, bool kShaped = false>
__host__ __device__ __forceinline__ void vjp_reverse(const ClassT<T>& C, const EnvT<T>& E, const T IA2[3],
                                                     const T Brb[3], const StateT<T, M>& s, const VjpTape<T>& tp,
                                                     StateT<T, M>& xb, T abar[M], T gdL[6], T gdQ[6], T gA[6],
                                                     T gDt[6]) {
#pragma clang fp contract(fast)
    const T qw = s.q[0], qx = s.q[1], qy = s.q[2], qz = s.q[3];
    const T R[3][3] = {{tp.R[0], tp.R[1], tp.R[2]}, {tp.R[3], tp.R[4], tp.R[5]}, {tp.R[6], tp.R[7], tp.R[8]}};
    const T* vc = tp.vc;
    const T* F = tp.F;
    const T* v = s.nu;
    const T* w = s.nu + 3;
    T vr[3], A1vr[3], P[3], L[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        vr[j] = v[j] - vc[j];
        A1vr[j] = E.A[j] * vr[j];
        P[j] = fma_(E.mass, v[j], A1vr[j]);
        L[j] = IA2[j] * w[j];
    }
    const bool amc = !(C.flags & kFlagNoAmc);
    T wvc[3] = {T(0), T(0), T(0)};
    if (amc) cross(w, vc, wvc);
    T nu1[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) nu1[j] = s.nu[j] + E.dtMinv[j] * F[j];
    const T h = C.half_dt;
    const T* w1 = nu1 + 3;
    const T c = tp.c, sh = tp.sh, dc = tp.dc, dsh = tp.dsh;
    const T d[4] = {c, sh * w1[0], sh * w1[1], sh * w1[2]};
    const T* nq = tp.nq;
    const T g = tp.g;
    T dg;
    if constexpr (std::is_same<T, double>::value) {
        dg = -0.5 * g * g * g;
    } else {
        dg = T(-0.5f);
    }
    // ------------------------------------------------------------------ reverse
    // q+ = g nq
    T gbar = T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) gbar += xb.q[j] * nq[j];
    const T n2b = dg * gbar;
    T nqb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) nqb[j] = g * xb.q[j] + T(2) * n2b * nq[j];
    // nq = q (x) d:  qb = nqb (x) conj(d),  db = conj(q) (x) nqb
    T qb[4], db[4];
    {
        const T dconj[4] = {d[0], -d[1], -d[2], -d[3]};
        const T qconj[4] = {qw, -qx, -qy, -qz};
        qmul(nqb, dconj, qb);
        qmul(qconj, nqb, db);
    }
    // d = (c, sh w1), c and sh functions of phi2 = h^2 |w1|^2
    const T shb = db[1] * w1[0] + db[2] * w1[1] + db[3] * w1[2];
    const T phi2b = db[0] * dc + shb * dsh;
    T nu1b[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        nu1b[j] = xb.nu[j];
        nu1b[3 + j] = xb.nu[3 + j] + sh * db[1 + j] + T(2) * (h * h) * phi2b * w1[j];
    }
    // p+ = p + dt R v+  (xb.p passes through unchanged)
    T Rb[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Rb[i][j] = C.dt * xb.p[i] * nu1[j];
        }
#pragma unroll
    for (int j = 0; j < 3; ++j) nu1b[j] += C.dt * (R[0][j] * xb.p[0] + R[1][j] * xb.p[1] + R[2][j] * xb.p[2]);
    // nu+ = nu + dtMinv F
    T Fb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        Fb[j] = E.dtMinv[j] * nu1b[j];
        gDt[j] += F[j] * nu1b[j];
    }
    T taub[6], gbb[3], vb[3] = {T(0), T(0), T(0)}, wb[3] = {T(0), T(0), T(0)}, vrb[3] = {T(0), T(0), T(0)},
                       vcb[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        taub[j] = Fb[j];
        taub[3 + j] = Fb[3 + j];
        gbb[j] = E.wmb * Fb[j];
    }
    // restoring moment rmom = Brb x gb, F_ang -= rmom
    {
        const T rmomb[3] = {-Fb[3], -Fb[4], -Fb[5]};
        T t[3];
        cross(rmomb, Brb, t);
#pragma unroll
        for (int j = 0; j < 3; ++j) gbb[j] += t[j];
    }
    // damping
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T bl = -Fb[j], ba = -Fb[3 + j];
        vrb[j] += bl * fma_(T(2) * E.dQ[j], abs_(vr[j]), E.dL[j]);
        gdL[j] += bl * vr[j];
        gdQ[j] += bl * abs_(vr[j]) * vr[j];
        wb[j] += ba * fma_(T(2) * E.dQ[3 + j], abs_(w[j]), E.dL[3 + j]);
        gdL[3 + j] += ba * w[j];
        gdQ[3 + j] += ba * abs_(w[j]) * w[j];
    }
    // current term hA = A1 (w x vc), F_lin -= hA
    if (amc) {
        T ub[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gA[j] += -Fb[j] * wvc[j];
            ub[j] = E.A[j] * -Fb[j];
        }
        cross_bar(w, vc, ub, wb, vcb);
    }
    // Coriolis, linear rows: cor_lin = w x P, F_lin -= cor_lin
    T Pb[3] = {T(0), T(0), T(0)};
    {
        const T cb[3] = {-Fb[0], -Fb[1], -Fb[2]};
        cross_bar(w, P, cb, wb, Pb);
    }
    // angular rows: cor_ang = w x L + vr x A1vr, F_ang -= cor_ang
    T Lb[3] = {T(0), T(0), T(0)}, A1vrb[3] = {T(0), T(0), T(0)};
    {
        const T cb[3] = {-Fb[3], -Fb[4], -Fb[5]};
        cross_bar(w, L, cb, wb, Lb);
        cross_bar(vr, A1vr, cb, vrb, A1vrb);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // L = (I + A2) w
        wb[j] += IA2[j] * Lb[j];
        gA[3 + j] += w[j] * Lb[j];
        // P = m v + A1vr
        vb[j] += E.mass * Pb[j];
        A1vrb[j] += Pb[j];
        // A1vr = A1 vr
        gA[j] += vr[j] * A1vrb[j];
        vrb[j] += E.A[j] * A1vrb[j];
        // vr = v - vc
        vb[j] += vrb[j];
        vcb[j] -= vrb[j];
    }
    // vc = R^T Vc, gb = R^T e_z
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Rb[i][j] += vcb[j] * E.Vc[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) Rb[2][j] += gbb[j];
    // R(q)
    qb[0] += T(2) * (-qz * Rb[0][1] + qy * Rb[0][2] + qz * Rb[1][0] - qx * Rb[1][2] - qy * Rb[2][0] + qx * Rb[2][1]);
    qb[1] += T(2) * (qy * Rb[0][1] + qz * Rb[0][2] + qy * Rb[1][0] - qw * Rb[1][2] + qz * Rb[2][0] + qw * Rb[2][1]) -
             T(4) * qx * (Rb[1][1] + Rb[2][2]);
    qb[2] += T(2) * (qx * Rb[0][1] + qw * Rb[0][2] + qx * Rb[1][0] + qz * Rb[1][2] - qw * Rb[2][0] + qz * Rb[2][1]) -
             T(4) * qy * (Rb[0][0] + Rb[2][2]);
    qb[3] += T(2) * (-qw * Rb[0][1] + qx * Rb[0][2] + qw * Rb[1][0] + qy * Rb[1][2] + qx * Rb[2][0] + qy * Rb[2][1]) -
             T(4) * qz * (Rb[0][0] + Rb[1][1]);
    // thrust and lag
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T fb = T(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) fb = fma_(C.Bk[j][i], taub[j], fb);
        const T nlb = fb * tp.fd[i] + xb.n[i];
        abar[i] = C.alpha[i] * nlb;
        xb.n[i] = (T(1) - C.alpha[i]) * nlb;
    }
    // write the adjoint of the state before the step (p passes through)
#pragma unroll
    for (int j = 0; j < 4; ++j) xb.q[j] = qb[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        xb.nu[j] = nu1b[j] + vb[j];
        xb.nu[3 + j] = nu1b[3 + j] + wb[j];
    }
}


// The vector-Jacobian product of one step (written out by hand in reverse order of the
// forward pass): its forward part, then its reverse part.
template <typename T, int M, bool kShaped = false>
__host__ __device__ __forceinline__ void step_vjp(const ClassT<T>& C, const EnvT<T>& E, const T IA2[3], const T Brb[3],
                                                  const StateT<T, M>& s, const T a[M], StateT<T, M>& xb, T abar[M],
                                                  T gdL[6], T gdQ[6], T gA[6], T gDt[6]) {
    VjpTape<T> tp;
    vjp_forward<T, M, kShaped>(C, E, IA2, Brb, s, a, tp);
    vjp_reverse<T, M, kShaped>(C, E, IA2, Brb, s, tp, xb, abar, gdL, gdQ, gA, gDt);
}

}  // namespace mgx
