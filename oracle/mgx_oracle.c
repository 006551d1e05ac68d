/*
 * FP64 CPU oracle for the batched underwater-vehicle step. TEST INFRASTRUCTURE ONLY:
 * nothing in the product links or calls this file.
 *
 * Each function cites the passage of MarineGym (arXiv 2503.09203) it follows, and the
 * reading taken where the paper leaves a choice open:
 *   - equation of motion, Eq. (1) and its rigid-body / hydrodynamic split, Eq. (2);
 *   - hydrodynamic wrench, Eq. (3), with the relative velocity v_r = v - v_c of
 *     Sec. III-B ("ocean currents");
 *   - rotor models and propeller thrust, Sec. III-D (zero-order, first-order models;
 *     quadratic thrust with a dead zone); forces applied at each actuator frame.
 * The pose is a unit quaternion rather than the Euler angles of Eq. (1)'s eta; the
 * rigid body is integrated here (semi-implicit Euler, exponential-map attitude update)
 * instead of by an external physics engine.
 */
#include "mgx_oracle.h"

#include <math.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t orc_sizeof_env(void) { return (int32_t)sizeof(orc_env); }
int32_t orc_sizeof_state(void) { return (int32_t)sizeof(orc_state); }

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int32_t orc_get_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

static void cross3(const double a[3], const double b[3], double out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Body -> world rotation matrix of a unit quaternion (w, x, y, z). */
void orc_rotation(const double q[4], double R[3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Hamilton product a (x) b. */
void orc_quat_mul(const double a[4], const double b[4], double out[4]) {
    double av[3] = {a[1], a[2], a[3]}, bv[3] = {b[1], b[2], b[3]}, c[3];
    cross3(av, bv, c);
    out[0] = a[0] * b[0] - (av[0] * bv[0] + av[1] * bv[1] + av[2] * bv[2]);
    for (int j = 0; j < 3; ++j) out[1 + j] = a[0] * bv[j] + b[0] * av[j] + c[j];
}

/* Rotor dynamics, Sec. III-D. First-order model dn/dt = (a - n)/tau held over one step
 * gives n+ = n + alpha (a - n) with alpha = 1 - exp(-dt/tau). The zero-order model maps
 * the command straight to the rotor state (alpha = 1, tau = 0). */
double orc_lag_factor(const orc_env* env, int32_t i) {
    if (env->tau[i] <= 0.0) return 1.0;
    if (env->flags & ORC_FLAG_LAG_EULER) return env->dt / env->tau[i];
    return 1.0 - exp(-env->dt / env->tau[i]);
}

/* Propeller thrust, Sec. III-D: quadratic in the rotor state beyond a dead zone,
 * f_i = k_i s_i |s_i| with s_i = sgn(n_i) max(|n_i| - delta_i, 0). The gain may differ by
 * direction (k_i for s_i >= 0, the reverse gain for s_i < 0; unset = symmetric). Each force
 * acts along the thruster axis e_i at the thruster position r_i; the spinning propeller
 * also turns the hull about its own axis with a torque c_i f_i (c_i signed by the
 * propeller's handedness). About the CoG the wrench is sum_i f_i [e_i ; r_i x e_i + c_i e_i]. */
void orc_thrust_wrench(const orc_env* env, const double n[ORC_MAX_THR], double tau[6]) {
    for (int j = 0; j < 6; ++j) tau[j] = 0.0;
    for (int i = 0; i < env->m; ++i) {
        if (env->kind[i] == ORC_FIN) continue;
        double mag = fabs(n[i]) - env->deadzone[i];
        double s = mag > 0.0 ? (n[i] >= 0.0 ? mag : -mag) : 0.0;
        double gain = env->k[i];
        if (s < 0.0 && env->k_rev[i] > 0.0) gain = env->k_rev[i];
        double f = gain * s * fabs(s);
        double e[3], len = sqrt(env->e[i][0] * env->e[i][0] + env->e[i][1] * env->e[i][1] +
                                env->e[i][2] * env->e[i][2]);
        for (int j = 0; j < 3; ++j) e[j] = env->e[i][j] / len;
        double mom[3];
        cross3(env->r[i], e, mom);
        for (int j = 0; j < 3; ++j) {
            tau[j] += f * e[j];
            tau[3 + j] += f * mom[j] + env->reaction[i] * f * e[j];
        }
    }
}

/* Rudder (fin) forces, Sec. III-D: a simplified lift and drag law whose forces depend on
 * the flow speed at the fin, its area and lift and drag coefficients that vary with the
 * angle of attack. Fin i sits at r_i and moves through the water with u = v_r + w x r_i.
 * Its plane is normal to the span axis s; in that plane the chord at zero deflection is c
 * (e_i without its span component) and nn = s x c. The rotor state n_i (after the shared
 * lag) sets the deflection delta = delta_max n_i, turning the chord toward nn. With
 * u_p the in-plane part of u and beta = atan2(u_p . nn, u_p . c) its direction, the angle
 * of attack is alpha = delta - beta. Flat-plate coefficients: lift K_L sin(alpha)cos(alpha)
 * |u_p|^2 along s x u_p / |u_p|, drag (K_D0 + K_D sin^2(alpha)) |u_p|^2 against u_p. The
 * force acts at r_i: the wrench [F ; r_i x F] is added to tau. */
void orc_fin_wrench(const orc_env* env, const double n[ORC_MAX_THR], const double vr[3], const double w[3],
                    double tau[6]) {
    for (int i = 0; i < env->m; ++i) {
        if (env->kind[i] != ORC_FIN) continue;
        double s[3], c[3], nn[3], u[3], wxr[3];
        double sl = sqrt(env->span[i][0] * env->span[i][0] + env->span[i][1] * env->span[i][1] +
                         env->span[i][2] * env->span[i][2]);
        for (int j = 0; j < 3; ++j) s[j] = env->span[i][j] / sl;
        double es = env->e[i][0] * s[0] + env->e[i][1] * s[1] + env->e[i][2] * s[2];
        for (int j = 0; j < 3; ++j) c[j] = env->e[i][j] - es * s[j];
        double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int j = 0; j < 3; ++j) c[j] /= cl;
        cross3(s, c, nn);
        cross3(w, env->r[i], wxr);
        for (int j = 0; j < 3; ++j) u[j] = vr[j] + wxr[j];
        double uc = u[0] * c[0] + u[1] * c[1] + u[2] * c[2];
        double un = u[0] * nn[0] + u[1] * nn[1] + u[2] * nn[2];
        double speed2 = uc * uc + un * un;
        if (speed2 == 0.0) continue;
        double speed = sqrt(speed2);
        double up[3], lift_dir[3];
        for (int j = 0; j < 3; ++j) up[j] = (uc * c[j] + un * nn[j]) / speed;
        cross3(s, up, lift_dir);
        double alpha = env->fin_max[i] * n[i] - atan2(un, uc);
        double sa = sin(alpha), ca = cos(alpha);
        double L = env->fin_lift[i] * sa * ca * speed2;
        double D = (env->fin_drag0[i] + env->fin_drag[i] * sa * sa) * speed2;
        double F[3], mom[3];
        for (int j = 0; j < 3; ++j) F[j] = L * lift_dir[j] - D * up[j];
        cross3(env->r[i], F, mom);
        for (int j = 0; j < 3; ++j) {
            tau[j] += F[j];
            tau[3 + j] += mom[j];
        }
    }
}

/* Rigid-body inertia about the body origin when the centre of gravity sits at r_g from it
 * (a payload): I_o = I_g + m (|r_g|^2 1 - r_g r_g^T) (parallel axes), I_g diagonal. */
static void inertia_origin(const orc_env* env, double Io[3][3]) {
    const double* r = env->rg;
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Io[i][j] = (i == j ? env->inertia[i] + env->mass * r2 : 0.0) - env->mass * r[i] * r[j];
}

/* M = M_RB + M_A with M_RB = [m 1, -m S(r_g); m S(r_g), I_o] (Eq. (2), body origin away from
 * the CoG) and M_A diagonal; S(x) y = x x y. */
void orc_mass_matrix(const orc_env* env, double M[36]) {
    double Io[3][3];
    inertia_origin(env, Io);
    const double* r = env->rg;
    const double m = env->mass;
    double S[3][3] = {{0.0, -r[2], r[1]}, {r[2], 0.0, -r[0]}, {-r[1], r[0], 0.0}};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) M[6 * i + j] = 0.0;
    for (int i = 0; i < 3; ++i) {
        M[6 * i + i] = m;
        for (int j = 0; j < 3; ++j) {
            M[6 * i + 3 + j] = -m * S[i][j];
            M[6 * (3 + i) + j] = m * S[i][j];
            M[6 * (3 + i) + 3 + j] = Io[i][j];
        }
    }
    for (int j = 0; j < 6; ++j) M[6 * j + j] += env->added[j];
}

/* Solves M x = b (6x6) by Gaussian elimination with partial pivoting. */
static void solve6(const double M_in[36], const double b_in[6], double x[6]) {
    double M[36], b[6];
    memcpy(M, M_in, sizeof M);
    memcpy(b, b_in, sizeof b);
    for (int c = 0; c < 6; ++c) {
        int p = c;
        for (int i = c + 1; i < 6; ++i)
            if (fabs(M[6 * i + c]) > fabs(M[6 * p + c])) p = i;
        if (p != c) {
            for (int j = 0; j < 6; ++j) {
                double t = M[6 * c + j];
                M[6 * c + j] = M[6 * p + j];
                M[6 * p + j] = t;
            }
            double t = b[c];
            b[c] = b[p];
            b[p] = t;
        }
        for (int i = c + 1; i < 6; ++i) {
            double f = M[6 * i + c] / M[6 * c + c];
            if (f == 0.0) continue;
            for (int j = c; j < 6; ++j) M[6 * i + j] -= f * M[6 * c + j];
            b[i] -= f * b[c];
        }
    }
    for (int i = 5; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < 6; ++j) s -= M[6 * i + j] * x[j];
        x[i] = s / M[6 * i + i];
    }
}

/* Right-hand-side terms of Eqs. (1)-(3) at attitude q and velocity nu, with the
 * already-lagged rotor state n_lagged:
 *   C_RB(nu) nu  = [m w x (v + w x r_g) ; m r_g x (w x v) + w x (I_o w)]
 *                  (reduces to [m w x v ; w x (I w)] with the origin at the CoG)
 *   C_A(nu_r) nu_r = [w x (A1 v_r) ; v_r x (A1 v_r) + w x (A2 w)]  (diagonal added mass)
 *   D(nu_r) nu_r = (d_L + d_Q |nu_r|) nu_r per DOF
 *   g(eta) = [-(W - B) g_b ; B r_b x g_b], g_b = R^T e_z, W = m g0
 *   hadd   = [A1 (w x v_c) ; 0]: the current seen in the body frame rotates with the
 *            body, so substituting v_r into -M_A d(nu)/dt of Eq. (3) leaves this term.
 * v_c = R^T V_c is the body-frame projection of the world current (Sec. III-B). */
void orc_terms_eval(const orc_env* env, const double q[4], const double nu[6],
                    const double n_lagged[ORC_MAX_THR], orc_terms* out) {
    double R[3][3];
    orc_rotation(q, R);
    const double* v = nu;
    const double* w = nu + 3;
    double gb[3], vc[3], vr[3];
    for (int j = 0; j < 3; ++j) {
        gb[j] = R[2][j];
        vc[j] = R[0][j] * env->current[0] + R[1][j] * env->current[1] + R[2][j] * env->current[2];
        vr[j] = v[j] - vc[j];
    }
    orc_thrust_wrench(env, n_lagged, out->tau);
    orc_fin_wrench(env, n_lagged, vr, w, out->tau);

    double t3[3], Iw[3], A1vr[3], A2w[3], t4[3], Io[3][3], wxr[3], vw[3], t5[3];
    inertia_origin(env, Io);
    cross3(w, env->rg, wxr);
    for (int j = 0; j < 3; ++j) vw[j] = v[j] + wxr[j];
    cross3(w, vw, t3);
    for (int j = 0; j < 3; ++j) Iw[j] = Io[j][0] * w[0] + Io[j][1] * w[1] + Io[j][2] * w[2];
    cross3(w, Iw, t4);
    double wxv[3];
    cross3(w, v, wxv);
    cross3(env->rg, wxv, t5);
    for (int j = 0; j < 3; ++j) {
        out->crb[j] = env->mass * t3[j];
        out->crb[3 + j] = env->mass * t5[j] + t4[j];
    }

    for (int j = 0; j < 3; ++j) {
        A1vr[j] = env->added[j] * vr[j];
        A2w[j] = env->added[3 + j] * w[j];
    }
    double c1[3], c2[3], c3[3];
    cross3(w, A1vr, c1);
    cross3(vr, A1vr, c2);
    cross3(w, A2w, c3);
    for (int j = 0; j < 3; ++j) {
        out->ca[j] = c1[j];
        out->ca[3 + j] = c2[j] + c3[j];
    }

    double nur[6] = {vr[0], vr[1], vr[2], w[0], w[1], w[2]};
    for (int j = 0; j < 6; ++j) out->damp[j] = (env->dlin[j] + env->dquad[j] * fabs(nur[j])) * nur[j];

    double W = env->mass * env->g0;
    double rbxg[3], rgxg[3];
    cross3(env->rb, gb, rbxg);
    cross3(env->rg, gb, rgxg);
    for (int j = 0; j < 3; ++j) {
        out->restore[j] = -(W - env->buoy) * gb[j];
        out->restore[3 + j] = env->buoy * rbxg[j] - W * rgxg[j];
    }

    double wxvc[3];
    cross3(w, vc, wxvc);
    int amc = !(env->flags & ORC_FLAG_NO_AMC);
    for (int j = 0; j < 3; ++j) {
        out->hadd[j] = amc ? env->added[j] * wxvc[j] : 0.0;
        out->hadd[3 + j] = 0.0;
    }

    for (int j = 0; j < 6; ++j)
        out->total[j] = out->tau[j] - out->crb[j] - out->ca[j] - out->damp[j] - out->restore[j] -
                        out->hadd[j];
}

/* d(nu)/dt = M^{-1} F (Eq. (1) solved for the acceleration). */
static void accel(const orc_env* env, const double F[6], double acc[6]) {
    double M[36];
    orc_mass_matrix(env, M);
    solve6(M, F, acc);
}

static void normalise4(double q[4]) {
    double s = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int j = 0; j < 4; ++j) q[j] /= s;
}

/* One step of the discrete map, in the order lag -> thrust -> forces -> acceleration
 * solve -> pose:
 *   n+  = n + alpha (clip(a, -1, 1) - n)
 *   nu+ = nu + dt (M_RB + M_A)^{-1} F(q, nu, n+)     (Eq. (1) solved for d(nu)/dt)
 *   p+  = p + dt R(q) v+
 *   q+  = normalise(q (x) (cos(th/2), sin(th/2) w+/|w+|)),  th = |w+| dt.
 * forces (optional): actuator wrench [6], then the hydrodynamic wrench of Eq. (3),
 * -M_A d(nu_r)/dt - C_A nu_r - D nu_r - g_A, with g_A the buoyancy part of g. */
void orc_step(const orc_env* env, orc_state* s, const double* a, double* forces) {
    double nl[ORC_MAX_THR] = {0};
    for (int i = 0; i < env->m; ++i) {
        double c = a[i] < -1.0 ? -1.0 : (a[i] > 1.0 ? 1.0 : a[i]);
        nl[i] = env->tau[i] > 0.0 ? s->n[i] + orc_lag_factor(env, i) * (c - s->n[i]) : c;
    }
    orc_terms t;
    orc_terms_eval(env, s->q, s->nu, nl, &t);
    double R[3][3];
    orc_rotation(s->q, R);
    double acc[6], nun[6];
    accel(env, t.total, acc);
    for (int j = 0; j < 6; ++j) nun[j] = s->nu[j] + env->dt * acc[j];
    if (forces) {
        double gb[3] = {R[2][0], R[2][1], R[2][2]}, rbxg[3];
        cross3(env->rb, gb, rbxg);
        for (int j = 0; j < 6; ++j) {
            double gA = j < 3 ? env->buoy * gb[j] : env->buoy * rbxg[j - 3];
            forces[j] = t.tau[j];
            forces[6 + j] = -env->added[j] * acc[j] - t.hadd[j] - t.ca[j] - t.damp[j] - gA;
        }
    }
    for (int j = 0; j < 3; ++j)
        s->p[j] += env->dt * (R[j][0] * nun[0] + R[j][1] * nun[1] + R[j][2] * nun[2]);
    double wn = sqrt(nun[3] * nun[3] + nun[4] * nun[4] + nun[5] * nun[5]);
    double dq[4] = {1.0, 0.0, 0.0, 0.0};
    if (wn > 0.0) {
        double half = 0.5 * wn * env->dt;
        double sh = sin(half) / wn;
        dq[0] = cos(half);
        dq[1] = sh * nun[3];
        dq[2] = sh * nun[4];
        dq[3] = sh * nun[5];
    }
    double qn[4];
    orc_quat_mul(s->q, dq, qn);
    normalise4(qn);
    memcpy(s->q, qn, sizeof qn);
    memcpy(s->nu, nun, sizeof nun);
    for (int i = 0; i < env->m; ++i) s->n[i] = nl[i];
}

static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

int32_t orc_rollout(int64_t n_envs, const orc_env* envs, orc_state* states, const double* actions,
                    int64_t n_rows, int32_t hold, int64_t t0, int64_t row0, int32_t n_steps,
                    double* traj, double* forces) {
    int32_t bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t e = 0; e < n_envs; ++e) {
        orc_state* s = &states[e];
        for (int32_t k = 0; k < n_steps; ++k) {
            int64_t row = floor_div(t0 + k, hold) - row0;
            if (row < 0 || row >= n_rows) {
                bad = 1;
                break;
            }
            const double* a = actions + (e * n_rows + row) * ORC_MAX_THR;
            double* f = forces ? forces + (e * n_steps + k) * 12 : 0;
            orc_step(&envs[e], s, a, f);
            if (traj) memcpy(traj + (e * n_steps + k) * ORC_STATE_LEN, s, sizeof(orc_state));
        }
    }
    return bad ? -1 : 0;
}

void orc_rollout_loss(int64_t n_envs, const orc_env* envs, const orc_state* states0,
                      const double* actions, int32_t horizon, const double* waypoints,
                      double act_weight, double* loss_out) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_envs; ++e) {
        orc_state s = states0[e];
        double L = 0.0;
        const double* w = waypoints + 3 * e;
        for (int32_t k = 0; k < horizon; ++k) {
            const double* a = actions + (e * horizon + k) * ORC_MAX_THR;
            orc_step(&envs[e], &s, a, 0);
            double d0 = s.p[0] - w[0], d1 = s.p[1] - w[1], d2 = s.p[2] - w[2];
            double aa = 0.0;
            for (int i = 0; i < envs[e].m; ++i) aa += a[i] * a[i];
            L += d0 * d0 + d1 * d1 + d2 * d2 + act_weight * aa;
        }
        loss_out[e] = L;
    }
}

/* ------------------------------------------------------------------ continuous reference */

static void smooth_action(const double* sp, int m, double t, double* a) {
    for (int i = 0; i < m; ++i) a[i] = sp[i] * sin(2.0 * M_PI * sp[8 + i] * t + sp[16 + i]);
}

/* Time derivative of the continuous model: rotor lag dn/dt = (a - n)/tau, Eq. (1) solved
 * for d(nu)/dt with the thrust of the current rotor state, dp/dt = R v,
 * dq/dt = 1/2 q (x) (0, w). Zero-order rotors follow the command algebraically. */
static void deriv(const orc_env* env, const double* a, const double x[ORC_STATE_LEN],
                  double dx[ORC_STATE_LEN]) {
    orc_state s;
    memcpy(&s, x, sizeof s);
    for (int i = 0; i < ORC_MAX_THR; ++i) dx[13 + i] = 0.0;
    for (int i = 0; i < env->m; ++i) {
        double c = a[i] < -1.0 ? -1.0 : (a[i] > 1.0 ? 1.0 : a[i]);
        if (env->tau[i] > 0.0)
            dx[13 + i] = (c - s.n[i]) / env->tau[i];
        else
            s.n[i] = c;
    }
    orc_terms t;
    orc_terms_eval(env, s.q, s.nu, s.n, &t);
    double R[3][3];
    orc_rotation(s.q, R);
    for (int j = 0; j < 3; ++j) dx[j] = R[j][0] * s.nu[0] + R[j][1] * s.nu[1] + R[j][2] * s.nu[2];
    double om[4] = {0.0, s.nu[3], s.nu[4], s.nu[5]}, qd[4];
    orc_quat_mul(s.q, om, qd);
    for (int j = 0; j < 4; ++j) dx[3 + j] = 0.5 * qd[j];
    accel(env, t.total, dx + 7);
}

void orc_rk4_smooth(int64_t n_envs, const orc_env* envs, orc_state* states,
                    const double* smooth_params, double h, int64_t n_steps) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_envs; ++e) {
        const orc_env* env = &envs[e];
        const double* sp = smooth_params + e * 24;
        double x[ORC_STATE_LEN], k1[ORC_STATE_LEN], k2[ORC_STATE_LEN], k3[ORC_STATE_LEN],
            k4[ORC_STATE_LEN], y[ORC_STATE_LEN], a[ORC_MAX_THR] = {0};
        memcpy(x, &states[e], sizeof x);
        for (int64_t k = 0; k < n_steps; ++k) {
            double t = (double)k * h;
            smooth_action(sp, env->m, t, a);
            deriv(env, a, x, k1);
            for (int j = 0; j < ORC_STATE_LEN; ++j) y[j] = x[j] + 0.5 * h * k1[j];
            smooth_action(sp, env->m, t + 0.5 * h, a);
            deriv(env, a, y, k2);
            for (int j = 0; j < ORC_STATE_LEN; ++j) y[j] = x[j] + 0.5 * h * k2[j];
            deriv(env, a, y, k3);
            for (int j = 0; j < ORC_STATE_LEN; ++j) y[j] = x[j] + h * k3[j];
            smooth_action(sp, env->m, t + h, a);
            deriv(env, a, y, k4);
            for (int j = 0; j < ORC_STATE_LEN; ++j)
                x[j] += h / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
            normalise4(x + 3);
            for (int i = 0; i < env->m; ++i)
                if (env->tau[i] <= 0.0) {
                    smooth_action(sp, env->m, t + h, a);
                    x[13 + i] = a[i];
                }
        }
        memcpy(&states[e], x, sizeof x);
    }
}

void orc_rollout_smooth(int64_t n_envs, const orc_env* envs, orc_state* states,
                        const double* smooth_params, int64_t n_steps) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_envs; ++e) {
        const double* sp = smooth_params + e * 24;
        double a[ORC_MAX_THR] = {0};
        for (int64_t k = 0; k < n_steps; ++k) {
            smooth_action(sp, envs[e].m, (double)k * envs[e].dt, a);
            orc_step(&envs[e], &states[e], a, 0);
        }
    }
}
