/*
 * FP64 CPU oracle for the batched underwater-vehicle step (MarineGym, arXiv 2503.09203,
 * Sec. III-B "GPU-accelerated underwater simulation pipeline", Eqs. (1)-(3), and Sec. III-D
 * "Multi-type UUV model library" for the rotor and thrust models).
 *
 * TEST INFRASTRUCTURE ONLY. Plain, slow, obviously correct: one environment at a time, in
 * double precision, in the order the method states. It shares no code with the device
 * path and must never be linked or called by the product library; only the tests, the
 * smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Conventions: NED world frame, FRD body frame, body origin at the centre of gravity,
 * quaternion (w, x, y, z) Hamilton product, body -> world. Velocity nu = [v; w] =
 * (u, v, w, p, q, r) in the body frame.
 */
#ifndef MGX_ORACLE_H
#define MGX_ORACLE_H
#include <stdint.h>

#define ORC_MAX_THR 8
#define ORC_STATE_LEN 21            /* p[3] q[4] nu[6] n[8] */

#define ORC_FLAG_NO_AMC 1u          /* drop the added-mass term from the rotating current */
#define ORC_FLAG_LAG_EULER 2u       /* rotor lag factor dt/tau instead of the exact hold */

#define ORC_PROPELLER 0
#define ORC_FIN 1

typedef struct {
    int32_t m;                  /* thrusters, 1..8 */
    uint32_t flags;
    double dt, g0;
    double mass;                /* rigid-body mass (kg) */
    double inertia[3];          /* principal moments about the CoG (kg m^2) */
    double added[6];            /* added-mass diagonal, positive */
    double dlin[6], dquad[6];   /* linear and quadratic damping per DOF */
    double buoy;                /* buoyancy force B (N) */
    double rb[3];               /* centre of buoyancy (m, body) */
    double current[3];          /* constant world-frame current (m/s) */
    double r[ORC_MAX_THR][3];   /* thruster positions (body) */
    double e[ORC_MAX_THR][3];   /* thrust directions (normalised here) */
    double k[ORC_MAX_THR];      /* thrust gain */
    double tau[ORC_MAX_THR];    /* rotor time constant; 0 = zero-order model */
    double deadzone[ORC_MAX_THR];
    double k_rev[ORC_MAX_THR];  /* reverse thrust gain (N at n = -1); 0 = same as k */
    double reaction[ORC_MAX_THR]; /* shaft torque per unit thrust about e (m), signed by
                                     the propeller's handedness */
    int32_t kind[ORC_MAX_THR];  /* ORC_PROPELLER or ORC_FIN */
    double span[ORC_MAX_THR][3];  /* fin: hinge (span) axis; e is then the chord at zero
                                     deflection (the component along the span is dropped) */
    double fin_max[ORC_MAX_THR];  /* fin: deflection at n = 1 (rad) */
    double fin_lift[ORC_MAX_THR]; /* fin: K_L = rho A c_L / 2 (kg/m) */
    double fin_drag0[ORC_MAX_THR]; /* fin: K_D0 = rho A c_D0 / 2 (kg/m) */
    double fin_drag[ORC_MAX_THR]; /* fin: K_D = rho A c_D / 2 (kg/m) */
    double rg[3];               /* centre of gravity relative to the body origin (payload);
                                   inertia is given about the centre of gravity */
} orc_env;

typedef struct {
    double p[3], q[4], nu[6], n[ORC_MAX_THR];
} orc_state;

/* Force terms of the equation of motion, each a 6-vector in the body frame. */
typedef struct {
    double tau[6];      /* actuator wrench */
    double crb[6];      /* C_RB(nu) nu */
    double ca[6];       /* C_A(nu_r) nu_r */
    double damp[6];     /* D(nu_r) nu_r */
    double restore[6];  /* g(eta) = g_RB + g_A */
    double hadd[6];     /* added-mass term from the rotating current projection */
    double total[6];    /* tau - crb - ca - damp - restore - hadd */
} orc_terms;

int32_t orc_sizeof_env(void);
int32_t orc_sizeof_state(void);
void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

void orc_rotation(const double q[4], double R[3][3]);
void orc_quat_mul(const double a[4], const double b[4], double out[4]);
double orc_lag_factor(const orc_env* env, int32_t i);
void orc_thrust_wrench(const orc_env* env, const double n[ORC_MAX_THR], double tau[6]);
void orc_fin_wrench(const orc_env* env, const double n[ORC_MAX_THR], const double vr[3], const double w[3],
                    double tau[6]);
void orc_terms_eval(const orc_env* env, const double q[4], const double nu[6],
                    const double n_lagged[ORC_MAX_THR], orc_terms* out);
/* M = M_RB + M_A, 6x6 row-major. */
void orc_mass_matrix(const orc_env* env, double M[36]);

/* One step; a = commanded actions [m]; forces (optional) = actuator wrench[6], hydro wrench[6]. */
void orc_step(const orc_env* env, orc_state* s, const double* a, double* forces);

/* Rollout over n_envs; env e at global step t = t0 + k uses row floor(t/hold) - row0 of
 * actions[e][n_rows][8]. traj (optional) [e][n_steps][21]; forces (optional) [e][n_steps][12].
 * Returns 0, or -1 if a row index falls outside [0, n_rows). */
int32_t orc_rollout(int64_t n_envs, const orc_env* envs, orc_state* states, const double* actions,
                    int64_t n_rows, int32_t hold, int64_t t0, int64_t row0, int32_t n_steps,
                    double* traj, double* forces);

/* Sum over k = 1..H of |p_k - w|^2 + act_weight |a_{k-1}|^2, per-step actions [e][H][8]. */
void orc_rollout_loss(int64_t n_envs, const orc_env* envs, const orc_state* states0,
                      const double* actions, int32_t horizon, const double* waypoints /*[e][3]*/,
                      double act_weight, double* loss_out);

/* Continuous-time reference: RK4 at step h with smooth actions a_i(t) = amp_i sin(2 pi f_i t + ph_i).
 * smooth_params = [e][3][8] (amp, freq, phase). The discrete map counterpart samples a(t_k). */
void orc_rk4_smooth(int64_t n_envs, const orc_env* envs, orc_state* states,
                    const double* smooth_params, double h, int64_t n_steps);
void orc_rollout_smooth(int64_t n_envs, const orc_env* envs, orc_state* states,
                        const double* smooth_params, int64_t n_steps);

#endif
