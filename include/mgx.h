/*
 * mgx — batched underwater-vehicle dynamics on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the device library. It advances thousands of independent vehicles
 * ("environments") by the step of MarineGym's GPU hydrodynamic pipeline (arXiv
 * 2503.09203, Sec. III-B, Eqs. (1)-(3); actuator models of Sec. III-D): rotor lag, thrust
 * through the thruster layout, rigid-body and added-mass Coriolis, linear plus quadratic
 * damping and restoring forces with the relative-velocity current substitution, the
 * (M_RB + M_A)^-1 acceleration solve, and quaternion pose integration.
 *
 * Conventions (all calls):
 *   - Units SI. World frame NED, body frame FRD, body origin at the centre of gravity.
 *     Quaternion (w, x, y, z), Hamilton product, body -> world. nu = (u, v, w, p, q, r).
 *   - Every function returns mgx_status. Nothing throws across the ABI. On failure the
 *     thread-local detail string is available from mgx_last_error().
 *   - Validation failures (MGX_E_INVALID) leave every object unchanged.
 *   - A HIP runtime failure inside a batch call marks the batch faulted; every later call
 *     on it returns MGX_E_STATE until mgx_batch_destroy().
 *   - Device pointers are plain HIP device addresses (e.g. torch tensor data_ptr()); the
 *     library never frees memory it did not allocate. Host inputs are copied before the
 *     call returns.
 *   - Calls are asynchronous on the batch's stream unless stated otherwise. A batch is not
 *     thread-safe; distinct batches may be used from distinct threads.
 *   - Precision: MGX_FP32 batches keep state, parameters and actions in float; MGX_FP64
 *     batches in double. Per-parameter-set setup (mass inverse, lag factors, thruster
 *     layout) always runs in double on the device and is rounded once.
 */
#ifndef MGX_H
#define MGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mgx_status;
#define MGX_OK 0
#define MGX_E_INVALID (-1)   /* bad argument; nothing changed */
#define MGX_E_NOMEM (-2)     /* device or host allocation failed */
#define MGX_E_DEVICE (-3)    /* no usable GPU, or a HIP call failed (see mgx_last_hip_error) */
#define MGX_E_NOT_SPD (-4)   /* M_RB + M_A of some environment is not positive definite */
#define MGX_E_NONFINITE (-5) /* mgx_batch_check: some environment holds a non-finite value */
#define MGX_E_BUDGET (-6)    /* serving: request larger than the memory budget */
#define MGX_E_STATE (-7)     /* batch faulted earlier, or called in the wrong order */

#define MGX_MAX_THRUSTERS 8
#define MGX_MAX_CLASSES 16
#define MGX_STATE_FIXED 13   /* p[3], q[4], nu[6]; then n[m] rotor states */
#define MGX_FORCE_LEN 12     /* actuator wrench[6], hydrodynamic wrench[6] */

/* precision */
#define MGX_FP32 4
#define MGX_FP64 8

/* batch flags */
#define MGX_FLAG_NO_AMC 1u     /* drop the added-mass term from the rotating current projection */
#define MGX_FLAG_LAG_EULER 2u  /* rotor lag factor dt/tau instead of 1 - exp(-dt/tau) */

/* step flags */
#define MGX_STEP_UNFUSED 1u    /* K launches of one step each instead of one launch of K steps */
#define MGX_STEP_STATS 2u      /* update batch statistics at the end of the call */

/* ------------------------------------------------------------------ errors, info */

const char* mgx_status_string(mgx_status s);
/* Copies the calling thread's last error detail into buf (NUL-terminated, truncated to len);
 * returns the full length. buf may be NULL to query the length. */
size_t mgx_last_error(char* buf, size_t len);
/* hipError_t value of the last failed HIP call on this thread (0 if none). */
int32_t mgx_last_hip_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t mgx_version(void);
/* Digest of the sources the library was compiled from (16 hex digits of SHA-256 over the
 * kernel sources and this header, by relative path and content; "unknown" when built
 * without it). A loader compares it with the digest of the sources beside it and refuses a
 * library built from other sources. Static string, never freed. */
const char* mgx_build_hash(void);
/* Number of visible HIP devices (MGX_E_DEVICE if the runtime reports none). */
mgx_status mgx_device_count(int32_t* count);

/* Algorithmic cost of one environment advanced by one step for a class with m thrusters,
 * counted on the host over the same step body the kernels run: flops (add, sub, mul = 1,
 * fused multiply-add = 2) and vector ALU operations (every add/sub/mul/fma/min/max/
 * select = 1; negation and absolute value are free operand modifiers). batch_flags:
 * MGX_FLAG_* plus MGX_COST_SHAPED to count the body of classes with dead zones or
 * reverse gains instead of the plain one. */
#define MGX_COST_SHAPED 0x80000000u
mgx_status mgx_step_cost(int32_t m, uint32_t batch_flags, double* flops, double* valu_ops);
/* The same count for the reverse sweep of a differentiable rollout: one environment-step
 * of the hand-written vector-Jacobian product (mgx_rollout_backward) given the step's
 * forward quantities, which the backward's recomputation of the step stores as it runs
 * (that recomputation is counted by mgx_step_cost). */
mgx_status mgx_vjp_cost(int32_t m, uint32_t batch_flags, double* flops, double* valu_ops);

/* Diagnostics: the per-wave phase times of the last step launch, four 100 MHz real-time
 * counter values per wave (entry, prologue loads landed, steps done, stores drained), wave
 * w of the launch at out[4 w .. 4 w + 3]; synchronises the device. Only a library compiled
 * with MGX_WAVE_TIMESTAMPS records them (the recording changes the kernels); any other
 * build returns MGX_E_STATE. */
mgx_status mgx_diag_wave_times(uint64_t* out, int64_t n_waves);
/* Diagnostics: the VALU issue rate. Every thread runs `chains` (1, 2, 4 or 8) independent
 * float multiply-add chains of 16 * iters links; n_threads (a multiple of 256) threads in
 * blocks of 256; *seconds = the best of three timed launches (HIP events, null stream;
 * allocates its own output). */
mgx_status mgx_diag_valu_probe(int32_t chains, int64_t n_threads, int32_t iters, double* seconds);
/* Diagnostics: the time per launch of `launches` back-to-back launches of a kernel that
 * does nothing, n_threads threads in blocks of `block` (the fixed cost every launch pays);
 * best of three timed batches. */
mgx_status mgx_diag_launch_floor(int64_t n_threads, int32_t block, int32_t launches, double* seconds);

/* ------------------------------------------------------------------ vehicle classes */

/* One vehicle class: the thruster layout and rotor models (Sec. III-D), principal
 * inertia about the centre of gravity, centre of buoyancy. Host memory, copied.
 * Thruster i with rotor state n_i (after the lag) pushes f_i = k_i s|s| when s >= 0 and
 * k_rev_i s|s| when s < 0, s = sgn(n_i) max(|n_i| - deadzone_i, 0), along e_i at r_i, and
 * turns the hull about e_i with the shaft torque reaction_i f_i: the wrench about the CoG
 * is f_i [e_i ; r_i x e_i + reaction_i e_i]. Zero-filled trailing fields keep the plain
 * symmetric propeller with no shaft torque. */
typedef struct {
    int32_t m;                          /* thrusters, 1..MGX_MAX_THRUSTERS */
    int32_t reserved;
    double r[MGX_MAX_THRUSTERS][3];     /* thruster positions, body frame (m) */
    double e[MGX_MAX_THRUSTERS][3];     /* thrust axes, body frame; normalised by the library */
    double k[MGX_MAX_THRUSTERS];        /* thrust gain (N at |n| = 1), > 0 */
    double tau[MGX_MAX_THRUSTERS];      /* rotor time constant (s), >= 0; 0 = zero-order rotor */
    double deadzone[MGX_MAX_THRUSTERS]; /* dead zone on |n|, in [0, 1) */
    double inertia[3];                  /* principal moments about the CoG (kg m^2), > 0 */
    double rb[3];                       /* centre of buoyancy, body frame (m) */
    double g0;                          /* gravitational acceleration (m/s^2), > 0 */
    double k_rev[MGX_MAX_THRUSTERS];    /* reverse thrust gain (N at n = -1), >= 0; 0 = k */
    double reaction[MGX_MAX_THRUSTERS]; /* shaft torque per unit thrust about e (m), signed
                                           by the propeller's handedness; finite */
    /* Rudders (Sec. III-D: lift and drag depending on the flow speed, the fin area and
     * coefficients that vary with the angle of attack). An actuator of kind MGX_ACT_FIN at
     * r moves through the water at u = v_r + w x r. Its plane is normal to span; e is the
     * chord at zero deflection (its span component is dropped) and nn = span x chord. The
     * lagged state n sets the deflection fin_max * n toward nn; the angle of attack a is
     * the deflection minus the angle of the in-plane flow u_p from the chord. Lift
     * fin_lift sin(a)cos(a)|u_p|^2 acts along span x u_p / |u_p|, drag
     * (fin_drag0 + fin_drag sin^2(a))|u_p|^2 against u_p, both at r. k, k_rev, reaction
     * and deadzone are not used for fins. */
    int32_t kind[MGX_MAX_THRUSTERS];    /* MGX_ACT_PROPELLER (0) or MGX_ACT_FIN (1) */
    double span[MGX_MAX_THRUSTERS][3];  /* fin hinge axis, not parallel to e */
    double fin_max[MGX_MAX_THRUSTERS];  /* deflection at n = 1 (rad), in (0, pi/2] */
    double fin_lift[MGX_MAX_THRUSTERS]; /* rho A c_L / 2 (kg/m), >= 0 */
    double fin_drag0[MGX_MAX_THRUSTERS]; /* rho A c_D0 / 2 (kg/m), >= 0 */
    double fin_drag[MGX_MAX_THRUSTERS]; /* rho A c_D / 2 (kg/m), >= 0 */
    /* Payload (Table II's external loads): the centre of gravity at rg from the body origin
     * (where positions, added mass, damping and the centre of buoyancy are given); inertia
     * stays given about the centre of gravity. Non-zero rg makes M_RB full,
     * [m 1, -m S(rg); m S(rg), I_g + m(|rg|^2 1 - rg rg^T)], adds the matching Coriolis terms
     * m w x (w x rg) and m rg x (w x v), and the weight's moment -W rg x g_b; dt M^-1 is then
     * inverted in double per environment (Cholesky). Such classes run per-class launches;
     * the server and the adjoint refuse them. |rg_j| < 10 m. */
    double rg[3];
} mgx_class_desc;

#define MGX_ACT_PROPELLER 0
#define MGX_ACT_FIN 1

/* Registers a class; *class_id receives its id (process-wide, never reused).
 * MGX_E_INVALID on a non-finite or out-of-range field, a zero-length thrust axis, or when
 * 4096 classes are already defined. */
mgx_status mgx_class_define(const mgx_class_desc* desc, int32_t* class_id);

/* Algorithmic cost of one environment-step of a defined class, counted like mgx_step_cost
 * over the body its batches run (plain, shaped thrust, or with fins). */
mgx_status mgx_class_step_cost(int32_t class_id, uint32_t batch_flags, double* flops, double* valu_ops);

/* ------------------------------------------------------------------ batches */

typedef struct mgx_batch mgx_batch;

/* Device allocator of a batch: alloc returns `bytes` of device memory on the batch's
 * device (NULL on failure, which the calling function reports as MGX_E_NOMEM); free
 * releases what alloc returned. Called only from inside library calls on the batch. */
typedef void* (*mgx_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mgx_free_fn)(void* ptr, void* ctx);

typedef struct {
    int32_t n_classes;          /* 1..MGX_MAX_CLASSES */
    int32_t precision;          /* MGX_FP32 or MGX_FP64 */
    const int32_t* class_ids;   /* [n_classes] from mgx_class_define (host) */
    const int64_t* n_envs;      /* [n_classes] environments per class, >= 1 (host) */
    double dt;                  /* step (s), > 0 */
    uint32_t flags;             /* MGX_FLAG_* */
    int32_t device;             /* HIP device ordinal; -1 = the calling thread's current device */
    void* stream;               /* hipStream_t for every call on the batch; NULL = null stream */
    /* Optional caller-owned device buffers (e.g. torch tensors), adopted: the batch works
     * in them in place and never frees them, so they must outlive it. Sizes and layout from
     * mgx_batch_plan (state_elems, record_elems elements of the batch precision). NULL: the
     * library allocates. At creation an adopted state keeps its valid slots as they are and
     * only its padded slots are set to rest. */
    void* state;
    void* record;
    /* Optional allocator for every device buffer the library allocates for this batch
     * (state and record unless adopted, bookkeeping, rollout checkpoints, autotuner
     * snapshots); both or neither. NULL: hipMalloc / hipFree. */
    mgx_alloc_fn alloc;
    mgx_free_fn free;
    void* alloc_ctx;
} mgx_batch_desc;

/* Memory layout of a batch. Environments are numbered globally 0..n_total-1, class by
 * class in the order given at creation. Each class segment is padded to a multiple of 64
 * environments (one wavefront); padded slots hold a benign state and are never reported.
 *   state   : class c at state_off[c], component-major: element (j, env) at
 *             state_off[c] + j * n_pad[c] + env, j < 13 + m[c]. Total state_elems.
 *   actions : one row per hold interval, row_elems elements per row; class c at
 *             action_off[c] within a row, element (i, env) at action_off[c] + i*n_pad[c] + env.
 *   forces  : per step, force_row_elems per row; class c at force_off[c], element (j, env)
 *             at force_off[c] + j * n_pad[c] + env, j < 12.
 * Element size is the batch precision (4 or 8 bytes). */
typedef struct {
    int32_t n_classes, precision;
    int64_t n_total, n_pad_total;
    int64_t state_elems, row_elems, force_row_elems;
    int32_t m[MGX_MAX_CLASSES];
    int64_t n[MGX_MAX_CLASSES], n_pad[MGX_MAX_CLASSES];
    int64_t env_off[MGX_MAX_CLASSES];     /* first global env id of the class */
    int64_t state_off[MGX_MAX_CLASSES], action_off[MGX_MAX_CLASSES], force_off[MGX_MAX_CLASSES];
    int64_t record_elems;                 /* parameter record: record_off[c] + row * n_pad[c] + env */
    int64_t record_off[MGX_MAX_CLASSES];
} mgx_layout;

/* The layout a batch created from desc would have (sizes of the state and record buffers a
 * caller may pass in desc->state / desc->record). Host only, no device needed.
 * MGX_E_INVALID on bad fields. */
mgx_status mgx_batch_plan(const mgx_batch_desc* desc, mgx_layout* out);

/* A batch of environments, each the vehicle model of Sec. III-B (Eqs. (1)-(3)) with the
 * actuators of Sec. III-D, sharing the class constants of its segment. Creates it on the
 * given device and stream and allocates its state, parameter record (unless adopted) and
 * bookkeeping. Synchronous. The step counter starts at 0. MGX_E_INVALID on bad fields;
 * MGX_E_DEVICE if no GPU is usable; MGX_E_NOMEM (also when a caller's allocator fails). */
mgx_status mgx_batch_create(const mgx_batch_desc* desc, mgx_batch** out);
mgx_status mgx_batch_destroy(mgx_batch* b);   /* synchronises its stream, frees; NULL is OK */
mgx_status mgx_batch_layout(const mgx_batch* b, mgx_layout* out);

/* Per-environment parameters, each an array over the global env id (n_total entries per
 * row), always double precision. Rows of 6 are DOF-major: element (j, env) at j*n_total+env.
 *   mass  [n]   rigid-body mass (kg), > 0
 *   added [6][n] added-mass diagonal (Fossen's -X_udot, ...; usually positive), finite, with
 *               M_RB + M_A positive definite
 *   dlin  [6][n] linear damping, >= 0;  dquad [6][n] quadratic damping, >= 0
 *   buoy  [n]   buoyancy force (N), >= 0
 *   current [3][n] constant world-frame water velocity (m/s)  (Sec. III-B, ocean currents) */
typedef struct {
    const double* mass;
    const double* added;
    const double* dlin;
    const double* dquad;
    const double* buoy;
    const double* current;
} mgx_env_params;

/* Per-parameter-set setup (Eq. (1)-(2): M = M_RB + M_A with M_RB = diag(m, m, m, I)):
 * computes dt*M^-1, W - B, lag factors and the thruster layout in double precision on the
 * device, rounds once to the batch precision. on_device = 1: the arrays are device
 * pointers; 0: host pointers (copied before the call returns). Every environment's values
 * are checked on the device before any record is written, and the call waits for that
 * check: MGX_E_INVALID for a non-finite or out-of-range value (ranges above), MGX_E_NOT_SPD
 * when some M_RB + M_A is not positive definite (a diagonal entry <= 0, or a Cholesky
 * pivot <= 0 with a payload); the batch is then unchanged. The record build itself stays
 * asynchronous. on_device = 2: device pointers taken without the prior check, nothing
 * waited for (for loops that rebuild known-good parameters); an invalid environment then
 * gets a NaN record and sets the batch's error word (mgx_batch_check). Must be called
 * before the first step (MGX_E_STATE otherwise). */
mgx_status mgx_batch_set_params(mgx_batch* b, const mgx_env_params* p, int32_t on_device);

/* ------------------------------------------------------------------ domain randomisation */

/* Sec. III-C: each parameter group of the per-environment record is drawn from a uniform,
 * a Gaussian or a custom piecewise distribution, for the environments chosen, and the
 * distributions may change between calls (curriculum). */
#define MGX_DR_FIXED 0      /* the class nominal itself */
#define MGX_DR_UNIFORM 1    /* lo + (hi - lo) u */
#define MGX_DR_GAUSSIAN 2   /* mean + std z (Box-Muller), clipped to [lo, hi] */
#define MGX_DR_PIECEWISE 3  /* piecewise-constant density over n_bins bins */
#define MGX_DR_MAX_BINS 8

typedef struct {
    int32_t kind;                       /* MGX_DR_* */
    int32_t relative;                   /* 1: the draw multiplies the class nominal; 0: it is the value */
    int32_t shared;                     /* vector groups: 1 = one draw for every entry */
    int32_t n_bins;                     /* piecewise: 1..MGX_DR_MAX_BINS */
    double lo, hi;                      /* uniform range; Gaussian clip range; lo <= hi */
    double mean, std;                   /* Gaussian; std >= 0 */
    double edges[MGX_DR_MAX_BINS + 1];  /* piecewise: n_bins + 1 increasing edges */
    double weights[MGX_DR_MAX_BINS];    /* piecewise: weights >= 0 with a positive sum */
} mgx_dr_dist;

typedef struct {
    mgx_dr_dist mass, added, dlin, dquad, buoy, current;
} mgx_dr_spec;

/* Redraws the parameters of environments (env_ids: host array of n global ids, or NULL
 * for all) and rebuilds their records exactly as mgx_batch_set_params would from the
 * drawn values. nominal: host, 23 doubles per class (mass, added[6], dlin[6], dquad[6],
 * buoyancy, current[3]). Draws: Philox4x32-10 with key (seed mod 2^32, 7 << 24) and
 * counter (global env id, epoch mod 2^32, j, 0), j = 0..22, two 53-bit uniforms per call;
 * uniform pairs per group: mass 0-1, added entry i 2+2i, linear damping 14+2i, quadratic
 * 26+2i, buoyancy 38, current axis a 40+2a (a shared group uses its first pair); Gaussian
 * from the pair by Box-Muller with the cosine branch; piecewise by inverting the running
 * weight sums. Every value a spec can produce must be a valid parameter (mass > 0, the
 * others >= 0, current any): MGX_E_INVALID otherwise, and on a bad spec, nominal or id.
 * Without a prior mgx_batch_set_params, env_ids must be NULL. Asynchronous on the batch
 * stream (the id upload is synchronous). */
mgx_status mgx_batch_resample(mgx_batch* b, const mgx_dr_spec* spec, const double* nominal, const int64_t* env_ids,
                              int64_t n, uint64_t seed, uint64_t epoch);

/* Reads every environment's parameters back from its record (host arrays laid out as in
 * mgx_env_params, n_total entries per row; values as rounded to the batch precision).
 * Synchronous. */
mgx_status mgx_batch_get_params(const mgx_batch* b, double* mass, double* added, double* dlin, double* dquad,
                                double* buoy, double* current);

/* Resets environments (an episode start, Sec. III-C: environments restart independently).
 * env_ids: host array of n global env ids, or NULL for all.
 * init_state: device pointer to a full state buffer in this batch's layout and precision;
 * the listed environments are copied from it. NULL: seeded state — p = 0, q uniform on
 * the unit 3-sphere (normalised Gaussian), nu ~ N(0, 0.2^2) per component, n = 0 — drawn
 * with Philox4x32-10 keyed by seed, for global env id e (see mgx_gen_actions for the
 * generator). MGX_E_INVALID on an id outside [0, n_total). Does not move the step counter. */
mgx_status mgx_batch_reset(mgx_batch* b, const int64_t* env_ids, int64_t n, const void* init_state,
                           uint64_t seed);

/* The step of Sec. III-B (Eqs. (1)-(3)) with the rotor and thrust models of Sec. III-D:
 * advances every environment by K >= 1 steps of dt (K = 0: the launch-shape K), fused in
 * one launch (MGX_STEP_UNFUSED: K launches of one step). Step k of the call (global step
 * t = t0 + k, t0 = the batch step counter) uses row floor(t / hold) - row0 of `actions`
 * (device pointer, n_rows rows in the layout above, batch precision). Commands are
 * clipped to [-1, 1]. MGX_E_INVALID if a needed row falls outside [0, n_rows).
 * traj: NULL or device [K][state_elems] — the state after each step.
 * forces: NULL or device [K][force_row_elems] — actuator and hydrodynamic wrench (Eq. (3),
 *         with d(nu)/dt the solved acceleration) of each step, body frame.
 * flags: MGX_STEP_*. Asynchronous. The step counter advances by K on the device. */
mgx_status mgx_batch_step(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                          int32_t K, uint32_t flags, void* traj, void* forces);

/* Step counter (host mirror, equal to the device counter once the stream has drained). */
mgx_status mgx_batch_get_step(const mgx_batch* b, int64_t* t);
mgx_status mgx_batch_set_step(mgx_batch* b, int64_t t);

/* Diagnostics: sets the batch's device step counter to t (t >= 0) on its stream without the
 * host's step count, which mgx_batch_get_step keeps returning. Step launches are enqueued
 * with the host's count as the step they expect to start at; after this call they find
 * the counter different, take the action rows the counter names and run their steps again
 * (the results are those of steps from t). For tests of that check; every other entry
 * point keeps the two counts equal. */
mgx_status mgx_diag_set_device_step(mgx_batch* b, int64_t t);

/* The vehicle state of Sec. III-B (position, attitude, body velocity nu) and the rotor
 * states of Sec. III-D. Copies the whole state (state_elems elements) out / in. to_host/from_host = 1: host
 * memory, and the call synchronises the stream; 0: device memory, asynchronous. */
mgx_status mgx_batch_get_state(mgx_batch* b, void* out, int32_t to_host);
mgx_status mgx_batch_set_state(mgx_batch* b, const void* in, int32_t from_host);

/* Batch statistics of the last call that passed MGX_STEP_STATS (synchronises the stream):
 * per class, over its valid environments, wavefront-reduced on the device. mean_kinetic is
 * the kinetic energy of Eq. (1)'s mass matrix M_RB + M_A (the full one with a payload). */
typedef struct {
    int64_t step;                                  /* step counter at that call's end */
    int64_t n_nonfinite[MGX_MAX_CLASSES];          /* envs with any non-finite state value */
    int64_t n_renorm64[MGX_MAX_CLASSES];           /* double-precision attitude renormalisations */
    double max_speed[MGX_MAX_CLASSES], mean_speed[MGX_MAX_CLASSES];   /* |v| (m/s) */
    double max_rate[MGX_MAX_CLASSES], mean_rate[MGX_MAX_CLASSES];     /* |w| (rad/s) */
    double mean_kinetic[MGX_MAX_CLASSES];          /* 1/2 nu^T (M_RB + M_A) nu (J) */
    double max_qdrift[MGX_MAX_CLASSES];            /* max | |q|^2 - 1 | before renormalising */
} mgx_stats;
mgx_status mgx_batch_get_stats(mgx_batch* b, mgx_stats* out);

/* Synchronises the stream and reports the device-side error word and non-finite count
 * (of the last MGX_STEP_STATS call). In order of precedence: MGX_E_NOT_SPD if a parameter
 * record (mgx_batch_resample, mgx_station_resample) was built from a mass matrix that is
 * not positive definite; MGX_E_INVALID if a record was built from an invalid value or a
 * kernel met an action row outside its buffer (both sticky until destroy); MGX_E_NONFINITE
 * (count in *n_nonfinite); MGX_OK. An invalid record holds NaN in its dt M^-1 rows, so its
 * environment also turns non-finite at its next step. */
mgx_status mgx_batch_check(mgx_batch* b, int64_t* n_nonfinite);
mgx_status mgx_batch_sync(mgx_batch* b);

/* Action stream generator on the device (the synthetic command streams of the benchmark
 * workloads; the paper's policies are not part of this library): fills `out` (device, rows x row_elems, batch
 * precision) with a = ((w >> 8) - 2^23) * 2^-23 in [-1, 1), where w is word (i mod 4) of
 * Philox4x32-10 (Salmon et al., SC'11) at key (seed mod 2^32, 4 << 24) and counter
 * (global env id, row_offset + row, i / 4, 0). Padded slots get 0. Asynchronous. */
mgx_status mgx_gen_actions(mgx_batch* b, void* out, int64_t rows, int64_t row_offset, uint64_t seed);

/* ------------------------------------------------------------------ launch shape, autotuner */

#define MGX_LAUNCH_PER_CLASS 0   /* one launch per class segment */
#define MGX_LAUNCH_PERSISTENT 1  /* one launch for all classes: per-class constants staged in
                                    LDS, waves pull 64-environment tiles from a device work
                                    counter (FP32 batches; steps without traj/forces; batches
                                    with a fin class keep per-class launches) */

typedef struct {
    int32_t mode;         /* MGX_LAUNCH_* */
    int32_t K;            /* steps per launch used when a call passes K = 0 */
    int32_t block;        /* threads per block (64, 128 or 256) */
    int32_t grid_per_cu;  /* persistent mode: blocks per compute unit */
    double us_per_chunk;  /* autotuner: measured time of one chunk with this shape */
    int32_t candidates;   /* autotuner: shapes measured */
    int32_t from_cache;   /* autotuner: 1 if taken from the cache without measuring */
} mgx_launch_shape;

/* Reads / sets the launch shape of a batch (validated; MGX_LAUNCH_PERSISTENT on a double
 * batch is MGX_E_INVALID). Default: per-class launches, K = 16, block 64 while the batch
 * has fewer 64-environment tiles than four per compute unit (a small batch then spreads
 * over as many compute units), else 256. */
mgx_status mgx_batch_get_shape(const mgx_batch* b, mgx_launch_shape* out);
mgx_status mgx_batch_set_shape(mgx_batch* b, const mgx_launch_shape* in);

/* Autotuner: times one chunk of chunk_steps steps (from the batch's current step, action
 * rows as in mgx_batch_step) for every candidate shape — launch mode, steps per launch K
 * dividing chunk_steps, block size, persistent grid — with HIP events on the batch stream,
 * keeps the fastest, and records it in a process-wide cache keyed by (GPU architecture,
 * precision, per-class thruster counts and padded sizes, hold, chunk_steps). A cache hit
 * applies the stored shape without measuring. The batch's state and step counter are
 * restored afterwards (synchronous). */
mgx_status mgx_autotune(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                        int32_t chunk_steps, mgx_launch_shape* out);
/* Cache persistence as plain text, one shape per line. */
mgx_status mgx_autotune_save(const char* path);
mgx_status mgx_autotune_load(const char* path);

/* ------------------------------------------------------------------ differentiable rollout */

/* Differentiable rollout of the step map of Sec. III-B (the paper trains model-free and
 * differentiates nothing; this reverse mode is an addition of the library, for losses over
 * positions and commands). Forward pass: H steps exactly as mgx_batch_step (same action
 * indexing, clip, launch per class; MGX_E_INVALID for a batch with a fin class, whose
 * adjoint is not written), additionally writing the position after every step
 * and the full state every ckpt_every steps into library-owned scratch (allocated on first
 * use, kept until destroy). pos_out: device [H][3 * n_pad_total], class c at
 * 3 * (sum of n_pad of the classes before c), element (j, env) at that offset + j * n_pad[c]
 * + env. The batch advances by H. The actions buffer must stay valid until the matching
 * mgx_rollout_backward. */
mgx_status mgx_rollout_forward(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                               int32_t H, int32_t ckpt_every, void* pos_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): mgx_rollout_forward with the
 * checkpoints and the segment scratch placed in a library-static device array of 64 MiB per
 * GPU instead of batch buffers allocated on first use; no allocation of any kind. Same
 * arguments, results and step-counter movement as mgx_rollout_forward, followed by the same
 * mgx_rollout_backward. MGX_E_INVALID (nothing launched) when the checkpoints
 * (P * ceil(H / ckpt_every) * state_elems bytes), the segment scratch
 * (P * 2 * ckpt_every * state_elems bytes), each rounded up to 256, and the segment tape
 * (P * 2 * ckpt_every * 36 * n_pad_total bytes) exceed 64 MiB; P is the element size. The array
 * is shared by every call on the GPU and keeps the last call's contents: a later
 * mgx_rollout_forward_static on any batch of the same GPU overwrites the checkpoints of an
 * earlier one, whose mgx_rollout_backward then returns MGX_E_STATE; calls that overlap on
 * one GPU (other threads, other streams) race. */
mgx_status mgx_rollout_forward_static(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                                      int32_t H, int32_t ckpt_every, void* pos_out);

/* Reverse-mode sweep of the last forward pass (vector-Jacobian product of the step map,
 * written out by hand): each environment recomputes every ckpt_every-step segment from its
 * checkpoint into scratch, then runs the adjoint backwards through it. Given
 * dpos = dL/d(position after step k) (device, pos_out layout), writes
 *   dactions: device [n_rows][row_elems] — dL/d(command) per action row (sum over the
 *             steps of the row; zero outside the clip range); rows the rollout did not
 *             use are left untouched;
 *   dparams : device [18 * n_pad_total] — per class at 18 * (padded offset), rows
 *             0-5 dL/d(d_L), 6-11 dL/d(d_Q), 12-17 dL/d(M_A diagonal) (through the
 *             Coriolis, current and mass-inverse terms).
 * Either output may be NULL. MGX_E_STATE if no forward pass is recorded. Asynchronous. */
mgx_status mgx_rollout_backward(mgx_batch* b, const void* dpos, void* dactions, void* dparams);

/* Diagnostic (host only, double precision): evaluates the kernels' step body and its
 * hand-written adjoint for one environment, so the adjoint can be checked against finite
 * differences without a GPU. cls: Bk[6][8] (layout columns times gains), alpha[8],
 * deadzone[8], inertia[3], rb[3], g0, dt, reverse-to-forward gain ratios[8] (82 doubles);
 * rec: the 30 record fields (dt M^-1[6],
 * m, M_A[6], d_L[6], d_Q[6], W - B, B, V_c[3]); state/xbar_in/state_out/xbar_out: 13 + m;
 * actions/abar_out: m; gparams_out: 24 = adjoints of d_L[6], d_Q[6], M_A[6] (direct
 * terms only), dt M^-1[6]. Used by no device path. */
mgx_status mgx_host_step_vjp(int32_t m, uint32_t batch_flags, const double* cls, const double* rec, const double* state,
                             const double* actions, const double* xbar_in, double* state_out, double* xbar_out,
                             double* abar_out, double* gparams_out);

/* ------------------------------------------------------------------ captured chunks */

typedef struct mgx_graph mgx_graph;

/* Captures a rollout chunk into a HIP graph: ceil(n_steps / K) step launches of K steps
 * (the last one shorter), exactly as mgx_batch_step would enqueue them for the same
 * arguments (MGX_STEP_UNFUSED: one step per launch; MGX_STEP_STATS: statistics on the last
 * launch). Capture happens on a private stream; nothing runs and the batch is unchanged.
 * Each replay runs on the batch's stream and advances the batch by n_steps. Because every
 * launch reads its step from the device counter, one graph walks through a rollout-long
 * action buffer: replay r uses rows floor(t/hold) - row0 for t from the batch's step at
 * replay time. Destroy graphs before their batch (mgx_batch_destroy returns MGX_E_STATE
 * while any is alive). */
mgx_status mgx_graph_capture(mgx_batch* b, const void* actions, int64_t n_rows, int64_t row0, int32_t hold,
                             int32_t n_steps, int32_t K, uint32_t flags, mgx_graph** out);
/* MGX_E_INVALID (nothing launched) if the rows needed at the batch's current step fall
 * outside [0, n_rows). Asynchronous. A replay from the step the graph was captured at is the
 * fastest for graphs of one-step launches: those launches then fetch their action rows
 * beside the state instead of after reading the device counter (the graph holds both forms
 * and the replay picks one; the results are the same). */
mgx_status mgx_graph_replay(mgx_graph* g);
mgx_status mgx_graph_destroy(mgx_graph* g);

/* ------------------------------------------------------------------ station-keeping task */

/* Station keeping (Sec. IV-B): each environment must reach and hold a target pose in
 * moving water, keeping its position error small and its attitude within limits. The task
 * runs on a batch's environments and state: every task step advances them under one held
 * command, then forms the observation, reward and termination in the same kernel, and an
 * environment whose episode ended starts the next one at once. The paper does not give the
 * observation, reward or termination; this library fixes the following.
 *   Episode start of global env g, episode k (seed from mgx_station_reset): 14 uniforms on
 *   [0, 1) of 53 bits from Philox4x32-10 at key (seed mod 2^32, 8 << 24) and counter
 *   (g, k, j, 0), j = 0..6, pairs (w0, w1) then (w2, w3) as in mgx_batch_resample. Target
 *   p* = target_box (2 u[0..2] - 1); target attitude a pure yaw pi (2 u3 - 1). Start at
 *   p = 0 with yaw pi (2 u4 - 1), roll tilt0 (2 u5 - 1), pitch tilt0 (2 u6 - 1),
 *   q0 = q_z(yaw) q_y(pitch) q_x(roll), nu_j = v0 (2 u[7+j] - 1), rotor states 0; in
 *   double, rounded once.
 *   Observation, in the state's layout (13 + m rows): the target position in the body frame
 *   R(q)^T (p* - p); the attitude error q*^-1 q with its scalar part >= 0; nu; the rotor
 *   states.
 *   Reward of a transition, on the state it ends in (a = the clipped command):
 *   exp(-|p* - p| / sigma_p) - w_att (1 - q_e,w^2) - w_act mean_i a_i^2; 0 if that state
 *   is not finite.
 *   terminated: not finite, or |p* - p| > d_max, or the body z axis leans more than
 *   tilt_max from the world z axis. truncated: the episode has taken max_steps task steps.
 *   An episode that ends restarts as episode k + 1 in the same step: obs is then the new
 *   episode's first observation; final_obs holds the observation of the state the
 *   transition ended in, for the environments whose episode ended. */
typedef struct mgx_station mgx_station;

typedef struct {
    double target_box;   /* half-width of the target position box (m), [0, 1e4] */
    double tilt0;        /* start roll and pitch half-range (rad), [0, pi/2] */
    double v0;           /* start velocity half-range per component, [0, 100] */
    double sigma_p;      /* reward position scale (m), > 0 */
    double w_att;        /* attitude penalty weight, >= 0 */
    double w_act;        /* command penalty weight, >= 0 */
    double d_max;        /* terminate beyond this distance from the target (m), > 0 */
    double tilt_max;     /* terminate beyond this lean from upright (rad), (0, pi] */
    int32_t max_steps;   /* truncate after this many task steps, >= 1 */
    int32_t substeps;    /* dynamics steps per task step with the command held, [1, 1000] */
} mgx_station_desc;

/* Creates the task on a batch (device buffers for the targets and episode counters,
 * hipMalloc; synchronous). The batch outlives it: mgx_batch_destroy returns MGX_E_STATE
 * while a task is alive. MGX_E_INVALID on a field outside its range. */
mgx_status mgx_station_create(mgx_batch* b, const mgx_station_desc* d, mgx_station** out);
mgx_status mgx_station_destroy(mgx_station* s);   /* synchronises the batch's stream; NULL is OK */

/* Starts episode 0 of every environment from `seed`: overwrites the batch state, draws the
 * targets, zeroes the episode counters. obs: NULL or device [state_elems] (batch layout and
 * precision), the first observations. Does not move the batch step counter. Asynchronous. */
mgx_status mgx_station_reset(mgx_station* s, uint64_t seed, void* obs);

/* n_steps >= 1 task steps in one launch per class, the state held in registers between
 * them (a Gym step is n_steps = 1). Step k
 * reads command row k of `actions` (device, n_steps rows of row_elems, the batch's action
 * layout and precision) and writes row k of every output, all device memory:
 *   obs, final_obs: [n_steps][state_elems], the batch's state layout (final_obs may be NULL;
 *   only the entries of environments whose episode ended at that step are written);
 *   reward: [n_steps][n_pad_total], batch precision; terminated, truncated:
 *   [n_steps][n_pad_total] bytes (0 / 1). Environment e of class c sits at slot
 *   sum_{c' < c} n_pad[c'] + e; padded slots get reward 0 and flags 0.
 * Does not move the batch step counter. MGX_E_STATE before mgx_batch_set_params or
 * mgx_station_reset. Asynchronous. */
mgx_status mgx_station_step(mgx_station* s, const void* actions, int32_t n_steps, void* obs, void* reward,
                            uint8_t* terminated, uint8_t* truncated, void* final_obs);

/* Episode index and steps taken in the current episode, per global env id (host arrays of
 * n_total). Synchronises the stream. */
mgx_status mgx_station_episodes(mgx_station* s, int32_t* episode, int32_t* steps);

/* Domain randomisation at episode start (Sec. III-C: parameters resampled for the
 * environments that reset): redraws, on the device, the parameters of every environment
 * whose episode started in the last mgx_station_reset or mgx_station_step call, exactly as
 * mgx_batch_resample(spec, nominal, those ids, seed, epoch) would with epoch = the
 * environment's current episode index, so each episode's parameters are a function of
 * (seed, env id, episode). Call it between task calls; an episode that starts and ends
 * within one call of several steps runs with the parameters it started with. spec and
 * nominal as for mgx_batch_resample (host memory). MGX_E_STATE before mgx_station_reset or
 * before the batch has parameters. Asynchronous. */
mgx_status mgx_station_resample(mgx_station* s, const mgx_dr_spec* spec, const double* nominal, uint64_t seed);

/* ------------------------------------------------------------------ serving */

/* Continuous-batching server. A scheduler thread owns a device arena of budget_bytes
 * (one hipMalloc at creation) from which every session's state and parameter record are
 * carved; requests are admitted first-fit in arrival order as memory frees up. Each
 * scheduling iteration takes every admitted request that has steps left, advances it by
 * up to chunk_steps steps (0: all remaining steps) in ONE persistent launch whose tiles
 * carry their own step counts, and runs on the next free stream of a small pool, so that
 * requests arriving while others run are launched at once and their work overlaps on the
 * device; chunks of one request are ordered with events. Actions are generated inside the
 * kernel from each session's seed with the generator of mgx_gen_actions (env id local to
 * the session, row floor(t / hold) with t counted from the session's first step), unless a
 * request brings its own command rows (mgx_request.actions). A session's state stays
 * resident between its requests. Results are bitwise the same
 * whatever else runs. */

typedef struct mgx_server mgx_server;

#define MGX_SERVE_FIFO 1u  /* one request at a time, its whole horizon in one launch, one stream (baseline) */

typedef struct {
    int32_t n_classes;
    const int32_t* class_ids;   /* [n_classes] from mgx_class_define */
    const double* nominal;      /* [n_classes][23]: mass, added[6], dlin[6], dquad[6], buoy, current[3] */
    double dt;
    uint32_t batch_flags;       /* MGX_FLAG_* */
    uint32_t serve_flags;       /* MGX_SERVE_* */
    int64_t budget_bytes;       /* device memory for session state + records */
    int32_t chunk_steps;        /* steps per iteration and request (0: all remaining) */
    int32_t max_active;         /* requests admitted at once (>= 1) */
    int32_t device;             /* -1: current device */
    int32_t streams;            /* concurrent iterations (0: 4; 1..16) */
} mgx_server_desc;

typedef struct {
    int32_t class_index;        /* index into mgx_server_desc.class_ids */
    int32_t hold;               /* action hold (>= 1) */
    int64_t n_envs;             /* >= 1 (new sessions); ignored when continuing */
    int32_t horizon;            /* steps to advance (>= 1) */
    int32_t keep;               /* 1: keep the session resident after this request */
    int64_t session;            /* -1: new session; else an id returned by an earlier request */
    uint64_t seed;              /* action stream (and initial state) seed of a new session */
    double arrival;             /* caller's timestamp (s, steady clock of mgx_server_now); 0 = now */
    /* Optional commands (e.g. a policy's), device float [action_rows][m][n_envs of the
     * session], clipped to [-1, 1] when used; NULL: generated from the session's seed. Row r
     * is applied to the request's steps in hold interval floor(t0 / hold) + r, t0 the
     * session's step count when the request is admitted (0 for a new session). A request
     * whose rows do not cover its horizon fails at admission (state 4). The buffer must
     * stay valid until the request is done. */
    const float* actions;
    int64_t action_rows;
} mgx_request;

typedef struct {
    int32_t state;              /* 0 queued, 1 running, 2 done, 3 cancelled, 4 failed */
    int32_t pad;
    int64_t session;            /* session id (valid once admitted) */
    int64_t steps_done;
    double t_arrival, t_admit, t_done;   /* mgx_server_now() clock */
} mgx_request_status;

typedef struct {
    int64_t submitted, completed, cancelled, queued, active;
    int64_t env_steps;          /* completed environment-steps */
    int64_t iterations;         /* launches */
    int64_t bytes_in_use, bytes_peak, budget_bytes;
    double p50_latency, p99_latency, mean_latency;   /* s, over completed requests */
    double wall;                /* s since creation */
} mgx_server_stats;

/* Seconds on the server clock (steady). */
double mgx_server_now(void);
/* MGX_E_INVALID for a class with fins (the server runs propeller classes). */
mgx_status mgx_server_create(const mgx_server_desc* d, mgx_server** out);
/* Thread-safe. MGX_E_BUDGET if the request alone needs more than the budget;
 * MGX_E_INVALID on bad fields or an unknown / busy session. *request_id receives an id. */
mgx_status mgx_server_submit(mgx_server* s, const mgx_request* r, int64_t* request_id);
/* Thread-safe; never blocks on the device. */
mgx_status mgx_server_poll(mgx_server* s, int64_t request_id, mgx_request_status* out);
/* Blocks until the request is done, cancelled or failed, or timeout_s elapses (MGX_E_STATE). */
mgx_status mgx_server_wait(mgx_server* s, int64_t request_id, double timeout_s, mgx_request_status* out);
/* Thread-safe. A queued request is dropped; a running one stops after its in-flight
 * iteration; its session is released unless it was kept by an earlier request. */
mgx_status mgx_server_cancel(mgx_server* s, int64_t request_id);
/* Copies a resident session's state ([13 + m][n_envs], component-major, float) to host
 * memory. MGX_E_INVALID if the session is not resident or capacity is short; MGX_E_STATE
 * while a request on the session is admitted. A request for the session that is queued or
 * submitted during the copy is admitted only after it, so the copy never mixes steps. */
mgx_status mgx_server_read_state(mgx_server* s, int64_t session, float* out, int64_t capacity);
/* Releases a kept session (after its requests finish; MGX_E_STATE while one runs or its
 * state is being read). */
mgx_status mgx_server_release(mgx_server* s, int64_t session);
mgx_status mgx_server_stats_get(mgx_server* s, mgx_server_stats* out);
/* Stops the scheduler after draining in-flight work; frees everything. */
mgx_status mgx_server_destroy(mgx_server* s);

#ifdef __cplusplus
}
#endif
#endif
