"""Seeded synthetic workloads: vehicle classes, per-environment parameters, initial
states, action streams, waypoints and serving traces.

This module only draws numbers. It holds none of the step's arithmetic: the oracle and
the device path each compute everything derived from these inputs (mass inverse, lag
factor, allocation, forces) on their own. Two screening checks look at a candidate class
the way a vehicle designer would (is the thruster layout able to push in every direction;
is the explicit step at this dt monotone for the damping drawn) and redraw if not.

Every value is drawn in float64 and rounded once to float32, so that both sides start
from the same float32 numbers (the oracle widens them back to float64).

Ranges follow the workloads of the paper's experiments as restated for this project:
mass 10-15 kg, added mass 0.1-0.5x the rigid-body diagonal, linear damping 1-10 and
quadratic damping 5-50 per degree of freedom, buoyancy 1.00-1.02x weight with the centre
of buoyancy 0-2 cm above the centre of gravity, thrust gain 20-40 N, lag time constant
0.05-0.15 s, actions uniform in [-1, 1].
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .philox import philox4x32, u53, action_value

MASTER_SEED = 250309203

STREAM_CLASS = 1
STREAM_ENV = 2
STREAM_INIT = 3
STREAM_ACTION = 4
STREAM_SERVE = 5
STREAM_WAYPOINT = 6

G0 = 9.81
TWO_PI = 2.0 * np.pi


def f32(x):
    """Round to float32 and widen back to float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _key(seed: int, stream: int, sub: int = 0):
    return np.array([seed & 0xFFFFFFFF, ((stream & 0xFF) << 24) | (sub & 0xFFFFFF)], dtype=np.uint64)


def _uniforms(seed, stream, sub, c0, c1, count):
    """``count`` float64 uniforms on [0,1) for counter prefix (c0, c1); c0 may be an array."""
    c0 = np.atleast_1d(np.asarray(c0, dtype=np.uint64))
    n_calls = (count + 1) // 2
    ctr = np.zeros(c0.shape + (n_calls, 4), dtype=np.uint64)
    ctr[..., 0] = c0[..., None]
    ctr[..., 1] = c1
    ctr[..., 2] = np.arange(n_calls, dtype=np.uint64)
    w = philox4x32(ctr, _key(seed, stream, sub))
    u = np.concatenate([u53(w[..., 0], w[..., 1])[..., None], u53(w[..., 2], w[..., 3])[..., None]], axis=-1)
    return u.reshape(c0.shape + (2 * n_calls,))[..., :count]


def _normals(u):
    """Box-Muller: pairs of uniforms -> pairs of standard normals (last axis even)."""
    u1 = 1.0 - u[..., 0::2]  # (0, 1]
    u2 = u[..., 1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(u.shape, dtype=np.float64)
    z[..., 0::2] = rad * np.cos(TWO_PI * u2)
    z[..., 1::2] = rad * np.sin(TWO_PI * u2)
    return z


@dataclass
class VehicleClass:
    """One vehicle class: thruster layout and the nominal per-environment parameters."""

    m: int
    r: np.ndarray          # [m,3] thruster positions in the body frame (m)
    e: np.ndarray          # [m,3] thrust directions (unit, then rounded to float32)
    k: np.ndarray          # [m]   thrust gain (N at |n| = 1)
    tau: np.ndarray        # [m]   rotor time constant (s); 0 = zero-order rotor model
    deadzone: np.ndarray   # [m]   dead zone on |n|
    inertia: np.ndarray    # [3]   principal moments about the centre of gravity (kg m^2)
    rb: np.ndarray         # [3]   centre of buoyancy in the body frame (m); z < 0 is above
    g0: float
    mass: float
    added: np.ndarray      # [6]   added-mass diagonal (positive entries)
    dlin: np.ndarray       # [6]
    dquad: np.ndarray      # [6]
    buoy: float            # buoyancy force (N)
    attempts: int = 1
    index: int = 0
    k_rev: np.ndarray | None = None     # [m] reverse thrust gain (N at n = -1); None = k
    reaction: np.ndarray | None = None  # [m] shaft torque per unit thrust about e (m); None = 0
    kind: np.ndarray | None = None      # [m] 0 propeller, 1 fin (rudder); None = all propellers
    span: np.ndarray | None = None      # [m,3] fin hinge axes (e is then the chord)
    fin_max: np.ndarray | None = None   # [m] fin deflection at n = 1 (rad)
    fin_lift: np.ndarray | None = None  # [m] rho A c_L / 2 (kg/m)
    fin_drag0: np.ndarray | None = None  # [m] rho A c_D0 / 2 (kg/m)
    fin_drag: np.ndarray | None = None  # [m] rho A c_D / 2 (kg/m)
    rg: np.ndarray | None = None        # [3] centre of gravity from the body origin (payload); None = 0


@dataclass
class EnvParams:
    """Per-environment parameters, one column per environment (float32 values in float64)."""

    mass: np.ndarray       # [N]
    added: np.ndarray      # [6,N]
    dlin: np.ndarray       # [6,N]
    dquad: np.ndarray      # [6,N]
    buoy: np.ndarray       # [N]
    current: np.ndarray    # [3,N] constant world-frame current (m/s)
    resampled: int = 0

    @property
    def n(self):
        return self.mass.shape[0]

    def subset(self, idx):
        return EnvParams(self.mass[idx], self.added[:, idx], self.dlin[:, idx], self.dquad[:, idx],
                         self.buoy[idx], self.current[:, idx])

    @staticmethod
    def concat(parts):
        return EnvParams(np.concatenate([p.mass for p in parts]),
                         np.concatenate([p.added for p in parts], axis=1),
                         np.concatenate([p.dlin for p in parts], axis=1),
                         np.concatenate([p.dquad for p in parts], axis=1),
                         np.concatenate([p.buoy for p in parts]),
                         np.concatenate([p.current for p in parts], axis=1),
                         sum(p.resampled for p in parts))


@dataclass
class State:
    """State columns: p [3,N], q [4,N] (w,x,y,z), nu [6,N] (u,v,w,p,q,r), n [m,N]."""

    p: np.ndarray
    q: np.ndarray
    nu: np.ndarray
    n: np.ndarray

    def stacked(self):
        return np.concatenate([self.p, self.q, self.nu, self.n], axis=0)

    @staticmethod
    def from_stacked(x, m):
        return State(x[0:3], x[3:7], x[7:13], x[13:13 + m])


# ----------------------------------------------------------------------------- screening

def _layout_columns(r, e):
    """[6,m] columns (e_i; r_i x e_i) of a thruster layout, for screening only."""
    return np.concatenate([e.T, np.cross(r, e).T], axis=0)


def layout_conditioning(r, e, lever=0.25):
    """sigma_min / sigma_max of the layout, moments scaled by 1/lever, over min(m,6) values."""
    cols = _layout_columns(r, e)
    cols = cols * np.array([1, 1, 1, 1 / lever, 1 / lever, 1 / lever])[:, None]
    s = np.linalg.svd(cols, compute_uv=False)
    kdim = min(cols.shape[1], 6)
    return s[kdim - 1] / s[0]


def damping_step_ratio(mass, inertia, added, dlin, dquad, buoy, g0, rb, k, r, e, dt,
                       nu_floor=0.8, current_bound=0.0):
    """Largest dt*lambda over the six degrees of freedom (vectorised over trailing env axis).

    lambda_j = (d_L + 2 d_Q nu_max) / M_jj, the local decay rate of the damped degree of
    freedom at the largest speed the available force could sustain; the explicit step
    decays monotonically when dt*lambda <= 1.
    """
    cols = np.abs(_layout_columns(r, e))  # [6,m]
    push = cols @ np.asarray(k)           # [6]
    mass = np.asarray(mass, dtype=np.float64)
    weight = mass * g0
    ratios = []
    for j in range(6):
        mjj = (mass if j < 3 else inertia[j - 3]) + added[j]
        if j < 3:
            fmax = push[j] + np.abs(weight - buoy)
        else:
            fmax = push[j] + buoy * np.linalg.norm(rb)
        dl, dq = dlin[j], dquad[j]
        numax = np.where(dq > 0, (-dl + np.sqrt(dl * dl + 4 * dq * fmax)) / (2 * np.maximum(dq, 1e-300)),
                         fmax / np.maximum(dl, 1e-300))
        numax = np.maximum(numax, nu_floor) + (current_bound if j < 3 else 0.0)
        ratios.append(dt * (dl + 2 * dq * numax) / mjj)
    return np.max(np.stack(ratios), axis=0)


# ----------------------------------------------------------------------------- classes

def draw_class(m: int, class_index: int = 0, seed: int = MASTER_SEED, dt: float = 0.01,
               min_conditioning: float = 0.05, max_attempts: int = 10000) -> VehicleClass:
    """Draw one vehicle class; redraw until the layout is well conditioned over min(m,6)
    directions and the nominal damping passes the step-ratio screen at ``dt``."""
    for attempt in range(max_attempts):
        u = _uniforms(seed, STREAM_CLASS, class_index, attempt, 0, 32 + 12 * m)[0]
        it = iter(u)

        def U(lo, hi):
            return lo + (hi - lo) * next(it)

        mass = U(10.0, 15.0)
        rho = np.array([U(0.25, 0.35) for _ in range(3)])
        inertia = mass * rho ** 2
        diag_rb = np.array([mass, mass, mass, *inertia])
        added = np.array([U(0.1, 0.5) for _ in range(6)]) * diag_rb
        dlin = np.array([U(1.0, 10.0) for _ in range(6)])
        dquad = np.array([U(5.0, 50.0) for _ in range(6)])
        beta = U(1.00, 1.02)
        h = U(0.0, 0.02)
        k = np.array([U(20.0, 40.0) for _ in range(m)])
        tau = np.array([U(0.05, 0.15) for _ in range(m)])
        r = np.array([[U(-0.25, 0.25), U(-0.20, 0.20), U(-0.10, 0.10)] for _ in range(m)])
        z = _normals(np.array([next(it) for _ in range(4 * m)]).reshape(m, 4))[:, :3]
        e = z / np.linalg.norm(z, axis=1, keepdims=True)
        cls = VehicleClass(
            m=m, r=f32(r), e=f32(e), k=f32(k), tau=f32(tau), deadzone=np.zeros(m),
            inertia=f32(inertia), rb=f32([0.0, 0.0, -h]), g0=G0, mass=float(f32(mass)),
            added=f32(added), dlin=f32(dlin), dquad=f32(dquad),
            buoy=float(f32(beta * mass * G0)), attempts=attempt + 1, index=class_index)
        if layout_conditioning(cls.r, cls.e) < min_conditioning:
            continue
        ratio = damping_step_ratio(cls.mass, cls.inertia, cls.added, cls.dlin, cls.dquad, cls.buoy,
                                   cls.g0, cls.rb, cls.k, cls.r, cls.e, dt)
        if ratio > 1.0:
            continue
        return cls
    raise RuntimeError("no class passed the screens")


def propeller_variants(cls: VehicleClass, seed: int = MASTER_SEED) -> VehicleClass:
    """The same class with the propeller variants switched on: a dead zone U[0.05, 0.15] on
    |n|, a reverse gain U[0.6, 0.85] times the forward gain (propellers push less astern),
    and a shaft torque of U[0.02, 0.05] m per unit thrust, handedness alternating with the
    thruster index (counter-rotating pairs)."""
    m = cls.m
    u = _uniforms(seed, STREAM_CLASS, 40 + cls.index, 0, 1, 3 * m)[0]
    sign = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    return replace(cls, deadzone=f32(0.05 + 0.10 * u[:m]), k_rev=f32(cls.k * (0.6 + 0.25 * u[m:2 * m])),
                   reaction=f32(sign * (0.02 + 0.03 * u[2 * m:])))


def rudder_class(seed: int = MASTER_SEED) -> VehicleClass:
    """A rudder-propeller vehicle (a main propeller astern and a cruciform tail): the hull
    of a drawn class, one propeller on the centre line pushing along x, and four fins at
    the tail with their chords along x, two with a horizontal hinge (pitch) and two with a
    vertical hinge (yaw). Fin deflection U[0.35, 0.5] rad at full command, servo lag
    U[0.05, 0.1] s, lift gain rho A c_L / 2 U[8, 15] kg/m, drag gains U[0.2, 0.4] and U[3, 6]
    kg/m (fins of about 0.01 m^2 in sea water)."""
    hull = draw_class(6, 30, seed)
    u = _uniforms(seed, STREAM_CLASS, 50, 0, 2, 32)[0]
    it = iter(u)

    def U(lo, hi):
        return lo + (hi - lo) * next(it)

    m = 5
    r = np.array([[-0.6, 0.0, 0.0], [-0.5, 0.1, 0.0], [-0.5, -0.1, 0.0], [-0.5, 0.0, 0.1], [-0.5, 0.0, -0.1]])
    e = np.tile([1.0, 0.0, 0.0], (m, 1))
    span = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    k = np.array([U(40.0, 60.0), 0.0, 0.0, 0.0, 0.0])
    tau = np.array([U(0.05, 0.15)] + [U(0.05, 0.10) for _ in range(4)])
    fin_max = np.array([0.0] + [U(0.35, 0.5) for _ in range(4)])
    fin_lift = np.array([0.0] + [U(8.0, 15.0) for _ in range(4)])
    fin_drag0 = np.array([0.0] + [U(0.2, 0.4) for _ in range(4)])
    fin_drag = np.array([0.0] + [U(3.0, 6.0) for _ in range(4)])
    return replace(hull, m=m, r=f32(r), e=f32(e), k=f32(k), tau=f32(tau), deadzone=np.zeros(m), k_rev=None,
                   reaction=None, kind=np.array([0, 1, 1, 1, 1], dtype=np.int32), span=f32(span),
                   fin_max=f32(fin_max), fin_lift=f32(fin_lift), fin_drag0=f32(fin_drag0), fin_drag=f32(fin_drag),
                   index=30)


def payload_class(seed: int = MASTER_SEED) -> VehicleClass:
    """The 6-thruster class carrying an off-centre payload: the centre of gravity moves to
    r_g = (U[-3, 3], U[-2, 2], U[0.5, 3]) cm from the body origin (below it, so the body
    stays upright), the inertia stays given about the centre of gravity."""
    c = plain_class(seed)
    u = _uniforms(seed, STREAM_CLASS, 60, 0, 3, 4)[0]
    rg = np.array([-0.03 + 0.06 * u[0], -0.02 + 0.04 * u[1], 0.005 + 0.025 * u[2]])
    return replace(c, rg=f32(rg), index=60)


def nominal_params(cls: VehicleClass, n: int) -> EnvParams:
    """Every environment at the class nominal, no current."""
    return EnvParams(np.full(n, cls.mass), np.repeat(cls.added[:, None], n, 1),
                     np.repeat(cls.dlin[:, None], n, 1), np.repeat(cls.dquad[:, None], n, 1),
                     np.full(n, cls.buoy), np.zeros((3, n)))


def randomised_params(cls: VehicleClass, n: int, seed: int = MASTER_SEED, env_offset: int = 0,
                      spread: float = 0.2, current_sigma: float = 0.3, dt: float = 0.01,
                      max_attempts: int = 1000) -> EnvParams:
    """Domain randomisation: one U[1-spread, 1+spread] factor per environment for each of
    mass, added mass (all six entries), damping (linear and quadratic together) and
    buoyancy; inertia stays at the class value. A constant world-frame current with
    N(0, current_sigma^2) per axis. Environments failing the damping screen redraw their
    factors (counted in ``resampled``)."""
    ids = np.arange(env_offset, env_offset + n, dtype=np.uint64)
    factors = np.empty((n, 4))
    pending = np.arange(n)
    resampled = 0
    cur = _normals(_uniforms(seed, STREAM_ENV, cls.index, ids, 0xFFFF, 4))[:, :3] * current_sigma
    cur_bound = 4.0 * current_sigma * np.sqrt(3.0)
    for attempt in range(max_attempts):
        u = _uniforms(seed, STREAM_ENV, cls.index, ids[pending], attempt, 4)
        factors[pending] = (1.0 - spread) + 2.0 * spread * u
        f = factors[pending].T
        mass = f32(cls.mass * f[0])
        added = f32(cls.added[:, None] * f[1])
        dlin = f32(cls.dlin[:, None] * f[2])
        dquad = f32(cls.dquad[:, None] * f[2])
        buoy = f32(cls.buoy * f[3])
        ratio = damping_step_ratio(mass, cls.inertia, added, dlin, dquad, buoy, cls.g0, cls.rb,
                                   cls.k, cls.r, cls.e, dt, current_bound=cur_bound)
        bad = ratio > 1.0
        if not bad.any():
            break
        resampled += int(bad.sum())
        pending = pending[bad]
    else:
        raise RuntimeError("damping screen did not pass")
    f = factors.T
    return EnvParams(f32(cls.mass * f[0]), f32(cls.added[:, None] * f[1]),
                     f32(cls.dlin[:, None] * f[2]), f32(cls.dquad[:, None] * f[2]),
                     f32(cls.buoy * f[3]), f32(cur.T), resampled)


# ----------------------------------------------------------------------------- states, actions

def initial_state(n: int, m: int, seed: int = MASTER_SEED, env_offset: int = 0,
                  sigma: float = 0.2) -> State:
    """p = 0; q uniform on the unit sphere in R^4 (normalised Gaussian); nu ~ N(0, sigma^2)
    per component; rotor states 0."""
    ids = np.arange(env_offset, env_offset + n, dtype=np.uint64)
    z = _normals(_uniforms(seed, STREAM_INIT, 0, ids, 0, 10))  # [n,10]
    q = z[:, :4] / np.linalg.norm(z[:, :4], axis=1, keepdims=True)
    nu = sigma * z[:, 4:10]
    return State(np.zeros((3, n)), f32(q.T), f32(nu.T), np.zeros((m, n)))


def action_words(n: int, m: int, rows: int, seed: int = MASTER_SEED, env_offset: int = 0,
                 row_offset: int = 0) -> np.ndarray:
    """Raw generator words [rows, m, n] for the action stream: counter (env, row, i // 4, 0)."""
    env = np.arange(env_offset, env_offset + n, dtype=np.uint64)
    row = np.arange(row_offset, row_offset + rows, dtype=np.uint64)
    n_calls = (m + 3) // 4
    ctr = np.zeros((rows, n_calls, n, 4), dtype=np.uint64)
    ctr[..., 0] = env[None, None, :]
    ctr[..., 1] = row[:, None, None]
    ctr[..., 2] = np.arange(n_calls, dtype=np.uint64)[None, :, None]
    w = philox4x32(ctr, _key(seed, STREAM_ACTION))        # [rows, calls, n, 4]
    w = np.moveaxis(w, -1, 2).reshape(rows, n_calls * 4, n)  # thruster i = 4*call + word
    return w[:, :m, :]


def actions(n: int, m: int, rows: int, seed: int = MASTER_SEED, env_offset: int = 0,
            row_offset: int = 0) -> np.ndarray:
    """float32 actions [rows, m, n], uniform on [-1, 1) with 2**-23 resolution."""
    return action_value(action_words(n, m, rows, seed, env_offset, row_offset))


def waypoints(n: int, seed: int = MASTER_SEED, sigma: float = 2.0, env_offset: int = 0) -> np.ndarray:
    """[3, n] targets, N(0, sigma^2) per axis."""
    ids = np.arange(env_offset, env_offset + n, dtype=np.uint64)
    z = _normals(_uniforms(seed, STREAM_WAYPOINT, 0, ids, 0, 4))[:, :3]
    return f32(sigma * z.T)


# ----------------------------------------------------------------------------- workloads

HETERO_M = (4, 5, 6, 8, 8)
HETERO_N = (512, 3000, 20000, 40000, 7000)


@dataclass
class Workload:
    name: str
    classes: list
    n_envs: list
    params: EnvParams
    state: list            # one State per class
    steps: int
    hold: int
    dt: float = 0.01
    extra: dict = field(default_factory=dict)

    @property
    def n_total(self):
        return int(sum(self.n_envs))

    def actions(self, rows: int, seed: int = MASTER_SEED, row_offset: int = 0):
        """Per-class action arrays [rows, m_c, n_c] for global environment ids."""
        out, off = [], 0
        for c, n in zip(self.classes, self.n_envs):
            out.append(actions(n, c.m, rows, seed, env_offset=off, row_offset=row_offset))
            off += n
        return out


def _build(name, classes, ns, steps, hold, dr, current_sigma, seed, dt=0.01):
    params, states, off = [], [], 0
    for c, n in zip(classes, ns):
        if dr:
            params.append(randomised_params(c, n, seed, off, current_sigma=current_sigma, dt=dt))
        else:
            params.append(nominal_params(c, n))
        states.append(initial_state(n, c.m, seed, off))
        off += n
    return Workload(name, list(classes), list(ns), EnvParams.concat(params), states, steps, hold, dt)


def mixed(classes, ns, steps: int = 100, seed: int = MASTER_SEED, hold: int = 10) -> Workload:
    """Any list of classes with the given environment counts, randomised parameters and
    currents, commands resampled every ``hold`` steps."""
    return _build(f"mixed_{sum(ns)}x{steps}", list(classes), list(ns), steps, hold, True, 0.3, seed)


def plain_class(seed: int = MASTER_SEED):
    """The 6-thruster class shared by the plain and randomised workloads."""
    return draw_class(6, 0, seed)


def hetero_classes(seed: int = MASTER_SEED):
    return [draw_class(m, 1 + i, seed) for i, m in enumerate(HETERO_M)]


def many_classes(seed: int = MASTER_SEED, steps: int = 100) -> Workload:
    """The widest batch the library accepts: 16 classes with 1..8 thrusters (each count
    twice) and ragged environment counts (1 to 1000, many not multiples of 64), randomised
    parameters and currents, actions resampled every 10 steps."""
    ms = [1 + (i % 8) for i in range(16)]
    classes = [draw_class(m, 20 + i, seed) for i, m in enumerate(ms)]
    ns = [1, 63, 64, 65, 127, 130, 200, 257, 3, 70, 129, 64, 500, 31, 96, 1000]
    return _build("many_classes_16", classes, ns, steps, 10, True, 0.3, seed)


def plain_small(seed: int = MASTER_SEED, n: int = 1024, steps: int = 1000) -> Workload:
    """One 6-thruster class, 1024 environments at the class nominal, no current, actions
    resampled every 10 steps."""
    return _build("plain_small_1024x1000", [plain_class(seed)], [n], steps, 10, False, 0.0, seed)


def randomised(seed: int = MASTER_SEED, n: int = 65536, steps: int = 1000) -> Workload:
    """The same class, 65,536 environments, +-20% per-environment randomisation and a
    constant N(0, 0.3^2) world current per environment, actions resampled every 10 steps."""
    return _build(f"dr_{n}x{steps}", [plain_class(seed)], [n], steps, 10, True, 0.3, seed)


def propellers(seed: int = MASTER_SEED, n: int = 65536, steps: int = 1000) -> Workload:
    """The randomised workload with the propeller variants of ``propeller_variants``: dead
    zones, direction-dependent gains and shaft torques on every thruster."""
    return _build(f"prop_{n}x{steps}", [propeller_variants(plain_class(seed), seed)], [n], steps, 10, True, 0.3,
                  seed)


def payload(seed: int = MASTER_SEED, n: int = 65536, steps: int = 1000) -> Workload:
    """The randomised workload with the payload class of ``payload_class``."""
    return _build(f"payload_{n}x{steps}", [payload_class(seed)], [n], steps, 10, True, 0.3, seed)


def rudders(seed: int = MASTER_SEED, n: int = 65536, steps: int = 1000) -> Workload:
    """The rudder-propeller class of ``rudder_class`` with the randomisation and currents of
    the randomised workload, commands resampled every 10 steps."""
    return _build(f"rudder_{n}x{steps}", [rudder_class(seed)], [n], steps, 10, True, 0.3, seed)


def heterogeneous(seed: int = MASTER_SEED, scale: float = 1.0, steps: int = 1000) -> Workload:
    """Five classes with 4, 5, 6, 8, 8 thrusters and 512/3000/20000/40000/7000 envs."""
    ns = [max(1, int(round(n * scale))) for n in HETERO_N]
    return _build(f"hetero_{sum(ns)}x{steps}", hetero_classes(seed), ns, steps, 10, False, 0.0, seed)


def differentiable(seed: int = MASTER_SEED, n: int = 8192, horizon: int = 256) -> Workload:
    """The 8-thruster class (the fourth heterogeneous class), per-step actions, a
    N(0, 2^2) waypoint per environment."""
    cls = draw_class(8, 4, seed)
    w = _build(f"adjoint_{n}x{horizon}", [cls], [n], horizon, 1, False, 0.0, seed)
    w.extra["waypoints"] = waypoints(n, seed)
    w.extra["act_weight"] = 1e-3
    return w


def serving_trace(seed: int = MASTER_SEED, rate: float = 200.0, duration: float = 60.0,
                  n_classes: int = 5, n_lo: int = 64, n_hi: int = 16384, h_max: int = 500,
                  session_p: float = 0.5, session_mean: float = 4.0):
    """Open-loop Poisson arrivals. Each request: arrival time, class, env count
    (log-uniform in [n_lo, n_hi]), horizon (uniform 1..h_max), session id (half of the
    requests continue an open session of the same class and size, geometric length with
    mean ``session_mean``), and a request seed for its action stream."""
    n_req_max = int(rate * duration * 2 + 100)
    u = _uniforms(seed, STREAM_SERVE, 0, np.arange(n_req_max, dtype=np.uint64), 0, 8)
    gaps = -np.log(1.0 - u[:, 0]) / rate
    t = np.cumsum(gaps)
    reqs = []
    open_sessions = []   # [session id, class, n, remaining]
    next_sid = 0
    for i in range(n_req_max):
        if t[i] > duration:
            break
        cont = open_sessions and u[i, 1] < session_p
        if cont:
            j = int(u[i, 2] * len(open_sessions))
            s = open_sessions[j]
            sid, cls, n = s[0], s[1], s[2]
            s[3] -= 1
            if s[3] <= 0:
                open_sessions.pop(j)
        else:
            cls = int(u[i, 3] * n_classes)
            n = int(round(np.exp(np.log(n_lo) + (np.log(n_hi) - np.log(n_lo)) * u[i, 4])))
            sid = next_sid
            next_sid += 1
            length = 1 + int(np.floor(np.log(1.0 - u[i, 5]) / np.log(1.0 - 1.0 / session_mean)))
            if length > 1:
                open_sessions.append([sid, cls, n, length - 1])
        horizon = 1 + int(u[i, 6] * h_max)
        reqs.append(dict(arrival=float(t[i]), cls=cls, n=n, horizon=horizon, session=sid,
                         seed=int((seed * 1000003 + i) & 0xFFFFFFFF), continues=bool(cont)))
    return reqs
