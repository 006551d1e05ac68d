"""Station-keeping task on top of the step, plain numpy in double precision (Sec. IV-B: the
vehicle must reach and hold a target pose in moving water, with its position error
converging and its attitude kept within limits; the task is an MDP behind a Gym-style
vector interface whose observation holds only the vehicle's own kinematics and the
task's parameters, and whose action is one command per actuator).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the device task kernel is checked
against it; the product never imports it.

The paper gives no observation, reward or termination; this module fixes one reading,
which the device implements independently from the same description:

- episode start, for global env id g, episode k and seed s: 14 uniforms on [0, 1) of 53
  bits from Philox4x32-10 at key (s mod 2^32, 8 << 24), counter (g, k, j, 0), j = 0..6,
  (w0, w1) then (w2, w3) of each call. Target position p* = b (2 u[0..2] - 1); target
  attitude a pure yaw psi* = pi (2 u3 - 1), q* = (cos psi*/2, 0, 0, sin psi*/2). Start
  at p = 0 with yaw psi = pi (2 u4 - 1), roll phi = t0 (2 u5 - 1), pitch theta =
  t0 (2 u6 - 1), q0 = q_z(psi) q_y(theta) q_x(phi) (rotations about the body's own axes
  in yaw, pitch, roll order), nu_j = v0 (2 u[7+j] - 1), rotor states 0. All in double,
  rounded once to the state's precision.
- observation (13 + m values, the state's own layout): the target position in the body
  frame R(q)^T (p* - p); the attitude error q_e = q*^-1 q, sign chosen so that its scalar
  part is >= 0; nu; the rotor states.
- reward of a transition, on the state it ends in, with a the clipped command held over
  it: exp(-d / sigma_p) - w_att (1 - q_e,w^2) - w_act mean_i a_i^2, where d = |p* - p| and
  1 - q_e,w^2 = sin^2 of half the attitude error angle. 0 if the state is not finite.
- terminated: the state is not finite, or d > d_max, or the body's z axis leans more than
  tilt_max from the world z axis (R(q)_zz < cos tilt_max). truncated: the episode has now
  taken max_steps task steps.
- a task step holds one command for `substeps` steps of the dynamics. When it ends an
  episode (terminated or truncated) the environment starts episode k + 1 at once; the
  returned observation is then the new episode's first, and `final_obs` holds the
  observation of the state the transition ended in (for every environment).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
from synth.philox import philox4x32, u53

STREAM_TASK = 8


@dataclass
class StationDesc:
    target_box: float = 2.0   # b: half-width of the target position box (m)
    tilt0: float = 0.2        # t0: initial roll and pitch half-range (rad)
    v0: float = 0.1           # initial velocity half-range per component
    sigma_p: float = 0.5      # reward position scale (m)
    w_att: float = 0.5        # attitude penalty weight
    w_act: float = 0.01       # command penalty weight
    d_max: float = 5.0        # terminate beyond this distance from the target (m)
    tilt_max: float = 1.2     # terminate beyond this lean from upright (rad)
    max_steps: int = 500      # truncate after this many task steps
    substeps: int = 1         # dynamics steps per task step


def start_uniforms(seed: int, env_ids, episodes) -> np.ndarray:
    """[n, 14] uniforms of the episode start draw."""
    ids = np.asarray(env_ids, dtype=np.uint64).ravel()
    ep = np.broadcast_to(np.asarray(episodes, dtype=np.uint64), ids.shape)
    ctr = np.zeros((ids.size, 7, 4), dtype=np.uint64)
    ctr[..., 0] = ids[:, None]
    ctr[..., 1] = (ep & np.uint64(0xFFFFFFFF))[:, None]
    ctr[..., 2] = np.arange(7, dtype=np.uint64)[None, :]
    key = np.array([seed & 0xFFFFFFFF, STREAM_TASK << 24], dtype=np.uint64)
    w = philox4x32(ctr, key)
    u = np.empty((ids.size, 14))
    u[:, 0::2] = u53(w[..., 0], w[..., 1])
    u[:, 1::2] = u53(w[..., 2], w[..., 3])
    return u


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of [..., 4] quaternions, scalar first."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def quat_axis(angle: np.ndarray, axis: int) -> np.ndarray:
    """Rotation by ``angle`` about body axis 0 (x), 1 (y) or 2 (z)."""
    q = np.zeros(np.shape(angle) + (4,))
    q[..., 0] = np.cos(0.5 * angle)
    q[..., 1 + axis] = np.sin(0.5 * angle)
    return q


def rot(q: np.ndarray) -> np.ndarray:
    """R(q) [..., 3, 3] of unit quaternions [..., 4]: body to world."""
    w, x, y, z = np.moveaxis(q, -1, 0)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def episode_start(desc: StationDesc, seed: int, env_ids, episodes, m: int):
    """(state AoS [n, 21], target [n, 7] = p*, q*) of the episode start draw, in double."""
    u = start_uniforms(seed, env_ids, episodes)
    n = u.shape[0]
    tgt = np.zeros((n, 7))
    tgt[:, 0:3] = desc.target_box * (2.0 * u[:, 0:3] - 1.0)
    tgt[:, 3:7] = quat_axis(np.pi * (2.0 * u[:, 3] - 1.0), 2)
    q0 = quat_mul(quat_mul(quat_axis(np.pi * (2.0 * u[:, 4] - 1.0), 2),
                           quat_axis(desc.tilt0 * (2.0 * u[:, 6] - 1.0), 1)),
                  quat_axis(desc.tilt0 * (2.0 * u[:, 5] - 1.0), 0))
    s = np.zeros((n, oracle.STATE_LEN))
    s[:, 3:7] = q0
    s[:, 7:13] = desc.v0 * (2.0 * u[:, 7:13] - 1.0)
    return s, tgt


def attitude_error(q: np.ndarray, q_target: np.ndarray) -> np.ndarray:
    """q*^-1 q with its scalar part made >= 0."""
    conj = q_target * np.array([1.0, -1.0, -1.0, -1.0])
    qe = quat_mul(conj, q)
    return np.where(qe[..., :1] < 0, -qe, qe)


def observe(state: np.ndarray, target: np.ndarray, m: int) -> np.ndarray:
    """[n, 13 + m] observations of AoS states [n, 21] with targets [n, 7]."""
    p, q = state[:, 0:3], state[:, 3:7]
    R = rot(q)
    o = np.zeros((state.shape[0], 13 + m))
    o[:, 0:3] = np.einsum("nji,nj->ni", R, target[:, 0:3] - p)
    o[:, 3:7] = attitude_error(q, target[:, 3:7])
    o[:, 7:13] = state[:, 7:13]
    o[:, 13:13 + m] = state[:, 13:13 + m]
    return o


def reward_done(desc: StationDesc, state: np.ndarray, target: np.ndarray, a_clipped: np.ndarray, m: int):
    """(reward [n], terminated [n] bool) of transitions ending in ``state``."""
    finite = np.all(np.isfinite(state[:, :13 + m]), axis=1)
    s = np.where(finite[:, None], state, 0.0)
    d = np.linalg.norm(target[:, 0:3] - s[:, 0:3], axis=1)
    qe = attitude_error(s[:, 3:7], target[:, 3:7])
    r = np.exp(-d / desc.sigma_p) - desc.w_att * (1.0 - qe[:, 0] ** 2) \
        - desc.w_act * np.mean(a_clipped[:, :m] ** 2, axis=1)
    r = np.where(finite, r, 0.0)
    up = rot(s[:, 3:7])[:, 2, 2]
    term = ~finite | (d > desc.d_max) | (up < np.cos(desc.tilt_max))
    return r, term


class StationOracle:
    """The task over n environments of one vehicle class: global ids env_off..env_off+n-1,
    or the given ``ids`` (one per entry of ``envs``)."""

    def __init__(self, desc: StationDesc, envs: np.ndarray, m: int, env_off: int = 0, ids=None):
        self.desc, self.envs, self.m = desc, envs, m
        self.ids = (np.arange(env_off, env_off + envs.shape[0], dtype=np.int64) if ids is None
                    else np.asarray(ids, dtype=np.int64))

    def reset(self, seed: int) -> np.ndarray:
        n = self.ids.size
        self.seed = seed
        self.episode = np.zeros(n, dtype=np.int64)
        self.t = np.zeros(n, dtype=np.int64)
        self.state, self.target = episode_start(self.desc, seed, self.ids, self.episode, self.m)
        return observe(self.state, self.target, self.m)

    def step(self, actions: np.ndarray):
        """One task step with commands [n, m]. Returns obs, reward, terminated, truncated,
        final_obs (all per environment)."""
        d, m = self.desc, self.m
        a = np.zeros((actions.shape[0], 1, oracle.MAX_THR))
        a[:, 0, :m] = actions
        self.state, _, _ = oracle.rollout(self.envs, self.state, a, d.substeps, d.substeps)
        a_clipped = np.clip(actions, -1.0, 1.0)
        r, term = reward_done(d, self.state, self.target, a_clipped, m)
        self.t += 1
        trunc = self.t >= d.max_steps
        final = observe(self.state, self.target, m)
        done = term | trunc
        if np.any(done):
            self.episode[done] += 1
            self.t[done] = 0
            s, tg = episode_start(d, self.seed, self.ids[done], self.episode[done], m)
            self.state[done] = s
            self.target[done] = tg
        obs = observe(self.state, self.target, m)
        return obs, r, term, trunc, final
