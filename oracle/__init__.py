"""ctypes front end of the FP64 CPU oracle (``mgx_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by
the CPU-baseline leg of ``bench.py``. The product library never imports or links it.
The C source is compiled here with gcc on first use (``build()``), independently of the
device library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mgx_oracle.c")
HDR = os.path.join(HERE, "mgx_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")
# A test may point the front end at another build of the oracle (planted-mistake checks).
_LIB_OVERRIDE = os.environ.get("MGX_ORACLE_LIB")

MAX_THR = 8
STATE_LEN = 21
FLAG_NO_AMC = 1
FLAG_LAG_EULER = 2

ENV_DTYPE = np.dtype([
    ("m", np.int32), ("flags", np.uint32), ("dt", np.float64), ("g0", np.float64),
    ("mass", np.float64), ("inertia", np.float64, 3), ("added", np.float64, 6),
    ("dlin", np.float64, 6), ("dquad", np.float64, 6), ("buoy", np.float64),
    ("rb", np.float64, 3), ("current", np.float64, 3), ("r", np.float64, (MAX_THR, 3)),
    ("e", np.float64, (MAX_THR, 3)), ("k", np.float64, MAX_THR), ("tau", np.float64, MAX_THR),
    ("deadzone", np.float64, MAX_THR), ("k_rev", np.float64, MAX_THR),
    ("reaction", np.float64, MAX_THR), ("kind", np.int32, MAX_THR), ("span", np.float64, (MAX_THR, 3)),
    ("fin_max", np.float64, MAX_THR), ("fin_lift", np.float64, MAX_THR), ("fin_drag0", np.float64, MAX_THR),
    ("fin_drag", np.float64, MAX_THR), ("rg", np.float64, 3)], align=True)
PROPELLER = 0
FIN = 1

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction, OpenMP)."""
    stale = (not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                    os.path.getmtime(HDR)))
    if force or stale:
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE", SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build()
            L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_sizeof_env.restype = ctypes.c_int32
        L.orc_sizeof_state.restype = ctypes.c_int32
        L.orc_get_threads.restype = ctypes.c_int32
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_lag_factor.restype = ctypes.c_double
        L.orc_lag_factor.argtypes = [P, ctypes.c_int32]
        L.orc_rotation.argtypes = [P, P]
        L.orc_quat_mul.argtypes = [P, P, P]
        L.orc_thrust_wrench.argtypes = [P, P, P]
        L.orc_fin_wrench.argtypes = [P, P, P, P, P]
        L.orc_mass_matrix.argtypes = [P, P]
        L.orc_terms_eval.argtypes = [P, P, P, P, P]
        L.orc_step.argtypes = [P, P, P, P]
        L.orc_rollout.restype = ctypes.c_int32
        L.orc_rollout.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P]
        L.orc_rollout_loss.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, ctypes.c_double, P]
        L.orc_rk4_smooth.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_int64]
        L.orc_rollout_smooth.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int64]
        assert L.orc_sizeof_env() == ENV_DTYPE.itemsize, "orc_env layout mismatch"
        assert L.orc_sizeof_state() == STATE_LEN * 8
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ----------------------------------------------------------------------------- packing

def make_envs(cls, params, dt: float, flags: int = 0, idx=None) -> np.ndarray:
    """Structured array of orc_env for one vehicle class and its per-environment params."""
    n = params.n if idx is None else len(idx)
    sel = slice(None) if idx is None else idx
    env = np.zeros(n, dtype=ENV_DTYPE)
    env["m"] = cls.m
    env["flags"] = flags
    env["dt"] = dt
    env["g0"] = cls.g0
    env["mass"] = params.mass[sel]
    env["inertia"] = cls.inertia
    env["added"] = params.added[:, sel].T
    env["dlin"] = params.dlin[:, sel].T
    env["dquad"] = params.dquad[:, sel].T
    env["buoy"] = params.buoy[sel]
    env["rb"] = cls.rb
    env["current"] = params.current[:, sel].T
    r = np.zeros((MAX_THR, 3)); r[:cls.m] = cls.r
    e = np.zeros((MAX_THR, 3)); e[:cls.m] = cls.e
    e[cls.m:, 0] = 1.0
    k = np.zeros(MAX_THR); k[:cls.m] = cls.k
    tau = np.zeros(MAX_THR); tau[:cls.m] = cls.tau
    dz = np.zeros(MAX_THR); dz[:cls.m] = cls.deadzone
    env["r"], env["e"], env["k"], env["tau"], env["deadzone"] = r, e, k, tau, dz
    krev = np.zeros(MAX_THR); react = np.zeros(MAX_THR)
    if getattr(cls, "k_rev", None) is not None:
        krev[:cls.m] = cls.k_rev
    if getattr(cls, "reaction", None) is not None:
        react[:cls.m] = cls.reaction
    env["k_rev"], env["reaction"] = krev, react
    if getattr(cls, "rg", None) is not None:
        env["rg"] = cls.rg
    if getattr(cls, "kind", None) is not None:
        kind = np.zeros(MAX_THR, dtype=np.int32); kind[:cls.m] = cls.kind
        span = np.zeros((MAX_THR, 3)); span[:cls.m] = cls.span
        env["kind"], env["span"] = kind, span
        for f in ("fin_max", "fin_lift", "fin_drag0", "fin_drag"):
            a = np.zeros(MAX_THR); a[:cls.m] = getattr(cls, f)
            env[f] = a
    return env


def pack_state(p, q, nu, n) -> np.ndarray:
    """Columns p[3,N], q[4,N], nu[6,N], n[m,N] -> AoS [N,21] float64."""
    N = p.shape[1]
    s = np.zeros((N, STATE_LEN))
    s[:, 0:3] = p.T
    s[:, 3:7] = q.T
    s[:, 7:13] = nu.T
    s[:, 13:13 + n.shape[0]] = n.T
    return s


def unpack_state(s: np.ndarray, m: int) -> np.ndarray:
    """AoS [N,21] -> stacked columns [13+m, N]."""
    return np.ascontiguousarray(np.concatenate([s[:, 0:13], s[:, 13:13 + m]], axis=1).T)


def pack_actions(a: np.ndarray) -> np.ndarray:
    """[rows, m, N] -> [N, rows, 8] float64."""
    rows, m, N = a.shape
    out = np.zeros((N, rows, MAX_THR))
    out[:, :, :m] = np.transpose(a, (2, 0, 1))
    return out


# ----------------------------------------------------------------------------- calls

def rollout(envs, state, actions, hold, n_steps, t0=0, row0=0, traj=False, forces=False):
    """Advance AoS ``state`` [N,21] in place; ``actions`` packed [N, rows, 8].
    Returns (traj [N,K,21] or None, forces [N,K,12] or None)."""
    L = lib()
    state = np.ascontiguousarray(state, dtype=np.float64)
    actions = np.ascontiguousarray(actions, dtype=np.float64)
    N, rows = actions.shape[0], actions.shape[1]
    assert state.shape == (N, STATE_LEN) and envs.shape == (N,)
    tr = np.zeros((N, n_steps, STATE_LEN)) if traj else None
    fo = np.zeros((N, n_steps, 12)) if forces else None
    rc = L.orc_rollout(N, _p(envs), _p(state), _p(actions), rows, int(hold), int(t0), int(row0),
                       int(n_steps), _p(tr), _p(fo))
    if rc != 0:
        raise IndexError("action row out of range")
    return state, tr, fo


def step(env_one, state_one, a, want_forces=False):
    s = np.ascontiguousarray(state_one, dtype=np.float64).copy()
    aa = np.zeros(MAX_THR)
    aa[:len(a)] = a
    f = np.zeros(12) if want_forces else None
    lib().orc_step(_p(env_one), _p(s), _p(aa), _p(f))
    return (s, f) if want_forces else s


def terms(env_one, q, nu, n_lagged):
    out = np.zeros(42)
    nl = np.zeros(MAX_THR)
    nl[:len(n_lagged)] = n_lagged
    lib().orc_terms_eval(_p(env_one), _p(np.ascontiguousarray(q, dtype=np.float64)),
                         _p(np.ascontiguousarray(nu, dtype=np.float64)), _p(nl), _p(out))
    names = ["tau", "crb", "ca", "damp", "restore", "hadd", "total"]
    return {k: out[6 * i:6 * i + 6] for i, k in enumerate(names)}


def rotation(q):
    R = np.zeros((3, 3))
    lib().orc_rotation(_p(np.ascontiguousarray(q, dtype=np.float64)), _p(R))
    return R


def quat_mul(a, b):
    out = np.zeros(4)
    lib().orc_quat_mul(_p(np.ascontiguousarray(a, dtype=np.float64)),
                       _p(np.ascontiguousarray(b, dtype=np.float64)), _p(out))
    return out


def thrust_wrench(env_one, n):
    out = np.zeros(6)
    nn = np.zeros(MAX_THR)
    nn[:len(n)] = n
    lib().orc_thrust_wrench(_p(env_one), _p(nn), _p(out))
    return out


def mass_matrix(env_one):
    """M = M_RB + M_A (6x6) of one environment."""
    out = np.zeros(36)
    lib().orc_mass_matrix(_p(env_one), _p(out))
    return out.reshape(6, 6)


def fin_wrench(env_one, n, vr, w):
    """Wrench of the fins of one environment at rotor state n, relative velocity vr, rate w."""
    out = np.zeros(6)
    nn = np.zeros(MAX_THR)
    nn[:len(n)] = n
    vr = np.ascontiguousarray(vr, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    lib().orc_fin_wrench(_p(env_one), _p(nn), _p(vr), _p(w), _p(out))
    return out


def lag_factor(env_one, i):
    return lib().orc_lag_factor(_p(env_one), int(i))


def rollout_loss(envs, state0, actions, horizon, waypoints, act_weight):
    """Per-environment loss; actions [N, H, 8], waypoints [N, 3]."""
    N = envs.shape[0]
    out = np.zeros(N)
    lib().orc_rollout_loss(N, _p(envs), _p(np.ascontiguousarray(state0, dtype=np.float64)),
                           _p(np.ascontiguousarray(actions, dtype=np.float64)), int(horizon),
                           _p(np.ascontiguousarray(waypoints, dtype=np.float64)), float(act_weight),
                           _p(out))
    return out


def rk4_smooth(envs, state, smooth, h, n_steps):
    state = np.ascontiguousarray(state, dtype=np.float64).copy()
    lib().orc_rk4_smooth(envs.shape[0], _p(envs), _p(state),
                         _p(np.ascontiguousarray(smooth, dtype=np.float64)), float(h), int(n_steps))
    return state


def rollout_smooth(envs, state, smooth, n_steps):
    state = np.ascontiguousarray(state, dtype=np.float64).copy()
    lib().orc_rollout_smooth(envs.shape[0], _p(envs), _p(state),
                             _p(np.ascontiguousarray(smooth, dtype=np.float64)), int(n_steps))
    return state
