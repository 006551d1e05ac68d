"""ctypes binding of the mgx C ABI (include/mgx.h).

Argument marshalling only: every computation happens in libmgx.so's HIP kernels. The
functions keep the C names; ``Batch`` is a small convenience wrapper that owns a batch
handle and passes torch tensors as device pointers with torch's current HIP stream.
The binding raises if the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# MGX_LIB selects another in-tree build of the same sources (e.g. the diagnostic one).
LIB_PATH = os.environ.get("MGX_LIB") or os.path.join(PKG, "libmgx.so")

MGX_OK = 0
MGX_E_INVALID = -1
MGX_E_NOMEM = -2
MGX_E_DEVICE = -3
MGX_E_NOT_SPD = -4
MGX_E_NONFINITE = -5
MGX_E_BUDGET = -6
MGX_E_STATE = -7

MAX_THRUSTERS = 8
MAX_CLASSES = 16
STATE_FIXED = 13
FORCE_LEN = 12
FP32 = 4
FP64 = 8
FLAG_NO_AMC = 1
FLAG_LAG_EULER = 2
COST_SHAPED = 0x80000000
ACT_PROPELLER = 0
ACT_FIN = 1
STEP_UNFUSED = 1
STEP_STATS = 2
LAUNCH_PER_CLASS = 0
LAUNCH_PERSISTENT = 1
SERVE_FIFO = 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, 4


class MgxError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class ClassDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("r", (ctypes.c_double * 3) * MAX_THRUSTERS), ("e", (ctypes.c_double * 3) * MAX_THRUSTERS),
                ("k", ctypes.c_double * MAX_THRUSTERS), ("tau", ctypes.c_double * MAX_THRUSTERS),
                ("deadzone", ctypes.c_double * MAX_THRUSTERS), ("inertia", ctypes.c_double * 3),
                ("rb", ctypes.c_double * 3), ("g0", ctypes.c_double),
                ("k_rev", ctypes.c_double * MAX_THRUSTERS), ("reaction", ctypes.c_double * MAX_THRUSTERS),
                ("kind", ctypes.c_int32 * MAX_THRUSTERS), ("span", (ctypes.c_double * 3) * MAX_THRUSTERS),
                ("fin_max", ctypes.c_double * MAX_THRUSTERS), ("fin_lift", ctypes.c_double * MAX_THRUSTERS),
                ("fin_drag0", ctypes.c_double * MAX_THRUSTERS), ("fin_drag", ctypes.c_double * MAX_THRUSTERS),
                ("rg", ctypes.c_double * 3)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("class_ids", ctypes.POINTER(ctypes.c_int32)), ("n_envs", ctypes.POINTER(ctypes.c_int64)),
                ("dt", ctypes.c_double), ("flags", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("state", ctypes.c_void_p), ("record", ctypes.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


class Layout(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_total", ctypes.c_int64), ("n_pad_total", ctypes.c_int64),
                ("state_elems", ctypes.c_int64), ("row_elems", ctypes.c_int64),
                ("force_row_elems", ctypes.c_int64),
                ("m", ctypes.c_int32 * MAX_CLASSES), ("n", ctypes.c_int64 * MAX_CLASSES),
                ("n_pad", ctypes.c_int64 * MAX_CLASSES), ("env_off", ctypes.c_int64 * MAX_CLASSES),
                ("state_off", ctypes.c_int64 * MAX_CLASSES), ("action_off", ctypes.c_int64 * MAX_CLASSES),
                ("force_off", ctypes.c_int64 * MAX_CLASSES), ("record_elems", ctypes.c_int64),
                ("record_off", ctypes.c_int64 * MAX_CLASSES)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("K", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("us_per_chunk", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("class_ids", ctypes.POINTER(ctypes.c_int32)),
                ("nominal", ctypes.POINTER(ctypes.c_double)), ("dt", ctypes.c_double),
                ("batch_flags", ctypes.c_uint32), ("serve_flags", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_int64), ("chunk_steps", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("device", ctypes.c_int32), ("streams", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("class_index", ctypes.c_int32), ("hold", ctypes.c_int32), ("n_envs", ctypes.c_int64),
                ("horizon", ctypes.c_int32), ("keep", ctypes.c_int32), ("session", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("arrival", ctypes.c_double), ("actions", ctypes.c_void_p),
                ("action_rows", ctypes.c_int64)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("pad", ctypes.c_int32), ("session", ctypes.c_int64),
                ("steps_done", ctypes.c_int64), ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "cancelled", "queued", "active", "env_steps",
                                               "iterations", "bytes_in_use", "bytes_peak", "budget_bytes")] + \
               [(k, ctypes.c_double) for k in ("p50_latency", "p99_latency", "mean_latency", "wall")]


class EnvParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("mass", "added", "dlin", "dquad", "buoy", "current")]


class DrDist(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("relative", ctypes.c_int32), ("shared", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("mean", ctypes.c_double),
                ("std", ctypes.c_double), ("edges", ctypes.c_double * 9), ("weights", ctypes.c_double * 8)]


class DrSpec(ctypes.Structure):
    _fields_ = [(k, DrDist) for k in ("mass", "added", "dlin", "dquad", "buoy", "current")]


DR_FIXED, DR_UNIFORM, DR_GAUSSIAN, DR_PIECEWISE = 0, 1, 2, 3


def dr_spec(groups: dict) -> DrSpec:
    """A DrSpec from {group: {kind, relative=1, shared=0, lo, hi, mean, std, edges, weights}}
    (groups left out are fixed at the nominal)."""
    s = DrSpec()
    for name, d in groups.items():
        g = getattr(s, name)
        g.kind = int(d["kind"])
        g.relative = int(d.get("relative", 1))
        g.shared = int(d.get("shared", 0))
        g.lo, g.hi = float(d.get("lo", 0.0)), float(d.get("hi", 0.0))
        g.mean, g.std = float(d.get("mean", 0.0)), float(d.get("std", 0.0))
        edges, weights = d.get("edges", []), d.get("weights", [])
        g.n_bins = len(weights)
        for k, v in enumerate(edges):
            g.edges[k] = float(v)
        for k, v in enumerate(weights):
            g.weights[k] = float(v)
    return s


class StationDesc(ctypes.Structure):
    _fields_ = [("target_box", ctypes.c_double), ("tilt0", ctypes.c_double), ("v0", ctypes.c_double),
                ("sigma_p", ctypes.c_double), ("w_att", ctypes.c_double), ("w_act", ctypes.c_double),
                ("d_max", ctypes.c_double), ("tilt_max", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("substeps", ctypes.c_int32)]


STATION_DEFAULTS = dict(target_box=2.0, tilt0=0.2, v0=0.1, sigma_p=0.5, w_att=0.5, w_act=0.01, d_max=5.0,
                        tilt_max=1.2, max_steps=500, substeps=1)


class Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64 * MAX_CLASSES),
                ("n_renorm64", ctypes.c_int64 * MAX_CLASSES),
                ("max_speed", ctypes.c_double * MAX_CLASSES), ("mean_speed", ctypes.c_double * MAX_CLASSES),
                ("max_rate", ctypes.c_double * MAX_CLASSES), ("mean_rate", ctypes.c_double * MAX_CLASSES),
                ("mean_kinetic", ctypes.c_double * MAX_CLASSES), ("max_qdrift", ctypes.c_double * MAX_CLASSES)]


P = ctypes.c_void_p
I32, I64, U32, U64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "mgx_build_hash": (ctypes.c_char_p, []),
    "mgx_diag_wave_times": (I32, [P, I64]),
    "mgx_diag_valu_probe": (I32, [I32, I64, I32, ctypes.POINTER(F64)]),
    "mgx_diag_launch_floor": (I32, [I64, I32, I32, ctypes.POINTER(F64)]),
    "mgx_status_string": (ctypes.c_char_p, [I32]),
    "mgx_last_error": (ctypes.c_size_t, [ctypes.c_char_p, ctypes.c_size_t]),
    "mgx_last_hip_error": (I32, []),
    "mgx_version": (I32, []),
    "mgx_device_count": (I32, [ctypes.POINTER(I32)]),
    "mgx_step_cost": (I32, [I32, U32, ctypes.POINTER(F64), ctypes.POINTER(F64)]),
    "mgx_vjp_cost": (I32, [I32, U32, ctypes.POINTER(F64), ctypes.POINTER(F64)]),
    "mgx_class_step_cost": (I32, [I32, U32, ctypes.POINTER(F64), ctypes.POINTER(F64)]),
    "mgx_class_define": (I32, [ctypes.POINTER(ClassDesc), ctypes.POINTER(I32)]),
    "mgx_batch_create": (I32, [ctypes.POINTER(BatchDesc), ctypes.POINTER(P)]),
    "mgx_batch_plan": (I32, [ctypes.POINTER(BatchDesc), ctypes.POINTER(Layout)]),
    "mgx_batch_destroy": (I32, [P]),
    "mgx_batch_layout": (I32, [P, ctypes.POINTER(Layout)]),
    "mgx_batch_set_params": (I32, [P, ctypes.POINTER(EnvParams), I32]),
    "mgx_batch_reset": (I32, [P, P, I64, P, U64]),
    "mgx_batch_resample": (I32, [P, ctypes.POINTER(DrSpec), P, P, I64, U64, U64]),
    "mgx_batch_get_params": (I32, [P, P, P, P, P, P, P]),
    "mgx_batch_step": (I32, [P, P, I64, I64, I32, I32, U32, P, P]),
    "mgx_batch_get_step": (I32, [P, ctypes.POINTER(I64)]),
    "mgx_batch_set_step": (I32, [P, I64]),
    "mgx_diag_set_device_step": (I32, [P, I64]),
    "mgx_batch_get_state": (I32, [P, P, I32]),
    "mgx_batch_set_state": (I32, [P, P, I32]),
    "mgx_batch_get_stats": (I32, [P, ctypes.POINTER(Stats)]),
    "mgx_batch_check": (I32, [P, ctypes.POINTER(I64)]),
    "mgx_batch_sync": (I32, [P]),
    "mgx_gen_actions": (I32, [P, P, I64, I64, U64]),
    "mgx_batch_get_shape": (I32, [P, ctypes.POINTER(LaunchShape)]),
    "mgx_batch_set_shape": (I32, [P, ctypes.POINTER(LaunchShape)]),
    "mgx_autotune": (I32, [P, P, I64, I64, I32, I32, ctypes.POINTER(LaunchShape)]),
    "mgx_autotune_save": (I32, [ctypes.c_char_p]),
    "mgx_autotune_load": (I32, [ctypes.c_char_p]),
    "mgx_rollout_forward": (I32, [P, P, I64, I64, I32, I32, I32, P]),
    "mgx_rollout_forward_static": (I32, [P, P, I64, I64, I32, I32, I32, P]),
    "mgx_rollout_backward": (I32, [P, P, P, P]),
    "mgx_host_step_vjp": (I32, [I32, U32, P, P, P, P, P, P, P, P, P]),
    "mgx_server_now": (ctypes.c_double, []),
    "mgx_server_create": (I32, [ctypes.POINTER(ServerDesc), ctypes.POINTER(P)]),
    "mgx_server_submit": (I32, [P, ctypes.POINTER(Request), ctypes.POINTER(I64)]),
    "mgx_server_poll": (I32, [P, I64, ctypes.POINTER(RequestStatus)]),
    "mgx_server_wait": (I32, [P, I64, F64, ctypes.POINTER(RequestStatus)]),
    "mgx_server_cancel": (I32, [P, I64]),
    "mgx_server_read_state": (I32, [P, I64, P, I64]),
    "mgx_server_release": (I32, [P, I64]),
    "mgx_server_stats_get": (I32, [P, ctypes.POINTER(ServerStats)]),
    "mgx_server_destroy": (I32, [P]),
    "mgx_graph_capture": (I32, [P, P, I64, I64, I32, I32, I32, U32, ctypes.POINTER(P)]),
    "mgx_graph_replay": (I32, [P]),
    "mgx_graph_destroy": (I32, [P]),
    "mgx_station_create": (I32, [P, ctypes.POINTER(StationDesc), ctypes.POINTER(P)]),
    "mgx_station_destroy": (I32, [P]),
    "mgx_station_reset": (I32, [P, U64, P]),
    "mgx_station_step": (I32, [P, P, I32, P, P, P, P, P]),
    "mgx_station_episodes": (I32, [P, P, P]),
    "mgx_station_resample": (I32, [P, ctypes.POINTER(DrSpec), P, U64]),
}

_lib = None


def check_build(L, root=None):
    """Raise ImportError unless the loaded library ``L`` was compiled from the sources under
    ``root`` (default: this tree), compared by ``mgx_build_hash``."""
    from . import build as _build
    want = _build.source_hash(root or _build.ROOT)
    got = L.mgx_build_hash().decode()
    if got != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (library {got}, tree {want}): "
                          "rebuild it with paper_2503_09203_amd.build.build()")


def lib():
    """Load libmgx.so (built in-tree by ``build()``); raise if it is missing or was built
    from sources other than the ones beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_09203_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.mgx_build_hash.restype = ctypes.c_char_p
        L.mgx_build_hash.argtypes = []
        check_build(L)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    lib().mgx_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def check(status, where):
    if status != MGX_OK:
        raise MgxError(status, where, last_error())
    return status


def _call(name, *args):
    return check(getattr(lib(), name)(*args), name)


# ----------------------------------------------------------------------------- C names

def mgx_version():
    return lib().mgx_version()


def mgx_diag_valu_probe(chains, n_threads, iters):
    t = F64()
    _call("mgx_diag_valu_probe", int(chains), int(n_threads), int(iters), ctypes.byref(t))
    return t.value


def mgx_diag_launch_floor(n_threads, block, launches):
    t = F64()
    _call("mgx_diag_launch_floor", int(n_threads), int(block), int(launches), ctypes.byref(t))
    return t.value


def mgx_build_hash() -> str:
    return lib().mgx_build_hash().decode()


def mgx_device_count():
    n = I32()
    _call("mgx_device_count", ctypes.byref(n))
    return n.value


def mgx_step_cost(m, flags=0):
    f, o = F64(), F64()
    _call("mgx_step_cost", int(m), int(flags), ctypes.byref(f), ctypes.byref(o))
    return f.value, o.value


def mgx_vjp_cost(m, flags=0):
    f, o = F64(), F64()
    _call("mgx_vjp_cost", int(m), int(flags), ctypes.byref(f), ctypes.byref(o))
    return f.value, o.value


def mgx_class_step_cost(class_id, flags=0):
    f, o = F64(), F64()
    _call("mgx_class_step_cost", int(class_id), int(flags), ctypes.byref(f), ctypes.byref(o))
    return f.value, o.value


def mgx_class_define(cls) -> int:
    """Register a vehicle class given any object with m, r, e, k, tau, deadzone,
    inertia, rb, g0 attributes and optional k_rev, reaction (e.g. a ``synth.VehicleClass``)."""
    d = ClassDesc()
    d.m = int(cls.m)
    for i in range(cls.m):
        for j in range(3):
            d.r[i][j] = float(cls.r[i][j])
            d.e[i][j] = float(cls.e[i][j])
        d.k[i] = float(cls.k[i])
        d.tau[i] = float(cls.tau[i])
        d.deadzone[i] = float(cls.deadzone[i])
    k_rev, reaction = getattr(cls, "k_rev", None), getattr(cls, "reaction", None)
    for i in range(cls.m):
        d.k_rev[i] = 0.0 if k_rev is None else float(k_rev[i])
        d.reaction[i] = 0.0 if reaction is None else float(reaction[i])
    if getattr(cls, "kind", None) is not None:
        for i in range(cls.m):
            d.kind[i] = int(cls.kind[i])
            for j in range(3):
                d.span[i][j] = float(cls.span[i][j])
            d.fin_max[i] = float(cls.fin_max[i])
            d.fin_lift[i] = float(cls.fin_lift[i])
            d.fin_drag0[i] = float(cls.fin_drag0[i])
            d.fin_drag[i] = float(cls.fin_drag[i])
    rg = getattr(cls, "rg", None)
    for j in range(3):
        d.inertia[j] = float(cls.inertia[j])
        d.rb[j] = float(cls.rb[j])
        d.rg[j] = 0.0 if rg is None else float(rg[j])
    d.g0 = float(cls.g0)
    cid = I32()
    _call("mgx_class_define", ctypes.byref(d), ctypes.byref(cid))
    return cid.value


class TorchAllocator:
    """Device allocator of a batch backed by torch's caching allocator on one stream; keeps
    the C callbacks alive for as long as the object lives (the batch's lifetime at least)."""

    def __init__(self, device, stream):
        self.device, self.stream = device, stream
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                ptr = _torch().cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None
            self.live[int(ptr)] = int(nbytes)
            return int(ptr)

        def _free(ptr, ctx):
            if ptr and self.live.pop(int(ptr), None) is not None:
                _torch().cuda.caching_allocator_delete(int(ptr))

        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)


def _batch_desc(class_ids, n_envs, dt, precision, flags, device, stream, state=0, record=0, allocator=None):
    n = len(class_ids)
    ids = (I32 * n)(*class_ids)
    ns = (I64 * n)(*n_envs)
    d = BatchDesc(n, precision, ids, ns, float(dt), int(flags), int(device), ctypes.c_void_p(int(stream)),
                  ctypes.c_void_p(int(state)), ctypes.c_void_p(int(record)),
                  allocator.alloc_fn if allocator else ALLOC_FN(), allocator.free_fn if allocator else FREE_FN(),
                  None)
    return d, (ids, ns)


def mgx_batch_plan(class_ids, n_envs, dt, precision=FP32, flags=0) -> Layout:
    d, keep = _batch_desc(class_ids, n_envs, dt, precision, flags, -1, 0)
    L = Layout()
    _call("mgx_batch_plan", ctypes.byref(d), ctypes.byref(L))
    return L


def mgx_batch_create(class_ids, n_envs, dt, precision=FP32, flags=0, device=-1, stream=0, state=0, record=0,
                     allocator=None):
    d, keep = _batch_desc(class_ids, n_envs, dt, precision, flags, device, stream, state, record, allocator)
    h = P()
    _call("mgx_batch_create", ctypes.byref(d), ctypes.byref(h))
    return h


def mgx_batch_destroy(h):
    _call("mgx_batch_destroy", h)


def mgx_batch_layout(h) -> Layout:
    L = Layout()
    _call("mgx_batch_layout", h, ctypes.byref(L))
    return L


def mgx_batch_set_params(h, ptrs: dict, on_device: int):
    p = EnvParams(*(ctypes.c_void_p(int(ptrs[k])) for k in ("mass", "added", "dlin", "dquad", "buoy", "current")))
    _call("mgx_batch_set_params", h, ctypes.byref(p), int(on_device))


def mgx_batch_reset(h, env_ids_ptr, n, init_state_ptr, seed):
    _call("mgx_batch_reset", h, env_ids_ptr, int(n), init_state_ptr, int(seed))


def mgx_batch_step(h, actions_ptr, n_rows, row0, hold, K, flags=0, traj_ptr=None, forces_ptr=None):
    _call("mgx_batch_step", h, actions_ptr, int(n_rows), int(row0), int(hold), int(K), int(flags),
          traj_ptr, forces_ptr)


def mgx_batch_get_step(h):
    t = I64()
    _call("mgx_batch_get_step", h, ctypes.byref(t))
    return t.value


def mgx_batch_set_step(h, t):
    _call("mgx_batch_set_step", h, int(t))


def mgx_diag_set_device_step(h, t):
    _call("mgx_diag_set_device_step", h, int(t))


def mgx_batch_get_state(h, out_ptr, to_host):
    _call("mgx_batch_get_state", h, out_ptr, int(to_host))


def mgx_batch_set_state(h, in_ptr, from_host):
    _call("mgx_batch_set_state", h, in_ptr, int(from_host))


def mgx_batch_get_stats(h) -> Stats:
    s = Stats()
    _call("mgx_batch_get_stats", h, ctypes.byref(s))
    return s


def mgx_batch_check(h):
    """Returns (status, n_nonfinite) without raising on the statuses the check reports
    (MGX_E_NONFINITE, MGX_E_INVALID, MGX_E_NOT_SPD)."""
    n = I64()
    st = lib().mgx_batch_check(h, ctypes.byref(n))
    if st not in (MGX_OK, MGX_E_NONFINITE, MGX_E_INVALID, MGX_E_NOT_SPD):
        check(st, "mgx_batch_check")
    return st, n.value


def mgx_batch_sync(h):
    _call("mgx_batch_sync", h)


def mgx_gen_actions(h, out_ptr, rows, row_offset, seed):
    _call("mgx_gen_actions", h, out_ptr, int(rows), int(row_offset), int(seed))


def mgx_batch_get_shape(h) -> LaunchShape:
    s = LaunchShape()
    _call("mgx_batch_get_shape", h, ctypes.byref(s))
    return s


def mgx_batch_set_shape(h, mode, K, block=256, grid_per_cu=2):
    s = LaunchShape(int(mode), int(K), int(block), int(grid_per_cu), 0.0, 0, 0)
    _call("mgx_batch_set_shape", h, ctypes.byref(s))


def mgx_autotune(h, actions_ptr, n_rows, row0, hold, chunk) -> LaunchShape:
    s = LaunchShape()
    _call("mgx_autotune", h, actions_ptr, int(n_rows), int(row0), int(hold), int(chunk), ctypes.byref(s))
    return s


def mgx_autotune_save(path):
    _call("mgx_autotune_save", str(path).encode())


def mgx_autotune_load(path):
    _call("mgx_autotune_load", str(path).encode())


def mgx_rollout_forward(h, actions_ptr, n_rows, row0, hold, H, ckpt_every, pos_ptr):
    _call("mgx_rollout_forward", h, actions_ptr, int(n_rows), int(row0), int(hold), int(H), int(ckpt_every), pos_ptr)


def mgx_rollout_forward_static(h, actions_ptr, n_rows, row0, hold, H, ckpt_every, pos_ptr):
    _call("mgx_rollout_forward_static", h, actions_ptr, int(n_rows), int(row0), int(hold), int(H), int(ckpt_every),
          pos_ptr)


def mgx_rollout_backward(h, dpos_ptr, dactions_ptr, dparams_ptr):
    _call("mgx_rollout_backward", h, dpos_ptr, dactions_ptr, dparams_ptr)


def mgx_host_step_vjp(m, flags, cls, rec, state, actions, xbar):
    """Host evaluation of the step body and its adjoint (double); numpy in, numpy out."""
    f = lambda x: np.ascontiguousarray(x, dtype=np.float64)
    cls, rec, state, actions, xbar = f(cls), f(rec), f(state), f(actions), f(xbar)
    s_out, xb_out, ab, gp = np.zeros(13 + m), np.zeros(13 + m), np.zeros(m), np.zeros(24)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    _call("mgx_host_step_vjp", int(m), int(flags), p(cls), p(rec), p(state), p(actions), p(xbar), p(s_out),
          p(xb_out), p(ab), p(gp))
    return s_out, xb_out, ab, gp


def mgx_graph_capture(h, actions_ptr, n_rows, row0, hold, n_steps, K, flags=0):
    g = P()
    _call("mgx_graph_capture", h, actions_ptr, int(n_rows), int(row0), int(hold), int(n_steps), int(K), int(flags),
          ctypes.byref(g))
    return g


def mgx_graph_replay(g):
    _call("mgx_graph_replay", g)


def mgx_graph_destroy(g):
    _call("mgx_graph_destroy", g)


# ----------------------------------------------------------------------------- wrapper

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Batch:
    """Owns one batch. Device buffers are torch tensors on the batch's device; every call
    goes to the library on torch's current stream at creation (or the one given)."""

    def __init__(self, classes, n_envs, dt=0.01, precision=FP32, flags=0, device=0, stream=None, state=None,
                 record=None, torch_allocator=False):
        """``state`` / ``record``: optional contiguous tensors of the batch precision on its
        device, adopted in place (sizes from ``mgx_batch_plan``; they must outlive the batch).
        ``torch_allocator``: take every buffer the library allocates from torch's caching
        allocator instead of hipMalloc."""
        torch = _torch()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.class_ids = [mgx_class_define(c) for c in classes]
        self.precision = precision
        self.dtype = torch.float32 if precision == FP32 else torch.float64
        plan = mgx_batch_plan(self.class_ids, list(n_envs), dt, precision, flags)
        for name, t, need in (("state", state, plan.state_elems), ("record", record, plan.record_elems)):
            if t is not None and (t.dtype != self.dtype or t.device != self.device or not t.is_contiguous()
                                  or t.numel() < need):
                raise ValueError(f"{name}: need a contiguous {self.dtype} tensor of >= {need} elements on "
                                 f"{self.device}")
        self._adopted = (state, record)
        self._allocator = TorchAllocator(self.device, stream) if torch_allocator else None
        self.h = mgx_batch_create(self.class_ids, list(n_envs), dt, precision, flags, device,
                                  stream.cuda_stream, 0 if state is None else state.data_ptr(),
                                  0 if record is None else record.data_ptr(), self._allocator)
        self.layout = mgx_batch_layout(self.h)
        self.m = [self.layout.m[c] for c in range(len(classes))]
        self.n = [self.layout.n[c] for c in range(len(classes))]
        self.n_pad = [self.layout.n_pad[c] for c in range(len(classes))]

    # -- lifetime
    def close(self):
        for g in list(getattr(self, "_graphs", [])):
            g.close()
        for t in list(getattr(self, "_stations", [])):
            t.close()
        if getattr(self, "h", None):
            mgx_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers
    def empty_state(self):
        return _torch().zeros(self.layout.state_elems, dtype=self.dtype, device=self.device)

    def empty_actions(self, rows):
        return _torch().zeros((rows, self.layout.row_elems), dtype=self.dtype, device=self.device)

    # -- calls
    def set_params(self, params, on_device=True):
        """``params``: object with mass[N], added[6,N], dlin[6,N], dquad[6,N], buoy[N],
        current[3,N] (numpy, float64)."""
        torch = _torch()
        names = ("mass", "added", "dlin", "dquad", "buoy", "current")
        if on_device:
            self._param_tensors = {k: torch.as_tensor(np.ascontiguousarray(getattr(params, k), dtype=np.float64),
                                                      device=self.device) for k in names}
            ptrs = {k: v.data_ptr() for k, v in self._param_tensors.items()}
            mgx_batch_set_params(self.h, ptrs, 1)
        else:
            arrs = {k: np.ascontiguousarray(getattr(params, k), dtype=np.float64) for k in names}
            mgx_batch_set_params(self.h, {k: v.ctypes.data for k, v in arrs.items()}, 0)

    def reset(self, env_ids=None, init_state=None, seed=0):
        ids = None
        n = 0
        if env_ids is not None:
            ids = np.ascontiguousarray(env_ids, dtype=np.int64)
            n = len(ids)
        mgx_batch_reset(self.h, None if ids is None else ids.ctypes.data_as(ctypes.c_void_p), n,
                        _ptr(init_state), seed)

    def resample(self, groups, nominal, env_ids=None, seed=0, epoch=0):
        """Redraw parameters on the device (``groups`` as for ``dr_spec``, or a ``DrSpec`` it
        built; ``nominal``: [n_classes, 23] float64)."""
        spec = groups if isinstance(groups, DrSpec) else dr_spec(groups)
        nom = np.ascontiguousarray(nominal, dtype=np.float64).reshape(-1)
        ids = None if env_ids is None else np.ascontiguousarray(env_ids, dtype=np.int64)
        _call("mgx_batch_resample", self.h, ctypes.byref(spec), nom.ctypes.data_as(ctypes.c_void_p),
              None if ids is None else ids.ctypes.data_as(ctypes.c_void_p), 0 if ids is None else len(ids),
              int(seed), int(epoch))

    def get_params(self) -> dict:
        """Every environment's parameters as stored (float64 arrays, mgx_env_params layout)."""
        N = self.layout.n_total
        out = {"mass": np.zeros(N), "added": np.zeros((6, N)), "dlin": np.zeros((6, N)),
               "dquad": np.zeros((6, N)), "buoy": np.zeros(N), "current": np.zeros((3, N))}
        _call("mgx_batch_get_params", self.h,
              *[out[k].ctypes.data_as(ctypes.c_void_p) for k in ("mass", "added", "dlin", "dquad", "buoy", "current")])
        return out

    def step(self, actions, K, hold=1, row0=0, flags=0, traj=None, forces=None):
        mgx_batch_step(self.h, _ptr(actions), actions.shape[0], row0, hold, K, flags, _ptr(traj), _ptr(forces))

    def get_state(self):
        out = self.empty_state()
        mgx_batch_get_state(self.h, _ptr(out), 0)
        return out

    def set_state(self, t):
        assert t.numel() == self.layout.state_elems and t.dtype == self.dtype and t.is_contiguous()
        mgx_batch_set_state(self.h, _ptr(t), 0)

    def gen_actions(self, rows, row_offset=0, seed=0):
        out = self.empty_actions(rows)
        mgx_gen_actions(self.h, _ptr(out), rows, row_offset, seed)
        return out

    def capture(self, actions, n_steps, K, hold=1, row0=0, flags=0):
        """A replayable chunk of n_steps (launches of K steps); see ``Graph``."""
        g = Graph(self, actions, n_steps, K, hold, row0, flags)
        self.__dict__.setdefault("_graphs", []).append(g)
        return g

    def stats(self):
        return mgx_batch_get_stats(self.h)

    def shape(self):
        return mgx_batch_get_shape(self.h)

    def set_shape(self, mode, K, block=256, grid_per_cu=2):
        mgx_batch_set_shape(self.h, mode, K, block, grid_per_cu)

    def autotune(self, actions, chunk, hold=1, row0=0):
        return mgx_autotune(self.h, _ptr(actions), actions.shape[0], row0, hold, chunk)

    def check(self):
        return mgx_batch_check(self.h)

    def sync(self):
        mgx_batch_sync(self.h)

    @property
    def t(self):
        return mgx_batch_get_step(self.h)

    @t.setter
    def t(self, v):
        mgx_batch_set_step(self.h, v)

    # -- layout helpers (host side, numpy)
    def pack_state(self, states):
        """List of per-class stacked state arrays [13+m, n] -> flat layout array."""
        out = np.zeros(self.layout.state_elems)
        for c, s in enumerate(states):
            off, np_, m = self.layout.state_off[c], self.n_pad[c], self.m[c]
            seg = out[off:off + (STATE_FIXED + m) * np_].reshape(STATE_FIXED + m, np_)
            seg[:, :s.shape[1]] = s
            seg[3, s.shape[1]:] = 1.0
        return out

    def unpack_state(self, flat):
        """Flat layout -> list of per-class [13+m, n]."""
        out = []
        for c in range(len(self.m)):
            off, np_, m, n = self.layout.state_off[c], self.n_pad[c], self.m[c], self.n[c]
            out.append(flat[off:off + (STATE_FIXED + m) * np_].reshape(STATE_FIXED + m, np_)[:, :n])
        return out

    def pack_actions(self, per_class):
        """List of per-class [rows, m, n] -> [rows, row_elems]."""
        rows = per_class[0].shape[0]
        out = np.zeros((rows, self.layout.row_elems))
        for c, a in enumerate(per_class):
            off, np_, m = self.layout.action_off[c], self.n_pad[c], self.m[c]
            out[:, off:off + m * np_].reshape(rows, m, np_)[:, :, :a.shape[2]] = a
        return out

    def unpack_actions(self, flat):
        out = []
        for c in range(len(self.m)):
            off, np_, m, n = self.layout.action_off[c], self.n_pad[c], self.m[c], self.n[c]
            out.append(flat[:, off:off + m * np_].reshape(flat.shape[0], m, np_)[:, :, :n])
        return out

    def unpack_forces(self, flat):
        """[K, force_row_elems] -> list of per-class [K, 12, n]."""
        out = []
        for c in range(len(self.m)):
            off = int(self.layout.force_off[c])
            np_, n = self.n_pad[c], self.n[c]
            out.append(flat[:, off:off + FORCE_LEN * np_].reshape(flat.shape[0], FORCE_LEN, np_)[:, :, :n])
        return out


class Graph:
    """A captured chunk of step launches; ``replay()`` advances its batch by n_steps."""

    def __init__(self, batch, actions, n_steps, K, hold=1, row0=0, flags=0):
        self.batch = batch
        self.actions = actions  # keep the buffer alive as long as the graph
        self.n_steps = n_steps
        self.g = mgx_graph_capture(batch.h, _ptr(actions), actions.shape[0], row0, hold, n_steps, K, flags)

    def replay(self):
        mgx_graph_replay(self.g)

    def close(self):
        if getattr(self, "g", None):
            mgx_graph_destroy(self.g)
            self.g = None
            gs = self.batch.__dict__.get("_graphs", [])
            if self in gs:
                gs.remove(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- station keeping

class Station:
    """Station-keeping task on a batch (``mgx_station_*`` in include/mgx.h). Outputs are
    flat device tensors in the batch layout; ``VecStationKeeping`` gives the Gym-style view
    of a one-class batch. ``desc`` overrides fields of ``STATION_DEFAULTS``."""

    def __init__(self, batch, **desc):
        unknown = set(desc) - set(STATION_DEFAULTS)
        if unknown:
            raise TypeError(f"unknown station fields {sorted(unknown)}")
        self.batch = batch
        self.desc = dict(STATION_DEFAULTS, **desc)
        cd = StationDesc(**self.desc)
        h = P()
        _call("mgx_station_create", batch.h, ctypes.byref(cd), ctypes.byref(h))
        self.h = h
        batch.__dict__.setdefault("_stations", []).append(self)
        self.pad_off = [int(x) for x in np.concatenate([[0], np.cumsum(batch.n_pad)])[:-1]]

    def _check(self, t, n, dtype=None):
        b = self.batch
        assert t.device == b.device and t.is_contiguous() and t.numel() == n, "buffer shape/device"
        assert dtype is None or t.dtype == dtype, "buffer dtype"

    def empty_outputs(self, n_steps, final_obs=True):
        torch = _torch()
        b, L = self.batch, self.batch.layout
        out = {"obs": torch.zeros((n_steps, L.state_elems), dtype=b.dtype, device=b.device),
               "reward": torch.zeros((n_steps, L.n_pad_total), dtype=b.dtype, device=b.device),
               "terminated": torch.zeros((n_steps, L.n_pad_total), dtype=torch.uint8, device=b.device),
               "truncated": torch.zeros((n_steps, L.n_pad_total), dtype=torch.uint8, device=b.device)}
        if final_obs:
            out["final_obs"] = torch.zeros((n_steps, L.state_elems), dtype=b.dtype, device=b.device)
        return out

    def reset(self, seed, obs=None):
        """Episode 0 of every environment; returns the first observations (flat layout)."""
        if obs is None:
            obs = self.batch.empty_state()
        self._check(obs, self.batch.layout.state_elems, self.batch.dtype)
        _call("mgx_station_reset", self.h, int(seed), _ptr(obs))
        return obs

    def step(self, actions, out=None):
        """``actions``: [n_steps, row_elems] device tensor; one task step per row. Returns
        ``out`` (``empty_outputs(n_steps)`` if None), row k holding step k's results."""
        b, L = self.batch, self.batch.layout
        n = actions.shape[0]
        self._check(actions, n * L.row_elems, b.dtype)
        if out is None:
            out = self.empty_outputs(n)
        self._check(out["obs"], n * L.state_elems, b.dtype)
        self._check(out["reward"], n * L.n_pad_total, b.dtype)
        for k in ("terminated", "truncated"):
            self._check(out[k], n * L.n_pad_total)
            assert out[k].element_size() == 1, f"{k}: one byte per environment (uint8 or bool)"
        fo = out.get("final_obs")
        if fo is not None:
            self._check(fo, n * L.state_elems, b.dtype)
        _call("mgx_station_step", self.h, _ptr(actions), n, _ptr(out["obs"]), _ptr(out["reward"]),
              _ptr(out["terminated"]), _ptr(out["truncated"]), _ptr(fo))
        return out

    def resample(self, groups, nominal, seed=0):
        """Redraw the parameters of the environments whose episode started in the last reset or
        step call, epoch = their episode index (``groups`` as for ``dr_spec``, or a ``DrSpec``
        it built, which saves rebuilding it every step; ``nominal``: [n_classes, 23] float64)."""
        spec = groups if isinstance(groups, DrSpec) else dr_spec(groups)
        nom = np.ascontiguousarray(nominal, dtype=np.float64).reshape(-1)
        _call("mgx_station_resample", self.h, ctypes.byref(spec), nom.ctypes.data_as(ctypes.c_void_p), int(seed))

    def per_env(self, flat):
        """[..., n_pad_total] -> per class [..., n] (padding dropped)."""
        return [flat[..., o:o + n] for o, n in zip(self.pad_off, self.batch.n)]

    def episodes(self):
        """(episode index, steps taken in it) per global env id, numpy int32."""
        N = self.batch.layout.n_total
        ep, st = np.zeros(N, np.int32), np.zeros(N, np.int32)
        _call("mgx_station_episodes", self.h, ep.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p))
        return ep, st

    def close(self):
        if getattr(self, "h", None):
            _call("mgx_station_destroy", self.h)
            self.h = None
            ts = self.batch.__dict__.get("_stations", [])
            if self in ts:
                ts.remove(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VecStationKeeping:
    """Gym-style vector environment: ``n`` station-keeping environments of one vehicle class
    stepped together on the device. ``reset(seed)`` -> (obs [n, 13+m], {}); ``step(actions
    [n, m])`` -> (obs, reward [n], terminated [n] bool, truncated [n] bool,
    {"final_obs": [n, 13+m]}). Episodes that end restart in the same step; final_obs rows
    are meaningful where terminated or truncated is set (the pre-reset observation). Returned
    tensors are views of device buffers that the next call overwrites."""

    def __init__(self, cls, params, n, dt=0.01, precision=FP32, device=0, **desc):
        self.batch = Batch([cls], [n], dt, precision, device=device)
        self.batch.set_params(params)
        self.task = Station(self.batch, **desc)
        self.num_envs, self.m = n, cls.m
        self.single_observation_shape = (STATE_FIXED + cls.m,)
        self.single_action_shape = (cls.m,)
        self.action_low, self.action_high = -1.0, 1.0
        self._act = self.batch.empty_actions(1)
        self._out = self.task.empty_outputs(1)

    def _view(self, flat):
        return flat.view(-1, self.batch.n_pad[0])[:, :self.num_envs].t()

    def reset(self, seed=0):
        self.task.reset(seed, self._out["obs"][0])
        return self._view(self._out["obs"][0]), {}

    def step(self, actions):
        n = self.num_envs
        self._act[0].view(self.m, self.batch.n_pad[0])[:, :n].copy_(actions.t())
        o = self.task.step(self._act, self._out)
        return (self._view(o["obs"][0]), o["reward"][0, :n], o["terminated"][0, :n].bool(),
                o["truncated"][0, :n].bool(), {"final_obs": self._view(o["final_obs"][0])})

    def close(self):
        self.task.close()
        self.batch.close()


# ----------------------------------------------------------------------------- serving

def mgx_server_now():
    return lib().mgx_server_now()


class Server:
    """Continuous-batching server (see mgx_server_* in include/mgx.h). ``classes``: vehicle
    class objects; ``nominal``: per class an object with mass, added[6], dlin[6], dquad[6],
    buoy, current[3] (scalars / vectors)."""

    def __init__(self, classes, nominal, dt=0.01, budget_bytes=1 << 30, chunk_steps=0, max_active=4096,
                 fifo=False, batch_flags=0, device=-1, streams=0):
        ids = [mgx_class_define(c) for c in classes]
        self.m = [c.m for c in classes]
        nom = np.zeros((len(classes), 23))
        for i, p in enumerate(nominal):
            nom[i] = np.concatenate([[p["mass"]], p["added"], p["dlin"], p["dquad"], [p["buoy"]], p["current"]])
        self._ids = (I32 * len(ids))(*ids)
        self._nom = np.ascontiguousarray(nom)
        d = ServerDesc(len(ids), self._ids, self._nom.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt),
                       int(batch_flags), SERVE_FIFO if fifo else 0, int(budget_bytes), int(chunk_steps),
                       int(max_active), int(device), int(streams))
        h = P()
        _call("mgx_server_create", ctypes.byref(d), ctypes.byref(h))
        self.h = h

    def submit(self, class_index, n_envs, horizon, seed, hold=10, keep=False, session=-1, arrival=0.0,
               actions=None):
        """``actions``: optional float32 device tensor [rows][m][n_envs] of commands (kept
        alive by the caller until the request is done)."""
        r = Request(int(class_index), int(hold), int(n_envs), int(horizon), 1 if keep else 0, int(session), int(seed),
                    float(arrival), ctypes.c_void_p(actions.data_ptr() if actions is not None else 0),
                    int(actions.shape[0]) if actions is not None else 0)
        rid = I64()
        _call("mgx_server_submit", self.h, ctypes.byref(r), ctypes.byref(rid))
        return rid.value

    def poll(self, rid) -> RequestStatus:
        st = RequestStatus()
        _call("mgx_server_poll", self.h, int(rid), ctypes.byref(st))
        return st

    def wait(self, rid, timeout=60.0) -> RequestStatus:
        st = RequestStatus()
        _call("mgx_server_wait", self.h, int(rid), float(timeout), ctypes.byref(st))
        return st

    def cancel(self, rid):
        _call("mgx_server_cancel", self.h, int(rid))

    def read_state(self, session, class_index, n_envs):
        out = np.zeros((STATE_FIXED + self.m[class_index], n_envs), dtype=np.float32)
        _call("mgx_server_read_state", self.h, int(session), out.ctypes.data_as(ctypes.c_void_p), out.size)
        return out

    def release(self, session):
        _call("mgx_server_release", self.h, int(session))

    def stats(self) -> ServerStats:
        s = ServerStats()
        _call("mgx_server_stats_get", self.h, ctypes.byref(s))
        return s

    def close(self):
        if getattr(self, "h", None):
            _call("mgx_server_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
