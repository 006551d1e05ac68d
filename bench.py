#!/usr/bin/env python3
"""Throughput of the batched underwater-vehicle step on one MI355X.

Workload (default): one 6-thruster vehicle class, 65,536 environments with +-20%
per-environment randomisation of mass, added mass, damping and buoyancy and a constant
N(0, 0.3^2) m/s world current each, 1000 steps of dt = 0.01 s, actions resampled every 10
steps. One benchmark step = one pass of the whole path over that batch: per-parameter-set
setup (double precision, on the device), reset from a resident initial state, and the
1000-step rollout as 16-step fused launches replayed from a captured HIP graph. Inputs
(parameters, initial states, the action stream) are resident in HBM before timing.

Prints one JSON line: env-steps/s, the roofline of the fused step kernel (per-launch
duration from HIP events on the batch's stream), the single-step kernel's HBM roofline,
and the FP64 CPU oracle timed on this host on a bounded sample of the same workload,
whose final states also give the parity of this run.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP32 env-steps/s vs FP64 oracle at stated error; serving p50/p99 latency"
PEAK_FP32_VECTOR = 157.3e12   # MI355X published FP32 vector peak (FLOP/s)
PEAK_HBM = 8.0e12             # MI355X HBM3E (B/s)


def bytes_per_env_step(m, K, hold, prec=4, rec_len=30):
    """Algorithmic HBM bytes per environment-step of one launch of K steps: state read and
    written once, record read once, one action row per hold interval."""
    state = (13 + m) * prec
    rows = min(K, math.ceil(K / hold) + 1) if hold > 1 else K
    return (2 * state + rec_len * prec + rows * m * prec) / K


# Hardware byte counters cannot be read from inside this process; the per-launch HBM traffic
# of the step kernel comes from the committed rocprofv3 summary, and only while the kernel
# sources still hash to the value recorded with those counters (else null).
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_step_dr65536x1000.md")
KERNEL_SOURCES = ("step.hpp", "env_loop.hpp", "kernels.hip", "kernels.hpp", "step_kernel.hpp", "step_f32.hip")


def kernel_sources_sha256(files=KERNEL_SOURCES):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2503_09203_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_line(path, files):
    """The 'traffic:' line of a committed profile (the figures before '; sources'), if the
    sources it names hash to the value recorded with the counters, else None."""
    import re

    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"^traffic: (.*); sources sha256 ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(2) != kernel_sources_sha256(files):
        return None
    return m.group(1)


# Profiles of the other step bodies at the same sizes, by workload.
VARIANT_TRAFFIC_PROFILES = {
    "dr": TRAFFIC_PROFILE,
    "propellers": os.path.join(ROOT, "profiles", "k_step_prop65536x1000.md"),
    "rudders": os.path.join(ROOT, "profiles", "k_step_rudder65536x1000.md"),
    "payload": os.path.join(ROOT, "profiles", "k_step_payload65536x1000.md"),
}


def recorded_traffic(workload="dr"):
    """{K: bytes per launch} from the workload's step profile 'traffic:' line, if its source
    hash matches."""
    import re

    line = traffic_line(VARIANT_TRAFFIC_PROFILES[workload], KERNEL_SOURCES)
    return {int(k): float(v) for k, v in re.findall(r"K=(\d+) (\d+) B/launch", line or "")}


# The same for the differentiable rollout's forward and backward kernels and the
# station-keeping task's step kernel.
ADJOINT_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_rollout_adjoint8192x256.md")
ADJOINT_SOURCES = ("adjoint.hip", "adjoint.hpp", "step.hpp", "env_loop.hpp", "kernels.hpp")
STATION_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_station_step65536.md")
STATION_SOURCES = ("station.hip", "step.hpp", "env_loop.hpp", "kernels.hpp")


HETERO_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_persistent_hetero70512x1024.md")
HETERO_SOURCES = ("persistent.hip", "step.hpp", "env_loop.hpp", "kernels.hpp")


def recorded_hetero_traffic():
    """{K: bytes per launch} of the persistent launch over the five-class batch of 70,512
    environments, if the persistent sources hash to the recorded value."""
    import re

    line = traffic_line(HETERO_TRAFFIC_PROFILE, HETERO_SOURCES)
    return {int(k): float(v) for k, v in re.findall(r"K=(\d+) (\d+) B/launch", line or "")}


def recorded_adjoint_traffic():
    """{"fwd": bytes, "bwd": bytes} per launch at 8192 envs x 256 steps, if the adjoint
    sources hash to the recorded value."""
    import re

    line = traffic_line(ADJOINT_TRAFFIC_PROFILE, ADJOINT_SOURCES)
    return {k: float(v) for k, v in re.findall(r"(fwd|bwd) (\d+) B/launch", line or "")}


def recorded_station_traffic():
    """{K: bytes per launch} of the station step at 65,536 envs for calls of K task steps,
    if the station sources hash to the recorded value."""
    import re

    line = traffic_line(STATION_TRAFFIC_PROFILE, STATION_SOURCES)
    return {int(k): float(v) for k, v in re.findall(r"K=(\d+) (\d+) B/launch", line or "")}


def parity_errors(gpu, ref):
    """Per-component max_env |gpu - ref| / max(|ref|, rms of the component)."""
    rms = np.sqrt(np.mean(ref * ref, axis=1, keepdims=True))
    return np.max(np.abs(gpu - ref) / np.maximum(np.abs(ref), np.maximum(rms, 1e-30)), axis=1)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed benchmark steps (full rollouts)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=65536, help="environments")
    ap.add_argument("--rollout", type=int, default=1000, help="steps per rollout")
    ap.add_argument("--chunk", type=int, default=16, help="steps per fused launch (K)")
    ap.add_argument("--block", type=int, default=256, help="threads per block of the step launches (64, 128 or 256)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU-oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="dr",
                    choices=["dr", "plain", "propellers", "rudders", "payload", "hetero", "serve", "adjoint", "resample",
                             "station"],
                    help="dr: the default benchmark line; plain: the small plain workload (1024 environments at the "
                         "class nominal, 1000 steps) in FP64 and FP32 batches beside the oracle on the same inputs; propellers: the same line with dead zones, reverse "
                         "gains and shaft torques on every thruster; rudders: the same line for a rudder-propeller "
                         "class (one propeller, four tail fins); payload: the same line with the centre of gravity "
                         "off the body origin (full mass matrix); hetero: five classes in one persistent launch; "
                         "serve: Poisson request trace through the continuous-batching server and the FIFO baseline; "
                         "adjoint: checkpointed forward and reverse sweep of the differentiable rollout; "
                         "resample: on-device domain randomisation of every environment's parameters; "
                         "station: the station-keeping task step (step, observation, reward, termination and "
                         "auto-reset in one kernel)")
    ap.add_argument("--station-class", default="dr", choices=["dr", "heavy8"],
                    help="station: the randomised workload's 6-thruster class, or an 8-thruster class (the "
                         "paper's station-keeping speed test uses an 8-thruster vehicle)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: requests per second")
    ap.add_argument("--sweep-rates", default="", help="serve: extra comma-separated rates, 5 s each")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: trace length (s)")
    ap.add_argument("--serve-chunk", type=int, default=0, help="serve: steps per iteration (0: whole horizon)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy (negation) of this many MiB, read and written once, so that "
                         "hardware byte counters collected over this run can be scaled against a known size")
    ap.add_argument("--counter-launches", action="store_true",
                    help="instead of the benchmark line, run a fixed set of plain launches for hardware counter "
                         "passes: 4 of K = 16 and 2 of K = 1000 at the default N")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line, print launch-duration sweeps over K and N")
    ap.add_argument("--probe", action="store_true",
                    help="instead of the benchmark line, print the VALU issue-rate probe (float multiply-add chains "
                         "at 1, 2 and 4 waves per SIMD) and the launch floor (back-to-back launches that do nothing)")
    ap.add_argument("--wave-phases", action="store_true",
                    help="instead of the benchmark line, print the per-wave phase times of the step kernel "
                         "(needs the diagnostic build: python -m paper_2503_09203_amd.build --wave-timestamps, "
                         "then MGX_LIB=<repo>/paper_2503_09203_amd/libmgx_wavets.so)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); environments are independent, "
              "so more GPUs would each run their own shard of the batch with no exchange.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2503_09203_amd import mgx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    mgx.lib()  # fail loudly if the HIP library is missing

    N, T, K, HOLD = args.n, args.rollout, args.chunk, 10
    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.sweep:
        sweep(args)
        return
    if args.probe:
        probe(args)
        return
    if args.wave_phases:
        wave_phases(args)
        return
    if args.workload == "plain":
        plain(args)
        return
    if args.counter_launches:
        counter_launches(args)
        return
    if args.workload == "hetero":
        hetero(args)
        return
    if args.workload == "serve":
        serve(args)
        return
    if args.workload == "adjoint":
        adjoint(args)
        return
    if args.workload == "resample":
        resample(args)
        return
    if args.workload == "station":
        station(args)
        return
    variant = args.workload  # dr, propellers or rudders
    make = {"dr": synth.randomised, "propellers": synth.propellers, "rudders": synth.rudders,
            "payload": synth.payload}[variant]
    w = make(n=N, steps=T)
    cls = w.classes[0]
    shaped = variant != "dr"
    # the remaining template arguments of k_step: fins, payload
    tmpl_tail = f"{str(variant == 'rudders').lower()},{str(variant == 'payload').lower()}"
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    b = mgx.Batch([cls], [N], w.dt, mgx.FP32)
    if args.block != 256:
        b.set_shape(mgx.LAUNCH_PER_CLASS, K, block=args.block)
    b.set_params(w.params, on_device=True)
    param_ptrs = {k: v.data_ptr() for k, v in b._param_tensors.items()}
    init = torch.tensor(b.pack_state([w.state[0].stacked()]), dtype=torch.float32, device=dev)
    rows = -(-T // HOLD)
    acts = b.gen_actions(rows, seed=synth.MASTER_SEED)
    graph = b.capture(acts, T, K, hold=HOLD)

    n_launch = -(-T // K)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def bench_step(i=None):
        mgx.mgx_batch_set_params(b.h, param_ptrs, 2)   # device arrays known valid: no host wait
        b.reset(init_state=init)
        b.t = 0
        if i is not None:
            ev[i][0].record(stream)
        graph.replay()
        if i is not None:
            ev[i][1].record(stream)

    for _ in range(args.warmup):
        bench_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bench_step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    final_state = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))[0]
    value = N * T * args.steps / elapsed

    # Fused kernel: HIP events on the batch's stream around every graph replay (the
    # rollout's n_launch kernel launches back to back); average launch duration =
    # elapsed / n_launch, so inter-kernel gaps count against the kernel.
    flops_es, ops_es = mgx.mgx_class_step_cost(mgx.mgx_class_define(cls))
    graph_s = np.array([a.elapsed_time(c) for a, c in ev]) * 1e-3
    fused_launch = float(graph_s.mean()) / n_launch
    fused_flops_per_launch = flops_es * N * T / n_launch

    # The same rollout as T single-step launches (graph-captured), timed the same way. The
    # capture is taken at step 0, the step every replay starts from, so each launch's
    # expected action row is the right one (replays from other steps fetch it after the
    # device counter instead).
    b.t = 0
    g1 = b.capture(acts, T, 1, hold=HOLD, flags=mgx.STEP_UNFUSED)
    reps1 = max(3, args.steps // 10)
    ev1 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps1 + 1)]
    t1 = None
    for i in range(reps1 + 1):
        if i == 1:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        b.reset(init_state=init)
        b.t = 0
        ev1[i][0].record(stream)
        g1.replay()
        ev1[i][1].record(stream)
    torch.cuda.synchronize()
    single_rate = N * T * reps1 / (time.perf_counter() - t1)
    per_replay = np.array([a.elapsed_time(c) for a, c in ev1[1:]]) * 1e-3 / T   # s per launch, per replay
    single_launch = float(per_replay.mean())
    single_launch_median = float(np.median(per_replay))
    rec_len = 45 if variant == "payload" else 30
    single_bytes = bytes_per_env_step(cls.m, 1, HOLD, rec_len=rec_len) * N
    traffic = recorded_traffic(variant) if (N, T, HOLD) == (65536, 1000, 10) else {}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{ {'dr': 'dr', 'propellers': 'prop', 'rudders': 'rudder', 'payload': 'payload'}[variant] }_{N}x{T}", "n_envs": N, "rollout_steps": T, "thrusters": cls.m, "hold": HOLD,
                   "launch_steps_K": K, "dt": w.dt, "current_sigma": 0.3, "randomisation": 0.2,
                   "path": "set_params + reset + graph of fused launches"},
        "roofline": {"bound": "alu", "achieved": fused_flops_per_launch / fused_launch / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": fused_flops_per_launch / fused_launch / PEAK_FP32_VECTOR, "traffic": traffic.get(K),
                     "traffic_unit": "B/launch",
                     "kernel": f"k_step<float,{cls.m},false,false,{str(shaped).lower()},{tmpl_tail}> K={K}", "launches_per_step": n_launch,
                     "launch_us_mean": fused_launch * 1e6, "flops_per_env_step": flops_es,
                     "valu_ops_per_env_step": ops_es},
        "single_step": {"env_steps_per_s": single_rate, "kernel": f"k_step<float,{cls.m},false,true,{str(shaped).lower()},{tmpl_tail}> K=1",
                        "launch_us_mean": single_launch * 1e6,
                        "launch_us_median_of_replays": single_launch_median * 1e6, "replays": int(len(per_replay)),
                        "roofline": {"bound": "hbm", "achieved": single_bytes / single_launch / 1e9,
                                     "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                     "frac": single_bytes / single_launch / PEAK_HBM,
                                     "bytes_per_env_step": bytes_per_env_step(cls.m, 1, HOLD, rec_len=rec_len),
                                     "traffic": traffic.get(1), "traffic_unit": "B/launch"}},
    }

    if not args.no_cpu_baseline:
        import oracle  # CPU baseline leg only

        envs_all = oracle.make_envs(cls, w.params, w.dt)
        st0 = w.state[0]
        full_state = oracle.pack_state(st0.p, st0.q, st0.nu, st0.n)
        a_host = synth.actions(N, cls.m, rows)
        # calibrate on 256 environments, then size the sample to the time target
        cal = np.arange(256)
        tc = time.perf_counter()
        oracle.rollout(envs_all[cal], full_state[cal].copy(), oracle.pack_actions(a_host[:, :, cal]), HOLD, T)
        rate_cal = 256 * T / (time.perf_counter() - tc)
        n_s = int(min(N, max(256, rate_cal * args.cpu_seconds / T)))
        idx = np.linspace(0, N - 1, n_s).round().astype(np.int64)
        acts_s = oracle.pack_actions(a_host[:, :, idx])
        st_s = full_state[idx].copy()
        tc = time.perf_counter()
        st_s, _, _ = oracle.rollout(envs_all[idx], st_s, acts_s, HOLD, T)
        cpu_elapsed = time.perf_counter() - tc
        ref = oracle.unpack_state(st_s, cls.m)
        err = parity_errors(final_state[:, idx], ref)
        # the same oracle on one thread, over the first 256 of the sample
        threads = oracle.get_threads()
        oracle.set_threads(1)
        t1 = time.perf_counter()
        oracle.rollout(envs_all[idx[:256]], full_state[idx[:256]].copy(), oracle.pack_actions(a_host[:, :, idx[:256]]),
                       HOLD, T)
        rate_1 = 256 * T / (time.perf_counter() - t1)
        oracle.set_threads(threads)
        out["cpu_baseline"] = {"value": n_s * T / cpu_elapsed, "unit": "env-steps/s", "cores": threads,
                               "kind": "oracle", "value_one_thread": rate_1,
                               "sample": f"{n_s} of {N} environments (evenly spaced ids) x {T} steps, FP64 C oracle, "
                                         f"OpenMP over environments, {cpu_elapsed:.1f} s; one thread: 256 of them"}
        tol = 1e-3
        out["parity"] = {"metric": "max over envs |gpu - oracle| / max(|oracle|, rms), per state component",
                         "step": T, "max_err": float(err.max()), "tolerance": tol, "pass": bool(err.max() <= tol),
                         "envs_checked": n_s}

    g1.close()
    graph.close()
    b.close()
    print(json.dumps(out), flush=True)


def plain(args):
    """The small plain workload: one 6-thruster class, 1024 environments at the class
    nominal, no current, 1000 steps, actions resampled every 10 steps. The rollout runs as
    one captured graph of 16-step launches, in an FP64 batch (the configuration's precision)
    and an FP32 one; every environment's final state is checked against the FP64 oracle,
    which is timed on the same inputs at one thread and at all threads."""
    import torch

    import oracle  # CPU baseline and parity leg
    import synth
    from paper_2503_09203_amd import mgx

    N, T, K, HOLD = 1024, 1000, 16, 10
    w = synth.plain_small(n=N, steps=T)
    cls = w.classes[0]
    rows = -(-T // HOLD)
    stream = torch.cuda.current_stream()
    out = {"metric": METRIC, "workload": f"plain_small_{N}x{T}", "unit": "env-steps/s", "n_envs": N,
           "rollout_steps": T, "launch_steps_K": K, "hold": HOLD, "thrusters": cls.m}
    envs = oracle.make_envs(cls, w.params, w.dt)
    x0 = oracle.pack_state(w.state[0].p, w.state[0].q, w.state[0].nu, w.state[0].n)
    a_host = oracle.pack_actions(synth.actions(N, cls.m, rows))
    for prec, name in ((mgx.FP64, "f64"), (mgx.FP32, "f32")):
        b = mgx.Batch([cls], [N], w.dt, prec)
        b.set_params(w.params)
        init = torch.tensor(b.pack_state([w.state[0].stacked()]), dtype=b.dtype, device="cuda:0")
        acts = b.gen_actions(rows, seed=synth.MASTER_SEED)
        g = b.capture(acts, T, K, hold=HOLD)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for i in range(args.warmup + args.steps):
            b.reset(init_state=init)
            b.t = 0
            if i >= args.warmup:
                ev[i - args.warmup][0].record(stream)
            g.replay()
            if i >= args.warmup:
                ev[i - args.warmup][1].record(stream)
        torch.cuda.synchronize()
        sec = float(np.mean([a.elapsed_time(c) for a, c in ev])) * 1e-3
        final = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))[0]
        g.close()
        b.close()
        ref, _, _ = oracle.rollout(envs, x0.copy(), a_host, HOLD, T)
        err = parity_errors(final, oracle.unpack_state(ref, cls.m))
        out[name] = {"ms_per_rollout": sec * 1e3, "env_steps_per_s": N * T / sec, "launch_us_mean": sec / -(-T // K) * 1e6,
                     "parity_max_err": float(err.max()), "tolerance": 1e-9 if prec == mgx.FP64 else 1e-3,
                     "pass": bool(err.max() <= (1e-9 if prec == mgx.FP64 else 1e-3)), "envs_checked": N}
    threads = oracle.get_threads()
    rates = {}
    for nt in (1, threads):
        oracle.set_threads(nt)
        tc = time.perf_counter()
        oracle.rollout(envs, x0.copy(), a_host, HOLD, T)
        rates[nt] = N * T / (time.perf_counter() - tc)
    oracle.set_threads(threads)
    out["value"] = out["f64"]["env_steps_per_s"]
    out["dtype"] = "f64"
    out["cpu_baseline"] = {"value": rates[threads], "unit": "env-steps/s", "cores": threads, "kind": "oracle",
                           "value_one_thread": rates[1],
                           "sample": f"all {N} environments x {T} steps, FP64 C oracle (OpenMP over environments)"}
    out["note"] = "16 waves on 1024 SIMDs: launch-latency bound (63 launches per rollout)"
    print(json.dumps(out), flush=True)


def probe(args):
    """VALU issue rate of plain float multiply-add chains at 1, 2 and 4 waves per SIMD, and
    the launch floor of kernels that do nothing (library diagnostics)."""
    from paper_2503_09203_amd import mgx

    simds, clock = 1024, 2.4e9
    iters = 2048
    for waves_per_simd in (1, 2, 4):
        n = simds * 64 * waves_per_simd
        for chains in (1, 2, 4, 8):
            sec = mgx.mgx_diag_valu_probe(chains, n, iters)
            wave_instr = n / 64 * 16 * iters * chains
            print(json.dumps({"probe": "valu", "chains": chains, "threads": n, "waves_per_simd": waves_per_simd,
                              "seconds": sec, "lane_fma_per_s": n * 16 * iters * chains / sec,
                              "tflops": 2 * n * 16 * iters * chains / sec / 1e12,
                              "cycles_per_wave_instr_per_simd": sec * clock / (wave_instr / simds)}), flush=True)
    for n, block in ((65536, 256), (65536, 64), (262144, 256), (4096, 256)):
        sec = mgx.mgx_diag_launch_floor(n, block, 1000)
        print(json.dumps({"probe": "launch_floor", "threads": n, "block": block, "us_per_launch": sec * 1e6}),
              flush=True)


def wave_phases(args):
    """Per-wave phase times of the step kernel (entry, prologue loads landed, steps done,
    stores drained) on the randomised workload, for K = 16 and K = 1, read after a run of
    back-to-back launches (the last launch's waves)."""
    import ctypes

    import torch

    import synth
    from paper_2503_09203_amd import mgx

    probe_buf = np.zeros((1, 4), dtype=np.uint64)
    if mgx.lib().mgx_diag_wave_times(probe_buf.ctypes.data_as(ctypes.c_void_p), 1) != mgx.MGX_OK:
        print("the loaded library records no wave times: build python -m paper_2503_09203_amd.build "
              "--wave-timestamps and set MGX_LIB to the built libmgx_wavets.so", file=sys.stderr)
        sys.exit(1)
    N, HOLD = args.n, 10
    w = synth.randomised(n=N, steps=1000)
    cls = w.classes[0]
    b = mgx.Batch([cls], [N], w.dt)
    b.set_params(w.params)
    init = torch.tensor(b.pack_state([w.state[0].stacked()]), dtype=torch.float32, device="cuda:0")
    acts = b.gen_actions(101, seed=synth.MASTER_SEED)
    nw = b.layout.n_pad_total // 64
    stream = torch.cuda.current_stream()
    for K, launches in ((16, 62), (1, 500)):
        b.reset(init_state=init)
        b.t = 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(launches):
            b.step(acts, K, hold=HOLD)
        e1.record(stream)
        torch.cuda.synchronize()
        buf = np.zeros((nw, 4), dtype=np.uint64)
        mgx._call("mgx_diag_wave_times", buf.ctypes.data_as(ctypes.c_void_p), nw)
        t = (buf - buf[:, 0].min()).astype(np.int64) * 10  # 100 MHz counter -> ns
        q = lambda x: {"p10": float(np.percentile(x, 10)), "p50": float(np.median(x)), "max": float(x.max())}
        print(json.dumps({"wave_phases": True, "n": N, "K": K, "waves": nw,
                          "launch_us_mean": e0.elapsed_time(e1) * 1e3 / launches,
                          "entry_ns": q(t[:, 0]), "loads_ns": q(t[:, 1] - t[:, 0]), "steps_ns": q(t[:, 2] - t[:, 1]),
                          "stores_ns": q(t[:, 3] - t[:, 2]), "end_ns": q(t[:, 3])}), flush=True)
    b.close()


def hetero(args):
    """Five vehicle classes (4, 5, 6, 8, 8 thrusters; 512 / 3000 / 20000 / 40000 / 7000
    envs) advanced 1024 steps as 32 captured 32-step chunks, launch shape from the
    autotuner, against the same chunks as one launch per class (K = 16)."""
    import torch

    import synth
    from paper_2503_09203_amd import mgx

    T, CHUNK, HOLD = 1024, 32, 10
    w = synth.heterogeneous(steps=T)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    b.set_params(w.params)
    init = torch.tensor(b.pack_state([s.stacked() for s in w.state]), dtype=torch.float32, device="cuda:0")
    b.set_state(init)
    acts = b.gen_actions(-(-T // HOLD) + 1, seed=synth.MASTER_SEED)
    stream = torch.cuda.current_stream()
    n = w.n_total
    flops = sum(mgx.mgx_step_cost(c.m)[0] * k for c, k in zip(w.classes, w.n_envs))

    def run(label):
        g = b.capture(acts, CHUNK, 0, hold=HOLD)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for i in range(args.warmup + args.steps):
            b.reset(init_state=init)
            b.t = 0
            if i >= args.warmup:
                ev[i - args.warmup][0].record(stream)
            for _ in range(T // CHUNK):
                g.replay()
            if i >= args.warmup:
                ev[i - args.warmup][1].record(stream)
        torch.cuda.synchronize()
        sec = float(np.mean([a.elapsed_time(c) for a, c in ev])) * 1e-3
        g.close()
        sh = b.shape()
        return {"label": label, "mode": "persistent" if sh.mode == mgx.LAUNCH_PERSISTENT else "per_class",
                "K": sh.K, "block": sh.block, "grid_per_cu": sh.grid_per_cu, "ms_per_rollout": sec * 1e3,
                "env_steps_per_s": n * T / sec, "tflops": flops * T / sec / 1e12}

    def run_rollout_graph(label):
        """The same rollout as one graph holding all T / CHUNK chunks (no host graph launch
        between chunks)."""
        g = b.capture(acts, T, 0, hold=HOLD)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for i in range(args.warmup + args.steps):
            b.reset(init_state=init)
            b.t = 0
            if i >= args.warmup:
                ev[i - args.warmup][0].record(stream)
            g.replay()
            if i >= args.warmup:
                ev[i - args.warmup][1].record(stream)
        torch.cuda.synchronize()
        sec = float(np.mean([a.elapsed_time(c) for a, c in ev])) * 1e-3
        g.close()
        return {"label": label, "ms_per_rollout": sec * 1e3, "env_steps_per_s": n * T / sec,
                "tflops": flops * T / sec / 1e12}

    b.set_shape(mgx.LAUNCH_PER_CLASS, 16)
    base = run("per-class launches, K=16")
    b.reset(init_state=init)
    b.t = 0
    tuned = b.autotune(acts, CHUNK, hold=HOLD)
    best = run("autotuned")
    whole = run_rollout_graph("autotuned, all chunks in one graph")
    final = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))
    out = {"metric": METRIC, "workload": f"hetero_{n}x{T}", "value": best["env_steps_per_s"], "unit": "env-steps/s",
           "n_envs": n, "classes": [c.m for c in w.classes], "n_per_class": w.n_envs, "chunk_steps": CHUNK,
           "autotune": {"candidates": tuned.candidates, "us_per_chunk": tuned.us_per_chunk}, "tuned": best,
           "tuned_rollout_graph": whole, "baseline": base,
           "speedup_vs_per_class": best["env_steps_per_s"] / base["env_steps_per_s"]}
    # Launches per chunk of the tuned shape: one persistent launch of K steps, or one launch
    # per class of K steps, CHUNK / K times.
    per_chunk = (CHUNK // best["K"]) * (1 if best["mode"] == "persistent" else len(w.classes))
    launch_us = best["ms_per_rollout"] * 1e3 / (T // CHUNK) / per_chunk
    out["roofline"] = {"bound": "alu", "kernel": "k_persistent<float>" if best["mode"] == "persistent" else "k_step (per class)",
                       "achieved": best["tflops"], "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                       "frac": best["tflops"] * 1e12 / PEAK_FP32_VECTOR,
                       "traffic": (recorded_hetero_traffic().get(best["K"]) if best["mode"] == "persistent" else None),
                       "traffic_unit": "B/launch",
                       "launches_per_chunk": per_chunk, "us_per_launch_with_gaps": launch_us,
                       "flops_per_env_step": flops / n}
    if not args.no_cpu_baseline:
        # the FP64 oracle per class on a bounded sample of that class's environments (the
        # last rollout's inputs), which also gives each class's parity after T steps
        import oracle  # CPU baseline leg only

        threads = oracle.get_threads()
        per_class, off = [], 0
        for c, nc, st in zip(w.classes, w.n_envs, w.state):
            idx = np.linspace(0, nc - 1, min(nc, 2048)).round().astype(np.int64)
            envs = oracle.make_envs(c, w.params.subset(off + idx), w.dt)
            x = oracle.pack_state(st.p[:, idx], st.q[:, idx], st.nu[:, idx], st.n[:, idx])
            a = oracle.pack_actions(synth.actions(nc, c.m, -(-T // HOLD) + 1, env_offset=off)[:, :, idx])
            tc = time.perf_counter()
            x, _, _ = oracle.rollout(envs, x, a, HOLD, T)
            sec = time.perf_counter() - tc
            err = parity_errors(final[len(per_class)][:, idx], oracle.unpack_state(x, c.m))
            per_class.append({"m": c.m, "n": nc, "sample": len(idx), "env_steps_per_s": len(idx) * T / sec,
                              "parity_max_err": float(err.max())})
            off += nc
        total = sum(p["sample"] for p in per_class) * T / sum(p["sample"] * T / p["env_steps_per_s"] for p in per_class)
        out["cpu_baseline"] = {"value": total, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
                               "per_class": per_class,
                               "sample": f"up to 2048 evenly spaced environments per class x {T} steps, FP64 C oracle"}
        out["parity"] = {"step": T, "max_err": max(p["parity_max_err"] for p in per_class), "tolerance": 1e-3,
                         "pass": all(p["parity_max_err"] <= 1e-3 for p in per_class)}
    b.close()
    print(json.dumps(out), flush=True)


def run_trace(srv, trace, mgx):
    """Open-loop replay: each request is submitted at its trace time (server clock). A
    request continuing a session is submitted in session order once the session is
    resident, keeping its trace arrival time (so the wait counts in its latency); a
    session stays resident until its last request. Returns per-request (arrival, admit,
    done, env-steps) for the requests that completed, and the number that did not."""
    order = {}
    last_of = {}
    for k, r in enumerate(trace):
        order[k] = order.get(("n", r["session"]), 0)
        order[("n", r["session"])] = order[k] + 1
        last_of[r["session"]] = k
    t0 = mgx.mgx_server_now() + 0.05
    first_rid, sid_of, queue, dead, ids = {}, {}, {}, set(), []
    # Submit on time: latency counts from the trace arrival, so oversleeping here (the
    # default 50 us timer slack) would be charged to the server.
    try:
        import ctypes

        ctypes.CDLL(None).prctl(29, 1000, 0, 0, 0)  # PR_SET_TIMERSLACK = 29, in ns
    except (OSError, AttributeError):
        pass

    def submit(k, r, sess):
        rid = srv.submit(r["cls"], r["n"], r["horizon"], seed=r["seed"], hold=10, keep=last_of[r["session"]] != k,
                         session=sess, arrival=t0 + r["arrival"])
        ids.append((rid, r))
        return rid

    i = 0
    last_report = t0
    n_dropped = 0
    while i < len(trace) or any(queue.values()):
        now = mgx.mgx_server_now()
        if now - last_report > 1.0:
            last_report = now
            st = srv.stats()
            print(f"  t={now - t0:6.1f}s submitted {len(ids)}/{len(trace)} held {sum(map(len, queue.values()))} "
                  f"queued {st.queued} active {st.active} done {st.completed}", file=sys.stderr, flush=True)
        while i < len(trace) and t0 + trace[i]["arrival"] <= now:
            r = trace[i]
            if order[i] == 0:
                first_rid[r["session"]] = submit(i, r, -1)
            else:
                queue.setdefault(r["session"], []).append((i, r))
            i += 1
        for sess, q in queue.items():
            if not q:
                continue
            if sess in dead:
                n_dropped += len(q)
                q.clear()
                continue
            if sess not in sid_of:
                st = srv.poll(first_rid[sess])
                if st.state in (mgx.REQ_CANCELLED, mgx.REQ_FAILED):
                    dead.add(sess)
                    continue
                if st.session < 0:
                    continue
                sid_of[sess] = st.session
            while q:  # in session order; the server admits each when the session is free
                k, r = q.pop(0)
                submit(k, r, sid_of[sess])
        nxt = t0 + trace[i]["arrival"] if i < len(trace) else now + 2e-4
        gap = nxt - mgx.mgx_server_now()
        if gap > 1e-4:  # sleep, then spin through the last 100 us before the next arrival
            time.sleep(min(gap - 1e-4, 2e-4))
    out = []
    for k, (rid, r) in enumerate(ids):
        if k % 500 == 0:
            st = srv.stats()
            print(f"  collecting {k}/{len(ids)}: queued {st.queued} active {st.active} done {st.completed}",
                  file=sys.stderr, flush=True)
        try:
            st = srv.wait(rid, timeout=60.0)
        except mgx.MgxError:
            n_dropped += 1
            continue
        if st.state == mgx.REQ_DONE:
            out.append((st.t_arrival, st.t_admit, st.t_done, r["n"] * r["horizon"]))
        else:
            n_dropped += 1
    return np.array(out), n_dropped


def serve(args):
    """Config: Poisson arrivals (rate, duration); class uniform over the five classes;
    environments log-uniform in [64, 16384]; horizon uniform in [1, 500]; half the requests
    continue an open session (state resident); 64 GB budget. Continuous batching against
    the FIFO one-request-at-a-time baseline on the same trace."""
    import synth
    from paper_2503_09203_amd import mgx

    classes = synth.hetero_classes()
    nominal = [dict(mass=c.mass, added=c.added, dlin=c.dlin, dquad=c.dquad, buoy=c.buoy, current=np.zeros(3))
               for c in classes]
    import faulthandler
    faulthandler.dump_traceback_later(900, exit=True)
    trace = synth.serving_trace(rate=args.rate, duration=args.duration)
    offered = sum(r["n"] * r["horizon"] for r in trace) / args.duration
    res = {}
    for mode in ("batched", "fifo"):
        srv = mgx.Server(classes, nominal, budget_bytes=64 << 30, chunk_steps=args.serve_chunk, fifo=(mode == "fifo"))
        print(f"{mode}: warm-up", file=sys.stderr, flush=True)
        warm = [srv.submit(i % 5, 1024, 50, seed=i) for i in range(10)]
        for w_ in warm:
            srv.wait(w_, timeout=30.0)
        print(f"{mode}: trace of {len(trace)} requests", file=sys.stderr, flush=True)
        a, dropped = run_trace(srv, trace, mgx)
        st = srv.stats()
        srv.close()
        lat = a[:, 2] - a[:, 0]
        span = a[:, 2].max() - a[:, 0].min()
        res[mode] = {"requests": int(len(a)), "not_completed": int(dropped), "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                     "mean_latency_ms": float(lat.mean() * 1e3),
                     "p99_queue_ms": float(np.percentile(a[:, 1] - a[:, 0], 99) * 1e3),
                     "env_steps_per_s": float(a[:, 3].sum() / span), "iterations": int(st.iterations),
                     "bytes_peak": int(st.bytes_peak)}
        print(json.dumps({"mode": mode, **res[mode]}), file=sys.stderr, flush=True)
    out = {"metric": METRIC, "workload": f"serve_{args.rate:g}rps_{args.duration:g}s", "unit": "env-steps/s",
           "value": res["batched"]["env_steps_per_s"], "offered_env_steps_per_s": offered,
           "requests": len(trace), "chunk_steps": args.serve_chunk, "budget_bytes": 64 << 30,
           "batched": res["batched"], "fifo_baseline": res["fifo"],
           "p99_ratio_fifo_over_batched": res["fifo"]["p99_latency_ms"] / res["batched"]["p99_latency_ms"]}
    sweep_out = []
    for rate in [float(x) for x in args.sweep_rates.split(",") if x.strip()]:
        tr = synth.serving_trace(rate=rate, duration=5.0)
        point = {"rate": rate, "requests": len(tr),
                 "offered_env_steps_per_s": sum(r["n"] * r["horizon"] for r in tr) / 5.0}
        for mode in ("batched", "fifo"):
            srv = mgx.Server(classes, nominal, budget_bytes=64 << 30, chunk_steps=args.serve_chunk,
                             fifo=(mode == "fifo"))
            a, dropped = run_trace(srv, tr, mgx)
            srv.close()
            lat = a[:, 2] - a[:, 0]
            point[mode] = {"p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                           "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                           "env_steps_per_s": float(a[:, 3].sum() / (a[:, 2].max() - a[:, 0].min())),
                           "not_completed": int(dropped)}
            print(json.dumps({"rate": rate, "mode": mode, **point[mode]}), file=sys.stderr, flush=True)
        sweep_out.append(point)
    if sweep_out:
        out["rate_sweep"] = sweep_out
    print(json.dumps(out), flush=True)


def adjoint(args):
    """The differentiable rollout: 8192 environments of the 8-thruster class, horizon 256,
    per-step actions, checkpoints every 32 steps. Times the forward (positions after every
    step, checkpoints) and the backward (per-segment recomputation and the reverse sweep,
    gradients for every action and per-environment d_L, d_Q, M_A) through the C ABI."""
    import ctypes

    import torch

    import synth
    from paper_2503_09203_amd import mgx

    N, H, CK = 8192, 256, 32
    w = synth.differentiable(n=N, horizon=H)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    b.set_params(w.params)
    init = torch.tensor(b.pack_state([w.state[0].stacked()]), dtype=torch.float32, device="cuda:0")
    acts = torch.tensor(b.pack_actions([w.actions(H)[0]]), dtype=torch.float32, device="cuda:0")
    L = b.layout
    pos = torch.empty((H, 3 * L.n_pad_total), dtype=torch.float32, device="cuda:0")
    dpos = torch.randn_like(pos)
    dact = torch.zeros_like(acts)
    dpar = torch.zeros(18 * L.n_pad_total, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    fw, bw = [], []
    for i in range(args.warmup + args.steps):
        b.set_state(init)
        b.t = 0
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        mgx.mgx_rollout_forward(b.h, vp(acts), H, 0, 1, H, CK, vp(pos))
        e[1].record(stream)
        mgx.mgx_rollout_backward(b.h, vp(dpos), vp(dact), vp(dpar))
        e[2].record(stream)
        torch.cuda.synchronize()
        if i >= args.warmup:
            fw.append(e[0].elapsed_time(e[1]) * 1e-3)
            bw.append(e[1].elapsed_time(e[2]) * 1e-3)
    f, g = float(np.mean(fw)), float(np.mean(bw))
    m = w.classes[0].m
    step_flops, _ = mgx.mgx_step_cost(m)
    vjp_flops, vjp_ops = mgx.mgx_vjp_cost(m)
    # backward: every step outside the last segment recomputed once from its checkpoint
    # (storing its forward quantities; the forward pass stores the last segment's), then the
    # reverse part of every step's vector-Jacobian product. Forward: every step, plus the last
    # segment's steps once more with their forward quantities.
    last = H - (H - 1) // CK * CK
    traffic = recorded_adjoint_traffic()
    bwd_flops = step_flops * N * (H - last) + vjp_flops * N * H
    fwd_flops = step_flops * N * (H + last)
    out = {"metric": METRIC, "workload": f"adjoint_{N}x{H}", "unit": "env-steps/s", "value": N * H / (f + g),
           "n_envs": N, "horizon": H, "checkpoint_every": CK, "thrusters": m,
           "forward_ms": f * 1e3, "backward_ms": g * 1e3, "forward_env_steps_per_s": N * H / f,
           "backward_env_steps_per_s": N * H / g, "backward_over_forward": g / f,
           "roofline": {"bound": "alu", "kernel": f"k_rollout_bwd<float,{m},false>",
                        "achieved": bwd_flops / g / 1e12, "peak": (PEAK_FP32_VECTOR / 1e12), "unit": "TFLOP/s",
                        "frac": bwd_flops / g / 1e12 / (PEAK_FP32_VECTOR / 1e12), "flops_per_env_step": bwd_flops / (N * H),
                        "vjp_flops_per_env_step": vjp_flops, "vjp_valu_ops_per_env_step": vjp_ops,
                        "launch_ms": g * 1e3, "traffic": traffic.get("bwd"), "traffic_unit": "B/launch"},
           "forward_roofline": {"bound": "alu", "kernel": f"k_rollout_fwd<float,{m},false>",
                                "achieved": fwd_flops / f / 1e12, "peak": (PEAK_FP32_VECTOR / 1e12),
                                "unit": "TFLOP/s", "frac": fwd_flops / f / 1e12 / (PEAK_FP32_VECTOR / 1e12),
                                "flops_per_env_step": fwd_flops / (N * H), "traffic": traffic.get("fwd"),
                                "traffic_unit": "B/launch"}}
    b.close()
    print(json.dumps(out), flush=True)


def resample(args):
    """On-device domain randomisation: every environment of the randomised workload's class
    redrawn (uniform mass and buoyancy, Gaussian added mass per entry and current per axis,
    piecewise shared linear damping, absolute uniform quadratic damping) and its record
    rebuilt; timed with HIP events over repeated calls (a new epoch each)."""
    import torch

    import synth
    from paper_2503_09203_amd import mgx

    N = args.n
    w = synth.randomised(n=N, steps=8)
    c = w.classes[0]
    b = mgx.Batch([c], [N], w.dt, mgx.FP32)
    nominal = np.concatenate([[c.mass], c.added, c.dlin, c.dquad, [c.buoy], np.zeros(3)])[None]
    spec = {"mass": {"kind": mgx.DR_UNIFORM, "lo": 0.8, "hi": 1.2},
            "added": {"kind": mgx.DR_GAUSSIAN, "mean": 1.0, "std": 0.1, "lo": 0.7, "hi": 1.3},
            "dlin": {"kind": mgx.DR_PIECEWISE, "edges": [0.5, 0.9, 1.0, 1.3, 2.0], "weights": [2, 0, 5, 1],
                     "shared": 1},
            "dquad": {"kind": mgx.DR_UNIFORM, "lo": 5.0, "hi": 50.0, "relative": 0},
            "buoy": {"kind": mgx.DR_UNIFORM, "lo": 0.99, "hi": 1.03},
            "current": {"kind": mgx.DR_GAUSSIAN, "mean": 0.0, "std": 0.3, "lo": -1.0, "hi": 1.0, "relative": 0}}
    s = torch.cuda.current_stream()
    for e in range(args.warmup):
        b.resample(spec, nominal, seed=1, epoch=e)
    reps = max(args.steps, 10)
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(s)
    for e in range(reps):
        b.resample(spec, nominal, seed=1, epoch=1000 + e)
    z.record(s)
    torch.cuda.synchronize()
    per = a.elapsed_time(z) * 1e-3 / reps
    # the redraw at episode start: one-step station-keeping calls with scattered restarts
    # (targets up to 3.5 m away, distance limit 2.6 m), each followed by the masked redraw
    b.set_params(w.params)
    st = mgx.Station(b, d_max=2.6)
    st.reset(1)
    act1 = b.gen_actions(1, seed=3)
    out1 = st.empty_outputs(1)
    t_rs, n_rs = [], []
    for k in range(40):
        st.step(act1, out1)
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(s)
        st.resample(spec, nominal, seed=5)
        r1.record(s)
        torch.cuda.synchronize()
        if k >= 5:
            t_rs.append(r0.elapsed_time(r1) * 1e3)
            n_rs.append(int((out1["terminated"] | out1["truncated"]).sum()))
    st.close()
    rec_bytes = 30 * 4
    out = {"metric": METRIC, "workload": f"resample_{N}", "unit": "envs/s", "value": N / per,
           "launch_us_mean": per * 1e6, "n_envs": N,
           "roofline": {"bound": "hbm (record writes)", "achieved": N * rec_bytes / per / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": N * rec_bytes / per / PEAK_HBM, "bytes_per_env": rec_bytes},
           "note": "46 Philox uniforms, 10 Box-Muller draws in double and the record rebuild per environment",
           "restart_redraw": {"us_median": float(np.median(t_rs)), "restarts_per_call": float(np.mean(n_rs)),
                              "note": "mgx_station_resample after each one-step task call (HIP events around the "
                                      "call, host side included)"}}
    b.close()
    print(json.dumps(out), flush=True)


def station(args):
    """Station-keeping task steps of the randomised workload's 65,536 environments: each
    task step advances every environment one step under its command, then writes its
    observation, reward and flags and restarts ended episodes. Timed with HIP events on the
    batch stream over `steps` calls of 100 task steps each (one launch per call, the state
    in registers across its steps, every output kept per step), and separately as Gym steps
    (one task step per call from Python); parity on 256 sampled environments over one call."""
    import time

    import torch

    import oracle
    import synth
    from oracle import station as S
    from paper_2503_09203_amd import mgx

    N, CH = args.n, 100
    desc = dict(mgx.STATION_DEFAULTS)
    if args.station_class == "heavy8":
        # the first 8-thruster class of the heterogeneous set, randomised like the dr workload
        c = synth.hetero_classes()[3]
        params, dt = synth.randomised_params(c, N), 0.01
    else:
        w = synth.randomised(n=N, steps=8)
        c, params, dt = w.classes[0], w.params, w.dt
    b = mgx.Batch([c], [N], dt, mgx.FP32)
    b.set_params(params)
    st = mgx.Station(b, **desc)
    acts = b.gen_actions(CH, seed=17)
    out = st.empty_outputs(CH)
    s = torch.cuda.current_stream()
    st.reset(99)
    for _ in range(args.warmup):
        st.step(acts, out)
    reps = max(args.steps, 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        st.step(acts, out)
    e1.record(s)
    torch.cuda.synchronize()
    elapsed = e0.elapsed_time(e1) * 1e-3
    per_launch = elapsed / (reps * CH)
    m, P = c.m, 4
    # per task step: command, observation, reward, two flag bytes (the pre-reset observation
    # and new target of the few environments that end an episode on top); once per call:
    # state and episode counters read and written, record and target read
    bytes_es = P * (m + (13 + m) + 1) + 2 + (P * (2 * (13 + m) + 30 + 7) + 2 * 8) / CH
    ep, _ = st.episodes()

    # Gym steps: one task step per call, Python and the library call included
    act1 = acts[:1].clone()
    out1 = st.empty_outputs(1)
    for _ in range(20):
        st.step(act1, out1)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_gym = 500
    torch.cuda.synchronize()
    g0.record(s)
    for _ in range(n_gym):
        st.step(act1, out1)
    g1.record(s)
    torch.cuda.synchronize()
    gym_step = g0.elapsed_time(g1) * 1e-3 / n_gym

    # parity: 256 sampled environments over one call of 100 task steps from a fresh reset
    st.reset(99)
    st.step(acts, out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    ids = np.sort(rng.choice(N, 256, replace=False))
    sd = S.StationDesc(**desc)
    envs = oracle.make_envs(c, params.subset(ids), dt)
    o = S.StationOracle(sd, envs, m, ids=ids)
    o.reset(99)
    host_acts = b.unpack_actions(acts.cpu().numpy().astype(np.float64))[0]
    obs_all = out["obs"].cpu().numpy().astype(np.float64)
    rew = out["reward"].cpu().numpy().astype(np.float64)
    term = out["terminated"].cpu().numpy().astype(bool)
    ok = np.ones(ids.size, bool)
    worst, flags_ok = 0.0, True

    def near(obs):
        d = np.linalg.norm(obs[:, 0:3], axis=1)
        up = 1.0 - 2.0 * (obs[:, 4] ** 2 + obs[:, 5] ** 2)
        return (np.abs(d - sd.d_max) < 2e-3) | (np.abs(up - np.cos(sd.tilt_max)) < 2e-3) | (np.abs(obs[:, 3]) < 2e-3)

    for k in range(CH):
        ro, rr, rt, _, rf = o.step(host_acts[k][:, ids].T)
        ok &= ~near(ro) & ~near(rf)
        dev = b.unpack_state(obs_all[k])[0][:, ids].T
        rms = np.sqrt(np.mean(ro[ok] ** 2, axis=0))
        worst = max(worst, float(np.max(np.abs(dev[ok] - ro[ok]) / np.maximum(np.abs(ro[ok]), rms), initial=0)),
                    float(np.max(np.abs(rew[k, ids][ok] - rr[ok]), initial=0)))
        flags_ok &= bool(np.array_equal(term[k, ids][ok], rt[ok]))

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu = 4096
        cids = np.arange(0, N, N // n_cpu)[:n_cpu]
        oc = S.StationOracle(sd, oracle.make_envs(c, params.subset(cids), dt), m, ids=cids)
        oc.reset(99)
        a_cpu = host_acts[:, :, cids]
        t0 = time.perf_counter()
        for k in range(CH):
            oc.step(a_cpu[k].T)
        dt_cpu = time.perf_counter() - t0
        cpu = {"value": n_cpu * CH / dt_cpu, "unit": "env-steps/s", "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"{n_cpu} of {N} environments (evenly spaced ids) x {CH} task steps, FP64 oracle "
                         f"(C step with OpenMP, numpy observation/reward/reset), {dt_cpu:.1f} s"}
    out_line = {
        "metric": "station-keeping task env-steps/s (step, observation, reward, termination, auto-reset)",
        "value": N / per_launch, "unit": "env-steps/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": elapsed / reps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"station_{'heavy8_' if args.station_class == 'heavy8' else ''}{N}", "n_envs": N, "task_steps_per_call": CH, "thrusters": m,
                   "station": desc, "path": "station step: one launch per call of 100 task steps, all outputs "
                                            "kept per step"},
        "roofline": {"bound": "hbm", "achieved": N * bytes_es / per_launch / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": N * bytes_es / per_launch / PEAK_HBM,
                     "traffic": (recorded_station_traffic().get(CH) if (N, args.station_class) == (65536, "dr")
                                 else None), "traffic_unit": "B/launch",
                     "kernel": f"k_station_step<float,{m},false,false,false,true>", "launch_us_mean": per_launch * CH * 1e6, "us_per_task_step": per_launch * 1e6,
                     "bytes_per_env_step": bytes_es},
        "episodes_started_per_env": float(np.mean(ep)),
        "gym_step": {"env_steps_per_s": N / gym_step, "us_per_step": gym_step * 1e6,
                     "note": "one task step per Python call (Station.step with one command row)"},
        "cpu_baseline": cpu,
        "parity": {"metric": "max over sampled envs and steps of obs relative error and reward abs error",
                   "max_err": worst, "tolerance": 2e-4, "flags_equal": flags_ok, "pass": worst <= 2e-4 and flags_ok,
                   "envs_checked": int(ok.sum()), "steps": CH}}
    st.close()
    b.close()
    print(json.dumps(out_line), flush=True)


def counter_launches(args):
    """Six plain launches of the step kernel (no graph) for counter passes: K = 16 four
    times, then K = 1000 twice, at N environments of the chosen single-class workload
    (the randomised one by default)."""
    import torch

    import synth
    from paper_2503_09203_amd import mgx

    N, HOLD = args.n, 10
    make = {"dr": synth.randomised, "propellers": synth.propellers, "rudders": synth.rudders,
            "payload": synth.payload}.get(args.workload)
    if make is None:
        raise SystemExit("--counter-launches takes the dr, propellers, rudders or payload workload")
    w = make(n=N, steps=1000)
    b = mgx.Batch(w.classes, [N], w.dt)
    b.set_params(w.params)
    init = torch.tensor(b.pack_state([w.state[0].stacked()]), dtype=torch.float32, device="cuda:0")
    acts = b.gen_actions(101, seed=synth.MASTER_SEED)
    for K in (16, 16, 16, 16, 1000, 1000):
        b.set_state(init)
        b.t = 0
        b.step(acts, K, hold=HOLD)
    torch.cuda.synchronize()
    b.close()
    print(json.dumps({"counter_launches": [16, 16, 16, 16, 1000, 1000], "n": N}), flush=True)


def sweep(args):
    """Per-launch durations over K at the default N, and over N for K = 1 and K = 16: a
    graph of L launches replayed between two HIP events on the batch stream (L x K steps
    from one resident state, the action buffer sized for them), so the numbers carry the
    launch floor as a rollout does but not the host's launch calls. One JSON line per point,
    with the bytes the batch's state, record and one step's actions occupy."""
    import torch

    import synth
    from paper_2503_09203_amd import mgx

    HOLD = 10
    cls = synth.plain_class()
    flops_es, _ = mgx.mgx_step_cost(cls.m)

    def measure(N, K):
        steps = int(min(4096, max(K, 1e9 * HOLD / (N * cls.m * 4)))) // K * K   # actions <= ~1 GB
        L = max(1, steps // K)
        p = synth.randomised_params(cls, N)
        st = synth.initial_state(N, cls.m)
        b = mgx.Batch([cls], [N], 0.01)
        b.set_params(p)
        init = torch.tensor(b.pack_state([st.stacked()]), dtype=torch.float32, device="cuda:0")
        acts = b.gen_actions(-(-L * K // HOLD) + 1)
        stream = torch.cuda.current_stream()
        b.t = 0
        g = b.capture(acts, L * K, K, hold=HOLD)
        best = None
        for rep in range(4):
            b.reset(init_state=init)
            b.t = 0
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            if rep:
                t = e0.elapsed_time(e1) * 1e-3 / L
                best = t if best is None else min(best, t)
        g.close()
        b.close()
        resident = N * ((13 + cls.m) * 4 + 30 * 4 + cls.m * 4)
        return {"n": N, "K": K, "launches": L, "launch_us": best * 1e6, "env_steps_per_s": N * K / best,
                "tflops": flops_es * N * K / best / 1e12,
                "gbps": bytes_per_env_step(cls.m, K, HOLD) * N * K / best / 1e9, "resident_mb": resident / 1e6}

    for K in (1, 2, 4, 8, 16, 32, 64, 128, 256, 1000):
        print(json.dumps({"sweep": "K", **measure(args.n, K)}), flush=True)
    for e in range(12, 23):
        for K in (1, 16):
            print(json.dumps({"sweep": "N", **measure(1 << e, K)}), flush=True)

if __name__ == "__main__":
    main()
