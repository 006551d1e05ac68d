"""How much the FP64 map itself amplifies FP32 rounding, per workload: the oracle run with
its state rounded to float32 after every step, against the plain oracle, after 1000 steps.
This floor is what an FP32 implementation that rounds its state every step starts from; the
1e-3 parity bar sits above it for every workload. The rudder class's trajectories amplify
rounding about 20 times more than the propeller classes' (its device step carries the
attitude's low-order words through a launch for that reason). CPU only."""
import numpy as np
import pytest

import oracle
import synth
from parity import RUDDER_SENSITIVE, component_errors


def _floor(make, n=65536, steps=1000):
    w = make(n=n, steps=steps)
    c = w.classes[0]
    envs = oracle.make_envs(c, w.params, w.dt)
    st = w.state[0]
    x0 = oracle.pack_state(st.p, st.q, st.nu, st.n)
    a = oracle.pack_actions(w.actions(steps // 10)[0])
    ref, _, _ = oracle.rollout(envs, x0.copy(), a, 10, steps)
    x = x0.copy()
    for k in range(steps):
        x, _, _ = oracle.rollout(envs, x, a, 10, 1, t0=k)
        x = x.astype(np.float32).astype(np.float64)
    g, r = oracle.unpack_state(x, c.m), oracle.unpack_state(ref, c.m)
    rms = np.sqrt(np.mean(r * r, axis=1, keepdims=True))
    per_env = (np.abs(g - r) / np.maximum(np.abs(r), rms)).max(axis=0)
    return component_errors(g, r).max(), per_env


def test_fp32_storage_floor_sets_the_bars():
    dr, _ = _floor(synth.randomised)
    rudder, per_env = _floor(synth.rudders)
    print(f"fp32 storage floor after 1000 steps: randomised {dr:.2e}, rudder {rudder:.2e}", flush=True)
    assert dr < 1e-4 and 10 * dr < 1e-3          # the 1e-3 bar sits far above the floor
    assert 5 * dr < rudder < 1e-3                  # the rudder class is much worse conditioned
    # the environments the rudder parity test adds to its sample are this floor's worst ten
    assert sorted(np.argsort(-per_env)[:10].tolist()) == sorted(RUDDER_SENSITIVE.tolist())
