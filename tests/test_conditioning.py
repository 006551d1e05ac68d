"""How much the FP64 map itself amplifies FP32 rounding, per workload: the oracle run with
its state rounded to float32 after every step, against the plain oracle, after 1000 steps.
This floor is what any FP32 implementation starts from; the parity bars are set well above
it (1e-3 for the propeller workloads, 5e-3 for the rudder class, whose floor is about 20
times higher). CPU only."""
import numpy as np
import pytest

import oracle
import synth
from parity import component_errors


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
    return component_errors(oracle.unpack_state(x, c.m), oracle.unpack_state(ref, c.m)).max()


def test_fp32_storage_floor_sets_the_bars():
    dr = _floor(synth.randomised)
    rudder = _floor(synth.rudders)
    print(f"fp32 storage floor after 1000 steps: randomised {dr:.2e}, rudder {rudder:.2e}", flush=True)
    assert dr < 1e-4 and 10 * dr < 1e-3          # the 1e-3 bar sits far above the floor
    assert 5 * dr < rudder < 1e-3                  # the rudder class is much worse conditioned
    assert 5 * rudder < 5e-3                       # and its 5e-3 bar still sits above its floor
