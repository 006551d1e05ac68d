"""Heterogeneous classes in one persistent launch, captured 32-step chunks and the
launch-shape autotuner."""
import os

import numpy as np
import pytest

import synth
from paper_2503_09203_amd import mgx

from gpu_helpers import device_actions, make_batch, run_pair, torch
from parity import component_errors

pytestmark = pytest.mark.gpu


def _advance(b, acts, steps, K, hold=10):
    done = 0
    while done < steps:
        k = min(K, steps - done)
        b.step(acts, k, hold=hold)
        done += k


@pytest.mark.parametrize("scale,block,gpc", [(0.05, 256, 2), (1.0, 256, 2), (1.0, 64, 1)])
def test_persistent_equals_per_class_bitwise(scale, block, gpc):
    """(1.0, 64, 1): 256 waves for 1,103 tiles, so most tiles come from the device counter
    after each wave's first one."""
    t = torch()
    w = synth.heterogeneous(scale=scale, steps=64)
    acts = w.actions(8)
    outs = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        b = make_batch(w)
        b.set_shape(mode, 16, block, gpc)
        _advance(b, device_actions(b, acts), 64, 16)
        outs.append(b.get_state())
        b.close()
    assert t.equal(outs[0], outs[1])


@pytest.mark.parametrize("block,gpc", [(256, 2), (64, 1)])
def test_persistent_statistics_match_per_class(block, gpc):
    w = synth.heterogeneous(scale=0.5, steps=20)
    acts = w.actions(2)
    st = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        b = make_batch(w)
        b.set_shape(mode, 20, block, gpc)
        b.step(device_actions(b, acts), 20, hold=10, flags=mgx.STEP_STATS)
        st.append(b.stats())
        assert b.check() == (mgx.MGX_OK, 0)
        b.close()
    for c in range(5):
        assert st[0].max_speed[c] == st[1].max_speed[c] and st[0].max_rate[c] == st[1].max_rate[c]
        assert abs(st[0].mean_speed[c] - st[1].mean_speed[c]) <= 1e-6 * st[0].mean_speed[c]
        assert abs(st[0].mean_kinetic[c] - st[1].mean_kinetic[c]) <= 1e-6 * st[0].mean_kinetic[c]
        assert st[1].n_nonfinite[c] == 0


def test_heterogeneous_full_size_persistent_graph_parity():
    """70,512 environments of five classes, persistent launches in captured 32-step
    chunks, 1000 steps; 600 sampled environments (all classes) against the oracle."""
    w = synth.heterogeneous(steps=1000)
    acts = w.actions(100)
    rng = np.random.default_rng(3)
    sample = [np.unique(np.concatenate([[0, n - 1], rng.choice(n, min(n, 118), replace=False)])) for n in w.n_envs]
    t = torch()
    b = make_batch(w)
    b.set_shape(mgx.LAUNCH_PERSISTENT, 8)
    a = device_actions(b, acts)
    g = b.capture(a, 32, 0, hold=10)
    for _ in range(31):
        g.replay()
    b.step(a, 8, hold=10)
    assert b.t == 1000
    gpu = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))
    g.close()
    b.close()
    import oracle
    from gpu_helpers import oracle_inputs
    for c, ((envs, st0), s) in enumerate(zip(oracle_inputs(w), sample)):
        st, _, _ = oracle.rollout(envs[s], st0[s].copy(), oracle.pack_actions(acts[c])[s], 10, 1000)
        err = component_errors(gpu[c][:, s], oracle.unpack_state(st, w.classes[c].m))
        assert err.max() <= 1e-3, (c, err)


def test_autotuner_restores_state_and_caches(tmp_path):
    t = torch()
    w = synth.heterogeneous(scale=0.1, steps=64)
    b = make_batch(w)
    a = device_actions(b, w.actions(8))
    b.step(a, 5, hold=10)
    before = b.get_state().clone()
    shape = b.autotune(a, 32, hold=10)
    assert shape.candidates >= 6 and shape.us_per_chunk > 0 and shape.from_cache == 0
    assert 32 % shape.K == 0
    assert t.equal(b.get_state(), before) and b.t == 5
    # stepping with the tuned shape continues the same trajectory as the default shape
    b.step(a, 32, hold=10)
    tuned = b.get_state().clone()
    b2 = make_batch(w)
    b2.step(device_actions(b2, w.actions(8)), 5, hold=10)
    b2.step(device_actions(b2, w.actions(8)), 32, hold=10)
    assert t.equal(b2.get_state(), tuned)
    again = b.autotune(a, 32, hold=10)
    assert again.from_cache == 1 and again.K == shape.K and again.mode == shape.mode
    path = tmp_path / "shapes.txt"
    mgx.mgx_autotune_save(path)
    assert path.read_text().count("\n") >= 2
    mgx.mgx_autotune_load(path)
    bad = tmp_path / "bad.txt"
    bad.write_text("garbage line\n")
    with pytest.raises(mgx.MgxError):
        mgx.mgx_autotune_load(bad)
    b.close()
    b2.close()


def test_shape_validation():
    w = synth.heterogeneous(scale=0.02, steps=4)
    b = make_batch(w, precision=mgx.FP64)
    with pytest.raises(mgx.MgxError):
        b.set_shape(mgx.LAUNCH_PERSISTENT, 16)
    with pytest.raises(mgx.MgxError):
        b.set_shape(mgx.LAUNCH_PER_CLASS, 16, block=512)
    b.close()


def test_switching_launch_modes_between_calls():
    """Per-class and persistent launches interleaved on one batch (the work counter of the
    persistent launch must be fresh whatever ran before)."""
    t = torch()
    w = synth.heterogeneous(scale=0.05, steps=40)
    acts = w.actions(5)
    ref = make_batch(w)
    _advance(ref, device_actions(ref, acts), 40, 5)
    b = make_batch(w)
    a = device_actions(b, acts)
    for i in range(8):
        b.set_shape(mgx.LAUNCH_PERSISTENT if i % 3 == 0 else mgx.LAUNCH_PER_CLASS, 5)
        b.step(a, 5, hold=10)
    assert t.equal(b.get_state(), ref.get_state())
    b.t = 0
    b.set_shape(mgx.LAUNCH_PERSISTENT, 5)
    b.step(a, 5, hold=10)
    b.close()
    ref.close()


def test_sixteen_classes_of_one_to_eight_thrusters():
    """The widest batch: 16 classes (1..8 thrusters, each twice) with ragged counts from 1
    to 1000 environments, 100 steps in 16-step launches. Per-class launches and the
    persistent launch (every class's constants staged in LDS) agree bitwise and match the
    oracle."""
    w = synth.many_classes(steps=100)
    acts = w.actions(11)
    finals = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        fin = []
        res = run_pair(w, acts, 10, [1, 100], chunk=16, shape=(mode, 16), final_state=fin)
        finals.append(fin[0])
        for k, pairs in res:
            bar = 1e-5 if k == 1 else 5e-4
            for c, (g, r) in enumerate(pairs):
                err = component_errors(g, r)
                assert np.all(err <= bar), (mode, k, c, err.max())
    assert np.array_equal(finals[0], finals[1])


def test_propeller_variant_classes_in_the_persistent_launch():
    """Two of the five classes with dead zones, reverse gains and shaft torques next to
    three plain ones: the persistent launch takes the shaped-thrust body per tile and
    agrees bitwise with per-class launches, and both match the oracle."""
    w = synth.heterogeneous(scale=0.05, steps=64)
    w.classes[1] = synth.propeller_variants(w.classes[1])
    w.classes[3] = synth.propeller_variants(w.classes[3])
    acts = w.actions(8)
    finals = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        fin = []
        res = run_pair(w, acts, 10, [1, 64], chunk=16, shape=(mode, 16), final_state=fin)
        finals.append(fin[0])
        for k, pairs in res:
            bar = 1e-5 if k == 1 else 5e-4
            for c, (g, r) in enumerate(pairs):
                err = component_errors(g, r)
                assert np.all(err <= bar), (mode, k, c, err.max())
    assert np.array_equal(finals[0], finals[1])


def test_fin_class_keeps_per_class_launches_in_persistent_mode():
    """A batch with a fin class asked for the persistent launch runs per-class launches
    (the persistent kernel holds the propeller bodies only): same state bitwise, and the
    oracle agrees."""
    hc = synth.hetero_classes()
    w = synth.mixed([hc[0], hc[1], synth.rudder_class(), hc[3]], [100, 150, 200, 130], steps=48)
    acts = w.actions(6)
    finals = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        fin = []
        res = run_pair(w, acts, 10, [1, 48], chunk=16, shape=(mode, 16), final_state=fin)
        finals.append(fin[0])
        for k, pairs in res:
            bar = 1e-5 if k == 1 else 5e-4
            for c, (g, r) in enumerate(pairs):
                assert np.all(component_errors(g, r) <= bar), (mode, k, c)
    assert np.array_equal(finals[0], finals[1])


def test_payload_class_in_a_mixed_batch():
    """A payload class (its records hold 15 more rows) between propeller and rudder
    classes: per-class and persistent-shaped launches agree bitwise and match the oracle."""
    hc = synth.hetero_classes()
    w = synth.mixed([hc[0], synth.payload_class(), synth.rudder_class(), hc[3]], [100, 150, 200, 130], steps=48)
    acts = w.actions(6)
    finals = []
    for mode in (mgx.LAUNCH_PER_CLASS, mgx.LAUNCH_PERSISTENT):
        fin = []
        res = run_pair(w, acts, 10, [1, 48], chunk=16, shape=(mode, 16), final_state=fin)
        finals.append(fin[0])
        for k, pairs in res:
            bar = 1e-5 if k == 1 else 5e-4
            for c, (g, r) in enumerate(pairs):
                assert np.all(component_errors(g, r) <= bar), (mode, k, c)
    assert np.array_equal(finals[0], finals[1])
