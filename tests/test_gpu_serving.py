"""Continuous-batching server: results do not depend on what else runs, sessions stay
resident, admission follows the memory budget, cancellation releases memory."""
import numpy as np
import pytest

import oracle
import synth
from paper_2503_09203_amd import mgx

from parity import component_errors

pytestmark = pytest.mark.gpu

CLASSES = None


def classes():
    global CLASSES
    if CLASSES is None:
        CLASSES = synth.hetero_classes()
    return CLASSES


def nominal(c):
    return dict(mass=c.mass, added=c.added, dlin=c.dlin, dquad=c.dquad, buoy=c.buoy, current=np.zeros(3))


def server(**kw):
    cs = classes()
    return mgx.Server(cs, [nominal(c) for c in cs], **kw)


def oracle_final(cls_index, n, horizon, seed, hold=10):
    c = classes()[cls_index]
    st = synth.initial_state(n, c.m, seed)
    x = oracle.pack_state(st.p, st.q, st.nu, st.n)
    rows = horizon // hold + 1
    a = synth.actions(n, c.m, rows, seed)
    envs = oracle.make_envs(c, synth.nominal_params(c, n), 0.01)
    x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(a), hold, horizon)
    return oracle.unpack_state(x, c.m)


def test_result_is_the_same_alone_and_in_the_mix():
    R = dict(class_index=2, n_envs=1000, horizon=137, seed=11)
    s1 = server(chunk_steps=32)
    r = s1.submit(**R, keep=True)
    st = s1.wait(r)
    alone = s1.read_state(st.session, 2, 1000)
    s1.close()

    s2 = server(chunk_steps=32)
    rng = np.random.default_rng(5)
    ids = []
    for i in range(12):
        ids.append(s2.submit(int(rng.integers(0, 5)), int(rng.integers(64, 5000)), int(rng.integers(1, 300)),
                             seed=100 + i))
        if i == 5:
            rid = s2.submit(**R, keep=True)
    for i in ids:
        s2.wait(i)
    st2 = s2.wait(rid)
    mixed = s2.read_state(st2.session, 2, 1000)
    stats = s2.stats()
    s2.close()
    assert np.array_equal(alone, mixed)
    assert stats.completed == 13 and stats.iterations > 5

    ref = oracle_final(2, 1000, 137, 11)
    assert component_errors(alone.astype(np.float64), ref).max() <= 5e-4


def test_fifo_baseline_gives_the_same_result():
    R = dict(class_index=4, n_envs=700, horizon=90, seed=3)
    outs = []
    for fifo in (False, True):
        s = server(chunk_steps=16, fifo=fifo)
        r = s.submit(**R, keep=True)
        st = s.wait(r)
        outs.append(s.read_state(st.session, 4, 700))
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_session_continuation_equals_one_long_request():
    s = server(chunk_steps=32)
    r1 = s.submit(class_index=3, n_envs=500, horizon=60, seed=21, keep=True)
    st1 = s.wait(r1)
    r2 = s.submit(class_index=3, n_envs=500, horizon=45, seed=0, keep=True, session=st1.session)
    st2 = s.wait(r2)
    assert st2.session == st1.session
    cont = s.read_state(st1.session, 3, 500)
    r3 = s.submit(class_index=3, n_envs=500, horizon=105, seed=21, keep=True)
    st3 = s.wait(r3)
    one = s.read_state(st3.session, 3, 500)
    s.release(st1.session)
    s.release(st3.session)
    assert s.stats().bytes_in_use == 0
    s.close()
    assert np.array_equal(cont, one)


def test_state_read_never_mixes_steps():
    """Reads of a session's state issued right after a continuing request is submitted
    either find the request admitted (MGX_E_STATE) or hold it back until the copy is done:
    every read returns the state before the request or after it, never a mix."""
    s = server(chunk_steps=8)
    r1 = s.submit(class_index=2, n_envs=16384, horizon=50, seed=31, keep=True)
    sid = s.wait(r1).session
    before = s.read_state(sid, 2, 16384)
    r2 = s.submit(class_index=2, n_envs=16384, horizon=200, seed=0, keep=True, session=sid)
    reads, refused = [], 0
    for _ in range(40):
        try:
            reads.append(s.read_state(sid, 2, 16384))
        except mgx.MgxError as e:
            assert e.status == mgx.MGX_E_STATE
            refused += 1
    s.wait(r2)
    after = s.read_state(sid, 2, 16384)
    s.release(sid)
    s.close()
    assert not np.array_equal(before, after)
    for x in reads:
        assert np.array_equal(x, before) or np.array_equal(x, after)
    print(f"reads {len(reads)}, refused while running {refused}", flush=True)


def test_caller_commands_drive_a_session():
    """A request may bring its own command rows. The generator's own rows given as caller
    commands reproduce the seed-driven result bit for bit; a continuing request with other
    commands (clipped) matches the oracle over both requests; rows that do not cover the
    horizon fail the request at admission."""
    import torch as t
    c, n, seed = 3, 700, 41
    m = classes()[c].m
    gen = synth.actions(n, m, 10, seed)                            # [rows, m, n]
    s = server(chunk_steps=16)
    r1 = s.submit(class_index=c, n_envs=n, horizon=90, seed=seed, keep=True)
    own = s.read_state(s.wait(r1).session, c, n)
    dev = t.tensor(gen, dtype=t.float32, device="cuda:0").contiguous()
    r2 = s.submit(class_index=c, n_envs=n, horizon=90, seed=seed, keep=True, actions=dev)
    sid = s.wait(r2).session
    given = s.read_state(sid, c, n)
    assert np.array_equal(own, given)
    # continue the second session at step 90 with other commands: hold intervals 9..14
    rng = np.random.default_rng(8)
    other = rng.uniform(-1.3, 1.3, size=(6, m, n)).astype(np.float32)
    dev2 = t.tensor(other, device="cuda:0").contiguous()
    r3 = s.submit(class_index=c, n_envs=n, horizon=55, seed=0, keep=True, session=sid, actions=dev2)
    s.wait(r3)
    got = s.read_state(sid, c, n)
    short = t.zeros((2, m, n), dtype=t.float32, device="cuda:0")
    r4 = s.submit(class_index=c, n_envs=n, horizon=55, seed=0, keep=True, session=sid, actions=short)
    with pytest.raises(mgx.MgxError):
        s.wait(r4)
    assert s.poll(r4).state == mgx.REQ_FAILED
    assert np.array_equal(s.read_state(sid, c, n), got)             # the failed request moved nothing
    s.release(sid)
    s.close()
    cl = classes()[c]
    st = synth.initial_state(n, m, seed)
    x = oracle.pack_state(st.p, st.q, st.nu, st.n)
    envs = oracle.make_envs(cl, synth.nominal_params(cl, n), 0.01)
    x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(gen), 10, 90)
    x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(other.astype(np.float64)), 10, 55, t0=90, row0=9)
    ref = oracle.unpack_state(x, m)
    assert component_errors(got.astype(np.float64), ref).max() <= 5e-4


def test_admission_waits_for_memory():
    """A budget of three 1024-environment sessions and nine requests: at no admission are
    more than two other sessions resident, and with 2000-step horizons the first three are
    still running while the rest are submitted, so later requests wait for memory."""
    c = classes()[3]
    per = 4 * 1024 * (13 + c.m + 30)       # bytes of one 1024-env session of class 3
    s = server(chunk_steps=16, budget_bytes=3 * per)
    ids = [s.submit(3, 1024, 2000, seed=i) for i in range(9)]
    with pytest.raises(mgx.MgxError) as e:
        s.submit(3, 4096, 10, seed=1)
    assert e.value.status == mgx.MGX_E_BUDGET
    sts = [s.wait(i, timeout=60) for i in ids]
    st = s.stats()
    s.close()
    assert all(x.state == mgx.REQ_DONE for x in sts)
    assert st.bytes_peak <= 3 * per and st.completed == 9
    adm = np.array([x.t_admit for x in sts])
    done = np.array([x.t_done for x in sts])
    for j in range(9):
        resident = sum(1 for i in range(9) if i != j and adm[i] <= adm[j] < done[i])
        assert resident <= 2, (j, resident)
    waited = np.sort(adm - np.array([x.t_arrival for x in sts]))
    assert waited[-1] > 3 * waited[0] and waited[-1] > 1e-4


def test_cancel_releases_the_session():
    s = server(chunk_steps=8)
    r = s.submit(1, 3000, 100000, seed=1)
    s.cancel(r)
    st = s.wait(r, timeout=30)
    assert st.state == mgx.REQ_CANCELLED
    assert s.stats().bytes_in_use == 0
    s.close()


def test_iterations_with_more_tiles_than_waves():
    """Three 50,000-environment requests share iterations on one stream: 2,346 tiles against
    the 2,048 waves of a launch, so the last tiles come from the device counter. Each result
    equals the same request run alone (whose iterations need no counter)."""
    reqs = [dict(class_index=c, n_envs=50000, horizon=40, seed=70 + c) for c in (1, 3, 4)]
    alone = []
    for R in reqs:
        s = server(chunk_steps=4, streams=1, budget_bytes=1 << 31)
        st = s.wait(s.submit(**R, keep=True), timeout=60)
        alone.append(s.read_state(st.session, R["class_index"], R["n_envs"]))
        s.close()
    s = server(chunk_steps=4, streams=1, budget_bytes=1 << 31)
    ids = [s.submit(**R, keep=True) for R in reqs]
    sts = [s.wait(i, timeout=60) for i in ids]
    mixed = [s.read_state(st.session, R["class_index"], R["n_envs"]) for st, R in zip(sts, reqs)]
    stats = s.stats()
    s.close()
    for a, m in zip(alone, mixed):
        assert np.array_equal(a, m)
    assert stats.completed == 3


def test_propeller_variant_class_is_served():
    """A class with dead zones, reverse gains and shaft torques, served next to the plain
    classes, matches the oracle."""
    cs = list(classes()) + [synth.propeller_variants(classes()[2])]
    s = mgx.Server(cs, [nominal(c) for c in cs], chunk_steps=32)
    r = s.submit(class_index=5, n_envs=700, horizon=90, seed=13, keep=True)
    other = s.submit(class_index=2, n_envs=300, horizon=40, seed=14)
    st = s.wait(r)
    s.wait(other)
    got = s.read_state(st.session, 5, 700)
    s.close()
    c = cs[5]
    ini = synth.initial_state(700, c.m, 13)
    x = oracle.pack_state(ini.p, ini.q, ini.nu, ini.n)
    a = synth.actions(700, c.m, 90 // 10 + 1, 13)
    envs = oracle.make_envs(c, synth.nominal_params(c, 700), 0.01)
    x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(a), 10, 90)
    ref = oracle.unpack_state(x, c.m)
    assert component_errors(got.astype(np.float64), ref).max() <= 5e-4


def test_server_refuses_fin_classes():
    cs = list(classes()) + [synth.rudder_class()]
    with pytest.raises(mgx.MgxError) as e:
        mgx.Server(cs, [nominal(c) for c in cs], chunk_steps=32)
    assert "has fins" in str(e.value)


def test_server_refuses_payload_classes():
    cs = list(classes()) + [synth.payload_class()]
    with pytest.raises(mgx.MgxError) as e:
        mgx.Server(cs, [nominal(c) for c in cs], chunk_steps=32)
    assert "payload" in str(e.value)
