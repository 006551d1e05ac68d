"""Station-keeping task on the device against the task oracle (``oracle/station.py``),
through the C ABI: episode start draws, observations, rewards, termination and truncation
flags, same-step auto-reset and episode counters, for one class and for a mixed batch,
with substeps, for the shaped, fin and payload bodies, and in float32 and float64.

Termination is decided in the batch precision on the device and in double in the oracle,
so where the oracle's distance or lean lies within `margin` of its threshold both decisions
are correct. Every environment is compared step by step over whole rollouts, including
every reset; one leaves the comparison only at a step where the two sides decide
differently, which must be such a near-threshold step (their episodes then part). The
attitude error's scalar part is kept non-negative, so near zero the two sides may hold the
same rotation with opposite vector parts: those are compared up to that sign."""
import numpy as np
import pytest

import oracle
import synth
from oracle import station as S
from paper_2503_09203_amd import mgx

from gpu_helpers import make_batch, oracle_inputs, torch

pytestmark = pytest.mark.gpu

DESC = dict(target_box=2.0, tilt0=0.3, v0=0.1, sigma_p=0.5, w_att=0.5, w_act=0.01, d_max=2.6, tilt_max=0.6,
            max_steps=40, substeps=1)


def run_both(w, desc, T, precision=mgx.FP32, seed=7, act_seed=3):
    """T task steps on the device and in the oracle with the same commands. Returns per
    class a list of per-step dicts with both sides' results."""
    t = torch()
    b = make_batch(w, precision)
    st = mgx.Station(b, **desc)
    obs0 = st.reset(seed).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(act_seed)
    acts = [rng.uniform(-1.2, 1.2, size=(T, c.m, n)).astype(np.float32) for c, n in zip(w.classes, w.n_envs)]
    dev_acts = t.tensor(b.pack_actions(acts), dtype=b.dtype, device=b.device)
    out = st.step(dev_acts)
    t.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    ep_dev, et_dev = st.episodes()
    st.close()
    b.close()
    res = []
    off = 0
    for c, (cls, n) in enumerate(zip(w.classes, w.n_envs)):
        envs = oracle_inputs(w)[c][0]
        o = S.StationOracle(S.StationDesc(**desc), envs, cls.m, env_off=off)
        steps = [{"obs_dev": b.unpack_state(obs0)[c].T, "obs_ref": o.reset(seed)}]
        for k in range(T):
            obs, r, term, trunc, final = o.step(acts[c][k].T.astype(np.float64))
            pad = sum(b.n_pad[:c])
            steps.append({
                "obs_dev": b.unpack_state(g["obs"][k].astype(np.float64))[c].T, "obs_ref": obs,
                "final_dev": b.unpack_state(g["final_obs"][k].astype(np.float64))[c].T, "final_ref": final,
                "r_dev": g["reward"][k, pad:pad + n].astype(np.float64), "r_ref": r,
                "term_dev": g["terminated"][k, pad:pad + n].astype(bool), "term_ref": term,
                "trunc_dev": g["truncated"][k, pad:pad + n].astype(bool), "trunc_ref": trunc})
        res.append({"steps": steps, "ep_dev": ep_dev[off:off + n], "et_dev": et_dev[off:off + n],
                    "ep_ref": o.episode.copy(), "et_ref": o.t.copy()})
        off += n
    return res


def ambiguous(obs, desc, margin):
    """Environments whose observation lies within `margin` of a termination decision:
    distance against d_max, or lean against tilt_max (R_zz of the state equals that of the
    attitude error, the target being a pure yaw)."""
    d = np.linalg.norm(obs[:, 0:3], axis=1)
    up = 1.0 - 2.0 * (obs[:, 4] ** 2 + obs[:, 5] ** 2)
    return (np.abs(d - desc["d_max"]) < margin) | (np.abs(up - np.cos(desc["tilt_max"])) < margin)


def align_sign(dev, ref):
    """The device observations with the attitude error's vector part (columns 4-6) turned to
    the oracle's sign. Both sides keep the scalar part (column 3) non-negative; where it is
    near zero they may hold the same rotation as q and -q, which then differ in the sign of
    the vector part only."""
    out = dev.copy()
    s = np.sign(np.sum(dev[:, 4:7] * ref[:, 4:7], axis=1))
    out[:, 4:7] *= np.where(s == 0, 1.0, s)[:, None]
    return out


def rel_err(dev, ref, ok):
    """max over the selected environments of |dev - ref| / max(|ref|, rms), per component,
    the rms taken over the whole batch's reference (as the parity metric does)."""
    if not ok.any():
        return 0.0
    rms = np.sqrt(np.mean(ref * ref, axis=0))
    d, r = align_sign(dev, ref)[ok], ref[ok]
    return float(np.max(np.abs(d - r) / np.maximum(np.abs(r), np.maximum(rms, 1e-30))))


def decide(alive, term_dev, term_ref, trunc_dev, trunc_ref, obs_ref, desc, margin, where):
    """Environments still compared after this step: a differing decision must lie within
    the margin of its threshold, and takes the environment out of the comparison."""
    differ = (term_dev != term_ref) | (trunc_dev != trunc_ref)
    bad = alive & differ & ~ambiguous(obs_ref, desc, margin)
    assert not bad.any(), f"{where}: decisions differ away from a threshold at {np.flatnonzero(bad)[:8]}"
    return alive & ~differ


def check(res, desc, tol, margin, min_compared=0.99, name=""):
    stats = {"resets": 0, "terminated": 0, "parted": 0}
    for cres in res:
        steps = cres["steps"]
        ok = np.ones(steps[0]["obs_ref"].shape[0], bool)
        assert rel_err(steps[0]["obs_dev"], steps[0]["obs_ref"], ok) <= tol, f"{name} reset obs"
        for k, s in enumerate(steps[1:], 1):
            ok = decide(ok, s["term_dev"], s["term_ref"], s["trunc_dev"], s["trunc_ref"], s["final_ref"], desc,
                        margin, f"{name} step {k}")
            e_obs = rel_err(s["obs_dev"], s["obs_ref"], ok)
            # the pre-reset observation is written for the environments that ended
            ended = ok & (s["term_ref"] | s["trunc_ref"])
            e_fin = rel_err(s["final_dev"], s["final_ref"], ended)
            e_r = float(np.max(np.abs(s["r_dev"][ok] - s["r_ref"][ok]), initial=0.0))
            assert e_obs <= tol and e_fin <= tol and e_r <= tol, f"{name} step {k}: {e_obs} {e_fin} {e_r}"
            stats["resets"] += int(np.sum((s["term_ref"] | s["trunc_ref"])[ok]))
            stats["terminated"] += int(np.sum(s["term_ref"][ok]))
        assert np.array_equal(cres["ep_dev"][ok], cres["ep_ref"][ok]), name
        assert np.array_equal(cres["et_dev"][ok], cres["et_ref"][ok]), name
        stats["parted"] += int((~ok).sum())
        assert ok.mean() >= min_compared, f"{name}: only {ok.mean():.3f} of the environments compared"
    print(name, stats, flush=True)
    return stats


@pytest.mark.parametrize("precision,tol,margin", [(mgx.FP32, 2e-4, 2e-3), (mgx.FP64, 1e-9, 1e-7)])
def test_reset_draws_match_the_oracle(precision, tol, margin):
    w = synth.plain_small(n=1000)  # 1000: a ragged last wave
    t = torch()
    b = make_batch(w, precision)
    st = mgx.Station(b, **DESC)
    obs = st.reset(123).cpu().numpy().astype(np.float64)
    state = b.get_state().cpu().numpy().astype(np.float64)
    ref_s, ref_t = S.episode_start(S.StationDesc(**DESC), 123, np.arange(1000), 0, 6)
    dt = np.float32 if precision == mgx.FP32 else np.float64
    dev_s = b.unpack_state(state)[0]
    # the start state is the double draw rounded once. The device and host sine and cosine
    # may each round differently by an ulp; in the quaternion (sums of products of them,
    # with cancellation in the small components) that shows at the scale of the unit norm
    ref = ref_s[:, :19].T
    scale = np.abs(ref)
    scale[3:7] = 1.0
    ulp = np.spacing(scale.astype(dt)).astype(np.float64)
    assert np.all(np.abs(dev_s - ref) <= (2 if dt is np.float32 else 8) * ulp)
    assert np.array_equal(dev_s[7:13], ref[7:13].astype(dt))   # velocities: no transcendental
    ref_o = S.observe(ref_s, ref_t, 6)
    assert rel_err(b.unpack_state(obs)[0].T, ref_o, np.ones(ref_o.shape[0], bool)) <= tol
    ep, et = st.episodes()
    assert not ep.any() and not et.any()
    st.close()
    b.close()
    t.cuda.synchronize()


@pytest.mark.parametrize("precision,tol,margin", [(mgx.FP32, 2e-4, 2e-3), (mgx.FP64, 1e-9, 1e-7)])
def test_rollout_with_resets_matches_the_oracle(precision, tol, margin):
    """1000 environments, 120 task steps: truncation every 40 steps, terminations by
    distance (targets up to 3.5 m away, d_max 2.6) and by lean (commands up to 1.2, lean
    limit 0.6 rad), each followed by the next episode's draw."""
    w = synth.randomised(n=1000, steps=10)
    res = run_both(w, DESC, 120, precision)
    stats = check(res, DESC, tol, margin, name=f"plain {precision}")
    assert stats["terminated"] > 100 and stats["resets"] > 2000, stats


def test_every_step_restarts():
    """Episodes of one step: every lane restarts at every step, so whole waves take the
    per-lane draw (the rollout tests take the wave-spread draw for scattered terminations
    and the per-lane one at the synchronised truncations)."""
    w = synth.randomised(n=1000, steps=10)
    desc = dict(DESC, max_steps=1)
    res = run_both(w, desc, 6)
    stats = check(res, desc, 2e-4, 2e-3, name="one-step episodes")
    assert stats["resets"] >= 0.9 * 6 * 1000


@pytest.mark.parametrize("n", [1, 65])
def test_ragged_segments(n):
    """One environment (63 padding lanes in its wave) and 65 (a second wave with one valid
    lane): the padding lanes stay in the wave for the spread restarts and report nothing."""
    t = torch()
    w = synth.randomised(n=n, steps=10)
    desc = dict(DESC, max_steps=7)
    res = run_both(w, desc, 30)
    check(res, desc, 2e-4, 2e-3, name=f"n={n}")
    b = make_batch(w)
    st = mgx.Station(b, **desc)
    st.reset(7)
    out = st.step(b.gen_actions(3, seed=2))
    rew = out["reward"].cpu().numpy()
    flags = out["terminated"].cpu().numpy() | out["truncated"].cpu().numpy()
    assert not rew[:, n:].any() and not flags[:, n:].any()
    st.close()
    b.close()
    t.cuda.synchronize()


def test_mixed_batch_with_substeps():
    """Five classes (4, 5, 6, 8, 8 thrusters) in one batch, three dynamics steps per task
    step: slots, per-class constants and the held command."""
    w = synth.heterogeneous(scale=0.02, steps=10)
    desc = dict(DESC, substeps=3, max_steps=25)
    res = run_both(w, desc, 60)
    check(res, desc, 3e-4, 2e-3, name="mixed")


@pytest.mark.parametrize("make", ["propellers", "rudders", "payload"])
@pytest.mark.parametrize("precision,tol,margin", [(mgx.FP32, 5e-4, 2e-3), (mgx.FP64, 1e-9, 1e-7)])
def test_variant_bodies(make, precision, tol, margin):
    w = getattr(synth, make)(n=700, steps=10)
    desc = dict(DESC, max_steps=30)
    res = run_both(w, desc, 45, precision)
    check(res, desc, tol, margin, name=f"{make} {precision}")


def test_vector_env_interface():
    """The Gym-style view: shapes and dtypes, the same numbers as the flat interface, a
    repeatable reset, and final observations on truncation."""
    t = torch()
    w = synth.plain_small(n=300)
    cls = w.classes[0]
    env = mgx.VecStationKeeping(cls, w.params, 300, w.dt, **dict(DESC, max_steps=3, d_max=100.0, tilt_max=3.0))
    obs, info = env.reset(seed=5)
    assert obs.shape == (300, 19) and obs.dtype == t.float32 and info == {}
    first = obs.clone()
    a = t.full((300, 6), 0.25, device=obs.device)
    for k in range(3):
        obs, r, term, trunc, info = env.step(a)
        assert r.shape == (300,) and term.dtype == t.bool and trunc.shape == (300,)
        assert not term.any() and bool(trunc.all()) == (k == 2)
    # after truncation every environment is in episode 1; final_obs is the episode's last
    ep, et = env.task.episodes()
    assert (ep == 1).all() and (et == 0).all()
    envs = oracle.make_envs(cls, w.params, w.dt)
    o = S.StationOracle(S.StationDesc(**dict(DESC, max_steps=3, d_max=100.0, tilt_max=3.0)), envs, 6)
    o.reset(5)
    for _ in range(3):
        ro, rr, _, _, rf = o.step(np.full((300, 6), 0.25))
    assert np.max(np.abs(info["final_obs"].cpu().numpy() - rf)) < 1e-4
    assert np.max(np.abs(obs.cpu().numpy() - ro)) < 1e-5
    obs2, _ = env.reset(seed=5)
    assert t.equal(obs2, first)
    env.close()


def test_full_size_sampled():
    """65,536 environments of the randomised workload, 200 task steps (five episodes each
    by truncation, plus terminations); 256 sampled environments against the oracle."""
    t = torch()
    w = synth.randomised(n=65536, steps=10)
    desc = dict(DESC, max_steps=40)
    b = make_batch(w)
    st = mgx.Station(b, **desc)
    st.reset(99)
    T = 200
    acts = b.gen_actions(T, seed=17)
    out = st.step(acts)
    t.cuda.synchronize()
    rng = np.random.default_rng(4)
    ids = np.sort(rng.choice(65536, 256, replace=False))
    ids[0], ids[-1] = 0, 65535
    envs = oracle.make_envs(w.classes[0], w.params.subset(ids), w.dt)
    o = S.StationOracle(S.StationDesc(**desc), envs, 6, ids=ids)
    o.reset(99)
    host_acts = b.unpack_actions(acts.cpu().numpy().astype(np.float64))[0]   # [T, m, n]
    obs_all = out["obs"].cpu().numpy().astype(np.float64)
    rew = out["reward"].cpu().numpy().astype(np.float64)
    term = out["terminated"].cpu().numpy().astype(bool)
    trunc = out["truncated"].cpu().numpy().astype(bool)
    ok = np.ones(ids.size, bool)
    n_reset = 0
    for k in range(T):
        ro, rr, rt, rtr, rf = o.step(host_acts[k][:, ids].T)
        ok = decide(ok, term[k, ids], rt, trunc[k, ids], rtr, rf, desc, 2e-3, f"step {k}")
        dev_o = b.unpack_state(obs_all[k])[0][:, ids].T
        assert rel_err(dev_o, ro, ok) <= 2e-4, k
        assert np.max(np.abs(rew[k, ids][ok] - rr[ok]), initial=0) <= 2e-4, k
        n_reset += int(np.sum((rt | rtr)[ok]))
    assert ok.mean() >= 0.99 and n_reset > 5 * 0.99 * ids.size
    st.close()
    b.close()


def test_parameters_redrawn_at_episode_start():
    """Domain randomisation at episode start: after the reset every environment holds the
    parameters of its episode 0; after task steps with scattered terminations, exactly the
    environments that restarted hold those of their new episode (the oracle sampler at
    epoch = episode index), and the others keep theirs."""
    import test_gpu_dr as G
    from oracle import dr_sampler as D
    t = torch()
    w = synth.randomised(n=700, steps=10)
    b = make_batch(w)
    st = mgx.Station(b, **DESC)
    nominal = np.stack([G.nominal_of(c) for c in w.classes])
    st.reset(7)
    st.resample(G.SPEC, nominal, seed=21)
    p0 = b.get_params()
    G.compare(p0, G.oracle_params(w.classes, w.n_envs, G.SPEC, 21, 0), mgx.FP32)
    out = st.step(b.gen_actions(4, seed=5))
    st.resample(G.SPEC, nominal, seed=21)
    p1 = b.get_params()
    t.cuda.synchronize()
    ended = (out["terminated"] | out["truncated"]).cpu().numpy().any(axis=0)[:700].astype(bool)
    ep, _ = st.episodes()
    assert 0 < ended.sum() < 700 and np.array_equal(ep > 0, ended)
    for k in ("mass", "added", "dlin", "dquad", "buoy", "current"):
        assert np.array_equal(p1[k][..., ~ended], p0[k][..., ~ended]), k
    ids = np.where(ended)[0]
    ref = {k: np.zeros_like(p1[k][..., ids]) for k in p1}
    for e in np.unique(ep[ids]):
        sel = ep[ids] == e
        r = D.sample(G.SPEC, nominal[0], ids[sel], 21, int(e))
        for k in ref:
            ref[k][..., sel] = r[k]
    G.compare(p1, ref, mgx.FP32, cols=ids)
    st.close()
    b.close()


def test_redraw_without_restarts_changes_nothing():
    """A call in which no episode ends leaves every parameter as it was, and a prebuilt
    DrSpec draws what its dictionary draws."""
    import test_gpu_dr as G
    t = torch()
    w = synth.randomised(n=300, steps=10)
    b = make_batch(w)
    st = mgx.Station(b, **dict(DESC, d_max=1e6, tilt_max=3.1, max_steps=1000))
    nominal = np.stack([G.nominal_of(c) for c in w.classes])
    st.reset(3)
    st.resample(mgx.dr_spec(G.SPEC), nominal, seed=8)
    p0 = b.get_params()
    G.compare(p0, G.oracle_params(w.classes, w.n_envs, G.SPEC, 8, 0), mgx.FP32)
    out = st.step(b.gen_actions(3, seed=1))
    assert not (out["terminated"] | out["truncated"]).any()
    st.resample(G.SPEC, nominal, seed=8)
    p1 = b.get_params()
    for k in p0:
        assert np.array_equal(p0[k], p1[k]), k
    st.close()
    b.close()
    t.cuda.synchronize()


def test_errors():
    t = torch()
    w = synth.plain_small(n=64)
    b = make_batch(w)
    with pytest.raises(mgx.MgxError):
        mgx.Station(b, **dict(DESC, sigma_p=0.0))
    with pytest.raises(mgx.MgxError):
        mgx.Station(b, **dict(DESC, substeps=0))
    st = mgx.Station(b, **DESC)
    with pytest.raises(mgx.MgxError):      # before reset
        st.step(b.empty_actions(1))
    st.reset(1)
    with pytest.raises(mgx.MgxError):      # the batch outlives its task
        mgx.mgx_batch_destroy(b.h)
    st.close()
    b.close()
    t.cuda.synchronize()
