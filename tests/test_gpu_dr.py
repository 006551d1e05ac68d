"""On-device domain randomisation against the oracle sampler: the parameters a batch draws
are the oracle's (bit-exact after rounding to the batch precision for uniform, piecewise
and fixed groups; the Gaussian groups within one unit in the last place in float32 and
eight in float64, since the device and host logarithm and cosine may each round
differently by an ulp, which the Box-Muller transform carries into the draw), subsets and
epochs redraw only what
they name, range updates reuse the same uniforms, and the dynamics run on the drawn
parameters match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dr_sampler as D
from paper_2503_09203_amd import mgx

from gpu_helpers import torch
from parity import component_errors

pytestmark = pytest.mark.gpu

SPEC = {
    "mass": {"kind": D.UNIFORM, "lo": 0.8, "hi": 1.2},
    "added": {"kind": D.GAUSSIAN, "mean": 1.0, "std": 0.1, "lo": 0.7, "hi": 1.3},
    "dlin": {"kind": D.PIECEWISE, "edges": [0.5, 0.9, 1.0, 1.3, 2.0], "weights": [2.0, 0.0, 5.0, 1.0], "shared": 1},
    "dquad": {"kind": D.UNIFORM, "lo": 5.0, "hi": 50.0, "relative": 0},
    "buoy": {"kind": D.UNIFORM, "lo": 0.99, "hi": 1.03},
    "current": {"kind": D.GAUSSIAN, "mean": 0.0, "std": 0.3, "lo": -1.0, "hi": 1.0, "relative": 0},
}


def nominal_of(c):
    return np.concatenate([[c.mass], c.added, c.dlin, c.dquad, [c.buoy], np.zeros(3)])


def oracle_params(classes, ns, spec, seed, epoch, ids=None):
    out = {k: [] for k in ("mass", "added", "dlin", "dquad", "buoy", "current")}
    off = 0
    for c, n in zip(classes, ns):
        gids = np.arange(off, off + n) if ids is None else ids[(ids >= off) & (ids < off + n)]
        s = D.sample(spec, nominal_of(c), gids, seed, epoch)
        for k in out:
            out[k].append(s[k])
        off += n
    return {k: np.concatenate(v, axis=-1) for k, v in out.items()}


def compare(dev, ref, precision, cols=None):
    dt = np.float32 if precision == mgx.FP32 else np.float64
    for k in ("mass", "added", "dlin", "dquad", "buoy", "current"):
        d = dev[k] if cols is None else dev[k][..., cols]
        r = ref[k].astype(dt).astype(np.float64)
        if SPEC.get(k, {}).get("kind") == D.GAUSSIAN:
            ulp = np.spacing(np.abs(r).astype(dt)).astype(np.float64) * (1 if dt is np.float32 else 8)
            assert np.all(np.abs(d - r) <= ulp), (k, np.abs(d - r).max())
            assert np.mean(d == r) > (0.99 if dt is np.float32 else 0.5), k
        else:
            assert np.array_equal(d, r), (k, np.abs(d - r).max())


@pytest.mark.parametrize("precision", [mgx.FP32, mgx.FP64])
def test_resample_matches_the_oracle_sampler(precision):
    w = synth.heterogeneous(scale=0.05, steps=8)
    b = mgx.Batch(w.classes, w.n_envs, w.dt, precision)
    nominal = np.stack([nominal_of(c) for c in w.classes])
    b.resample(SPEC, nominal, seed=11, epoch=0)
    compare(b.get_params(), oracle_params(w.classes, w.n_envs, SPEC, 11, 0), precision)
    b.close()


def test_subsets_and_epochs_redraw_only_what_they_name():
    w = synth.heterogeneous(scale=0.05, steps=8)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    nominal = np.stack([nominal_of(c) for c in w.classes])
    b.resample(SPEC, nominal, seed=3, epoch=0)
    before = b.get_params()
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(w.n_total, 500, replace=False))
    b.resample(SPEC, nominal, env_ids=ids, seed=3, epoch=1)
    after = b.get_params()
    keep = np.setdiff1d(np.arange(w.n_total), ids)
    for k in before:
        assert np.array_equal(before[k][..., keep], after[k][..., keep]), k
    compare(after, oracle_params(w.classes, w.n_envs, SPEC, 3, 1, ids), mgx.FP32, cols=ids)
    b.close()


def test_range_update_reuses_the_uniforms():
    """A curriculum widens a uniform range from +-10% to +-40%: at the same seed and epoch
    each environment's deviation from the nominal grows by exactly the same factor."""
    w = synth.randomised(n=4096, steps=8)
    c = w.classes[0]
    b = mgx.Batch([c], [4096], w.dt, mgx.FP64)
    nominal = nominal_of(c)[None]
    devs = []
    for half in (0.1, 0.4):
        b.resample({"mass": {"kind": D.UNIFORM, "lo": 1 - half, "hi": 1 + half}}, nominal, seed=5, epoch=2)
        devs.append(b.get_params()["mass"] / c.mass - 1)
    assert np.allclose(devs[1], 4 * devs[0], rtol=1e-12, atol=1e-15)
    assert 0.09 < np.abs(devs[0]).max() <= 0.1 and 0.36 < np.abs(devs[1]).max() <= 0.4
    b.close()


def test_dynamics_on_drawn_parameters_match_the_oracle():
    t = torch()
    w = synth.heterogeneous(scale=0.05, steps=32)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    nominal = np.stack([nominal_of(c) for c in w.classes])
    b.resample(SPEC, nominal, seed=7, epoch=0)
    b.reset(seed=9)
    acts = w.actions(4)
    dev_acts = t.tensor(b.pack_actions(acts), dtype=b.dtype, device=b.device)
    for _ in range(2):
        b.step(dev_acts, 16, hold=10)
    got = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))
    drawn = b.get_params()          # the oracle runs on the stored (rounded) values
    off = 0
    for ci, (c, n) in enumerate(zip(w.classes, w.n_envs)):
        p = synth.EnvParams(drawn["mass"][off:off + n], drawn["added"][:, off:off + n], drawn["dlin"][:, off:off + n],
                            drawn["dquad"][:, off:off + n], drawn["buoy"][off:off + n],
                            drawn["current"][:, off:off + n])
        envs = oracle.make_envs(c, p, w.dt)
        st = synth.initial_state(n, c.m, 9, off)
        x = oracle.pack_state(st.p, st.q, st.nu, st.n)
        x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(acts[ci]), 10, 32)
        err = component_errors(got[ci], oracle.unpack_state(x, c.m))
        assert err.max() <= 1e-4, (ci, err.max())
        off += n
    b.close()


def test_bad_specs_are_refused():
    w = synth.randomised(n=256, steps=8)
    c = w.classes[0]
    b = mgx.Batch([c], [256], w.dt)
    nominal = nominal_of(c)[None]
    with pytest.raises(mgx.MgxError) as e:
        b.resample(SPEC, nominal, env_ids=[1, 2], seed=1)      # subset before any parameters
    assert e.value.status == mgx.MGX_E_STATE
    bad = [{"mass": {"kind": D.UNIFORM, "lo": -0.1, "hi": 1.2}},
           {"dlin": {"kind": D.PIECEWISE, "edges": [1.0, 0.5], "weights": [1.0]}},
           {"dlin": {"kind": D.PIECEWISE, "edges": [0.5, 1.0], "weights": [0.0]}},
           {"added": {"kind": D.GAUSSIAN, "mean": 1.0, "std": -1.0, "lo": 0.5, "hi": 1.5}},
           {"buoy": {"kind": 9}}]
    for spec in bad:
        with pytest.raises(mgx.MgxError) as e:
            b.resample(spec, nominal, seed=1)
        assert e.value.status == mgx.MGX_E_INVALID, spec
    b.resample(SPEC, nominal, seed=1)
    with pytest.raises(mgx.MgxError):
        b.resample(SPEC, nominal, env_ids=[256], seed=1)
    b.close()


def test_resample_rebuilds_payload_records():
    """Drawn parameters of a payload class go through the full dt M^-1 inversion: the
    dynamics on them match the oracle."""
    t = torch()
    w = synth.payload(n=700, steps=32)
    c = w.classes[0]
    b = mgx.Batch([c], [700], w.dt)
    b.resample(SPEC, nominal_of(c)[None], seed=4, epoch=0)
    b.reset(seed=2)
    acts = w.actions(4)
    b.step(t.tensor(b.pack_actions(acts), dtype=b.dtype, device=b.device), 32, hold=10)
    got = b.unpack_state(b.get_state().cpu().numpy().astype(np.float64))[0]
    d = b.get_params()
    p = synth.EnvParams(d["mass"], d["added"], d["dlin"], d["dquad"], d["buoy"], d["current"])
    envs = oracle.make_envs(c, p, w.dt)
    st = synth.initial_state(700, c.m, 2)
    x = oracle.pack_state(st.p, st.q, st.nu, st.n)
    x, _, _ = oracle.rollout(envs, x, oracle.pack_actions(acts[0]), 10, 32)
    assert component_errors(got, oracle.unpack_state(x, c.m)).max() <= 1e-4
    b.close()
