"""The seeded input generator: published Philox vectors, determinism, ranges, exactness."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = synth.philox4x32(np.array(v[0:4], dtype=np.uint64), np.array(v[4:6], dtype=np.uint64))
        assert [int(x) for x in out] == v[6:10]


def test_actions_exact_and_in_range():
    a = synth.actions(300, 8, 7)
    assert a.dtype == np.float32 and a.shape == (7, 8, 300)
    assert a.min() >= -1.0 and a.max() < 1.0
    # exactly k * 2^-23
    k = a.astype(np.float64) * 2 ** 23
    assert np.array_equal(k, np.round(k))
    # a window of rows and envs equals the same slice of the full stream
    b = synth.actions(100, 8, 3, env_offset=50, row_offset=2)
    assert np.array_equal(b, a[2:5, :, 50:150])
    assert abs(float(a.mean())) < 0.02 and abs(float(a.std()) - 1 / np.sqrt(3)) < 0.01


def test_determinism_and_ranges():
    c1 = synth.plain_class()
    c2 = synth.plain_class()
    assert np.array_equal(c1.r, c2.r) and c1.mass == c2.mass
    assert 10 <= c1.mass <= 15
    assert np.all((c1.k >= 20) & (c1.k <= 40)) and np.all((c1.tau >= 0.05) & (c1.tau <= 0.15))
    assert 1.0 <= c1.buoy / (c1.mass * c1.g0) <= 1.02 + 1e-6
    assert -0.02 <= c1.rb[2] <= 0.0
    diag = np.array([c1.mass] * 3 + list(c1.inertia))
    assert np.all((c1.added / diag >= 0.1 - 1e-6) & (c1.added / diag <= 0.5 + 1e-6))
    assert synth.layout_conditioning(c1.r, c1.e) >= 0.05
    for x in (c1.r, c1.e, c1.k, c1.added, c1.dlin):
        assert np.array_equal(x, x.astype(np.float32).astype(np.float64))


def test_randomisation_and_screen():
    c = synth.plain_class()
    p = synth.randomised_params(c, 4096)
    assert np.all(np.abs(p.mass / c.mass - 1) <= 0.2 + 1e-6)
    assert np.all(np.abs(p.added / c.added[:, None] - 1) <= 0.2 + 1e-6)
    r = p.dlin / c.dlin[:, None]
    assert np.allclose(r, r[0:1], rtol=1e-6)                   # one damping factor per env
    assert np.allclose(p.dquad / c.dquad[:, None], r[0:1], rtol=1e-6)
    assert abs(p.current.std() - 0.3) < 0.02
    ratio = synth.damping_step_ratio(p.mass, c.inertia, p.added, p.dlin, p.dquad, p.buoy, c.g0, c.rb,
                                     c.k, c.r, c.e, 0.01, current_bound=4 * 0.3 * np.sqrt(3))
    assert np.all(ratio <= 1.0)


def test_initial_state():
    s = synth.initial_state(20000, 6)
    assert np.allclose(np.linalg.norm(s.q, axis=0), 1, atol=1e-6)
    assert abs(s.nu.std() - 0.2) < 0.01 and np.all(s.p == 0) and np.all(s.n == 0)
    # uniform on S^3: E[w^2] = 1/4
    assert abs((s.q ** 2).mean() - 0.25) < 0.01


def test_heterogeneous_layouts():
    cs = synth.hetero_classes()
    assert [c.m for c in cs] == [4, 5, 6, 8, 8]
    for c in cs:
        assert synth.layout_conditioning(c.r, c.e) >= 0.05


def test_serving_trace():
    reqs = synth.serving_trace(duration=10.0)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0) and abs(len(reqs) / 10.0 - 200) < 30
    n = np.array([r["n"] for r in reqs])
    assert n.min() >= 64 and n.max() <= 16384
    h = np.array([r["horizon"] for r in reqs])
    assert h.min() >= 1 and h.max() <= 500
    assert 0.3 < np.mean([r["continues"] for r in reqs]) < 0.6
