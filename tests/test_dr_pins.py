"""Pins for the domain-randomisation sampler of ``oracle/dr_sampler.py`` (Sec. III-C):
its draws follow the distributions they claim to. Each check compares sample statistics
with the distribution's closed form at a CLT-sized tolerance (about five standard
errors), on 2^16 environments."""
import numpy as np
import pytest
from scipy import stats

from oracle import dr_sampler as D

N = 1 << 16
NOM = np.arange(1.0, 24.0)        # mass 1, added 2..7, dlin 8..13, dquad 14..19, buoy 20, current 21..23
IDS = np.arange(N)


def test_uniform_distribution():
    s = D.sample({"mass": {"kind": D.UNIFORM, "lo": 0.8, "hi": 1.2}}, NOM, IDS, 5, 0)["mass"]
    assert s.min() >= 0.8 and s.max() < 1.2
    assert abs(s.mean() - 1.0) < 5 * 0.4 / np.sqrt(12 * N)
    assert abs(s.var() - 0.4 ** 2 / 12) < 5 * 0.4 ** 2 / 12 * np.sqrt(0.8 / N)
    assert stats.kstest(s, "uniform", args=(0.8, 0.4)).pvalue > 1e-4


def test_gaussian_distribution_and_clip():
    wide = {"kind": D.GAUSSIAN, "mean": 0.1, "std": 0.3, "lo": -5, "hi": 5, "relative": 0}
    s = D.sample({"current": wide}, NOM, IDS, 6, 0)["current"]
    for a in range(3):
        assert abs(s[a].mean() - 0.1) < 5 * 0.3 / np.sqrt(N)
        assert abs(s[a].std() - 0.3) < 5 * 0.3 / np.sqrt(2 * N)
        assert stats.kstest(s[a], "norm", args=(0.1, 0.3)).pvalue > 1e-4
    # clipped at one standard deviation: the share sitting on each bound is Phi(-1)
    tight = dict(wide, lo=-0.2, hi=0.4)
    s = D.sample({"current": tight}, NOM, IDS, 6, 0)["current"][0]
    p = stats.norm.cdf(-1.0)
    for frac in ((s == -0.2).mean(), (s == 0.4).mean()):
        assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / N)
    assert s.min() == -0.2 and s.max() == 0.4


def test_piecewise_distribution():
    edges, w = [0.5, 0.9, 1.0, 1.3, 2.0], [2.0, 0.0, 5.0, 1.0]
    s = D.sample({"dquad": {"kind": D.PIECEWISE, "edges": edges, "weights": w, "shared": 1}}, NOM, IDS, 7, 0)
    x = s["dquad"][0] / NOM[13]
    assert np.allclose(s["dquad"], NOM[13:19, None] * x[None, :], rtol=1e-15, atol=0)   # shared draw
    counts = np.histogram(x, bins=edges)[0] / N
    for c, wk in zip(counts, w):
        p = wk / sum(w)
        assert abs(c - p) < 5 * np.sqrt(p * (1 - p) / N) + 1e-12
    for k in (0, 2, 3):                    # uniform inside each bin
        inb = x[(x >= edges[k]) & (x < edges[k + 1])]
        half = (edges[k + 1] - edges[k]) / 2
        assert abs(inb.mean() - (edges[k] + half)) < 5 * half / np.sqrt(3 * inb.size)
    assert not np.any((x >= 0.9) & (x < 1.0))


def test_groups_slots_and_determinism():
    spec = {"mass": {"kind": D.UNIFORM, "lo": 0.5, "hi": 1.5},
            "added": {"kind": D.UNIFORM, "lo": 0.5, "hi": 1.5, "shared": 0},
            "buoy": {"kind": D.FIXED}}
    a = D.sample(spec, NOM, IDS[:1000], 9, 3)
    b = D.sample(spec, NOM, IDS[:1000], 9, 3)
    c = D.sample(spec, NOM, IDS[:1000], 9, 4)
    assert np.array_equal(a["added"], b["added"]) and not np.array_equal(a["added"], c["added"])
    assert np.all(a["buoy"] == NOM[19]) and np.all(a["dlin"] == NOM[7:13, None])
    f = a["added"] / NOM[1:7, None]
    assert np.abs(np.corrcoef(f)[np.triu_indices(6, 1)]).max() < 0.15      # independent entries
    # a spec change in one group leaves the other groups' draws unchanged
    d = D.sample(dict(spec, mass={"kind": D.GAUSSIAN, "mean": 1, "std": 0.1, "lo": 0.5, "hi": 1.5}), NOM,
                 IDS[:1000], 9, 3)
    assert np.array_equal(a["added"], d["added"]) and not np.array_equal(a["mass"], d["mass"])
