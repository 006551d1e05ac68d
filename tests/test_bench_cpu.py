"""Host-side checks of bench.py that need no GPU: the one-GPU refusal, the algorithmic byte
counts it divides by, and the recorded hardware-counter traffic it reports only while the
kernel sources match the ones the counters were taken with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_single_step_bytes_per_env_step():
    # m = 6, FP32: state read and written (2 x 19 x 4), record 30 x 4, one action row 6 x 4
    assert bench.bytes_per_env_step(6, 1, 10) == 2 * 19 * 4 + 30 * 4 + 6 * 4
    # payload records have 45 rows
    assert bench.bytes_per_env_step(6, 1, 10, rec_len=45) == 2 * 19 * 4 + 45 * 4 + 6 * 4


def test_recorded_traffic_follows_the_sources():
    t = bench.recorded_traffic()
    if t:  # recorded for exactly these sources
        assert set(t) == {1, 16} and all(v > 0 for v in t.values())
    line = [l for l in open(os.path.join(ROOT, "profiles", "k_step_dr65536x1000.md")) if l.startswith("traffic:")]
    assert len(line) == 1
    assert (bench.kernel_sources_sha256() in line[0]) == bool(t)


def test_recorded_adjoint_traffic_follows_the_sources():
    t = bench.recorded_adjoint_traffic()
    if t:  # recorded for exactly these sources
        assert set(t) == {"fwd", "bwd"} and all(v > 0 for v in t.values())
    line = [l for l in open(os.path.join(ROOT, "profiles", "k_rollout_adjoint8192x256.md")) if l.startswith("traffic:")]
    assert len(line) == 1
    assert (bench.kernel_sources_sha256(bench.ADJOINT_SOURCES) in line[0]) == bool(t)


def test_recorded_station_traffic_follows_the_sources():
    t = bench.recorded_station_traffic()
    if t:  # recorded for exactly these sources
        assert set(t) == {1, 100} and all(v > 0 for v in t.values())
    line = [l for l in open(os.path.join(ROOT, "profiles", "k_station_step65536.md")) if l.startswith("traffic:")]
    assert len(line) == 1
    assert (bench.kernel_sources_sha256(bench.STATION_SOURCES) in line[0]) == bool(t)


def test_recorded_traffic_of_every_step_body_follows_the_sources():
    for wl, path in bench.VARIANT_TRAFFIC_PROFILES.items():
        t = bench.recorded_traffic(wl)
        if t:
            assert set(t) == {1, 16} and all(v > 0 for v in t.values()), wl
        line = [l for l in open(path) if l.startswith("traffic:")]
        assert len(line) == 1, wl
        assert (bench.kernel_sources_sha256() in line[0]) == bool(t), wl


def test_recorded_hetero_traffic_follows_the_sources():
    t = bench.recorded_hetero_traffic()
    if t:
        assert set(t) == {32} and all(v > 0 for v in t.values())
    line = [l for l in open(os.path.join(ROOT, "profiles", "k_persistent_hetero70512x1024.md")) if l.startswith("traffic:")]
    assert len(line) == 1
    assert (bench.kernel_sources_sha256(bench.HETERO_SOURCES) in line[0]) == bool(t)
