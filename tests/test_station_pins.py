"""Pins of the station-keeping task oracle (``oracle/station.py``) against what the
mathematics fixes: the quaternion algebra's defining products, textbook elementary
rotations and the Z-Y-X Euler composition, worked examples of the body-frame target and
the attitude error, the attitude error's angle against the trace of R*^T R, closed forms
of the reward, the termination thresholds, and the episode bookkeeping (truncation,
auto-reset to the next episode's draw, a non-finite state, held commands over substeps)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import station as S


def elem(axis, a):
    c, s = np.cos(a), np.sin(a)
    if axis == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == 1:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def test_hamilton_basis_products():
    one, i, j, k = np.eye(4)
    mul = S.quat_mul
    assert np.array_equal(mul(i, i), -one) and np.array_equal(mul(j, j), -one) and np.array_equal(mul(k, k), -one)
    assert np.array_equal(mul(i, j), k) and np.array_equal(mul(j, k), i) and np.array_equal(mul(k, i), j)
    assert np.array_equal(mul(j, i), -k) and np.array_equal(mul(mul(i, j), k), -one)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rotation_of_axis_quaternion_is_textbook_matrix(axis):
    for a in (-2.5, -0.3, 0.0, 0.7, 3.0):
        assert np.allclose(S.rot(S.quat_axis(np.array(a), axis)), elem(axis, a), atol=1e-15)


def test_rotation_composes_like_the_product():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(50, 4)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(50, 4)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    assert np.allclose(S.rot(S.quat_mul(a, b)), S.rot(a) @ S.rot(b), atol=1e-14)
    # the C oracle's own rotation agrees with this one
    for q in a[:5]:
        assert np.allclose(oracle.rotation(q), S.rot(q), atol=1e-15)


def test_episode_start_is_zyx_euler_of_the_draws():
    d = S.StationDesc(target_box=1.5, tilt0=0.3, v0=0.2)
    ids = np.arange(100, 164)
    s, tg = S.episode_start(d, 42, ids, 5, 6)
    u = S.start_uniforms(42, ids, 5)
    psi, phi, th = np.pi * (2 * u[:, 4] - 1), 0.3 * (2 * u[:, 5] - 1), 0.3 * (2 * u[:, 6] - 1)
    for e in range(ids.size):
        R = elem(2, psi[e]) @ elem(1, th[e]) @ elem(0, phi[e])
        assert np.allclose(S.rot(s[e, 3:7]), R, atol=1e-14)
        # the angles come back from the matrix (Z-Y-X extraction)
        assert np.isclose(np.arctan2(R[1, 0], R[0, 0]), psi[e], atol=1e-12)
        assert np.isclose(-np.arcsin(R[2, 0]), th[e], atol=1e-12)
        assert np.isclose(np.arctan2(R[2, 1], R[2, 2]), phi[e], atol=1e-12)
        assert np.allclose(S.rot(tg[e, 3:7]), elem(2, np.pi * (2 * u[e, 3] - 1)), atol=1e-14)
    assert np.all(np.abs(tg[:, 0:3]) <= 1.5) and np.all(s[:, 0:3] == 0) and np.all(s[:, 13:] == 0)
    assert np.all(np.abs(s[:, 7:13]) <= 0.2)
    assert np.allclose(np.linalg.norm(s[:, 3:7], axis=1), 1.0, atol=1e-15)
    # episodes and seeds give independent draws; the same key and counter the same draw
    s2, _ = S.episode_start(d, 42, ids, 6, 6)
    s3, _ = S.episode_start(d, 43, ids, 5, 6)
    s4, _ = S.episode_start(d, 42, ids[3:4], 5, 6)
    assert not np.allclose(s[:, 3:7], s2[:, 3:7]) and not np.allclose(s[:, 3:7], s3[:, 3:7])
    assert np.array_equal(s4[0], s[3])


def test_start_draw_distributions():
    """Over 20,000 draws: target coordinates and start velocities uniform on [-b, b] and
    [-v0, v0] (mean 0, variance b^2/3), target and start yaw uniform on the circle (mean
    resultant length near 0), roll and pitch within +-t0 with variance t0^2/3."""
    d = S.StationDesc(target_box=1.5, tilt0=0.3, v0=0.2)
    n = 20000
    s, tg = S.episode_start(d, 5, np.arange(n), 2, 6)
    se = lambda var: 4 * np.sqrt(var / n)   # four standard errors of a mean
    for x, h in ((tg[:, 0:3], 1.5), (s[:, 7:13], 0.2)):
        assert np.all(np.abs(x.mean(axis=0)) < se(h * h / 3))
        assert np.allclose(x.var(axis=0), h * h / 3, rtol=0.05)
    yaw_t = 2 * np.arctan2(tg[:, 6], tg[:, 3])
    R = S.rot(s[:, 3:7])
    yaw0 = np.arctan2(R[:, 1, 0], R[:, 0, 0])
    for a in (yaw_t, yaw0):
        assert abs(np.mean(np.exp(1j * a))) < 4 / np.sqrt(n)
        assert np.allclose(np.var(np.mod(a + np.pi, 2 * np.pi) - np.pi), np.pi ** 2 / 3, rtol=0.05)
    pitch, roll = -np.arcsin(R[:, 2, 0]), np.arctan2(R[:, 2, 1], R[:, 2, 2])
    for a in (pitch, roll):
        assert np.all(np.abs(a) <= 0.3 + 1e-12) and np.allclose(a.var(), 0.09 / 3, rtol=0.05)


def test_start_uniforms_use_the_published_generator():
    # counter (g, k, j, 0) at key (seed, 8 << 24); word pairs (w0, w1), (w2, w3) as 53-bit uniforms
    u = S.start_uniforms(7, [12], [3])
    ctr = np.array([[12, 3, 4, 0]], dtype=np.uint64)
    w = synth.philox4x32(ctr, np.array([7, 8 << 24], dtype=np.uint64))[0]
    assert u[0, 8] == synth.u53(w[0], w[1]) and u[0, 9] == synth.u53(w[2], w[3])


def test_observation_worked_example():
    # at p = (1, 0, 0) turned 90 degrees left (body x = world y), target at (1, 2, 0):
    # the target lies 2 m straight ahead
    q = S.quat_axis(np.array(np.pi / 2), 2)
    st = np.zeros((1, 21)); st[0, 0] = 1.0; st[0, 3:7] = q; st[0, 7:13] = np.arange(6); st[0, 13:16] = [0.1, 0.2, 0.3]
    tg = np.zeros((1, 7)); tg[0, 0:3] = [1.0, 2.0, 0.0]; tg[0, 3] = 1.0
    o = S.observe(st, tg, 3)
    assert np.allclose(o[0, 0:3], [2.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(o[0, 3:7], [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)], atol=1e-15)
    assert np.array_equal(o[0, 7:13], np.arange(6)) and np.array_equal(o[0, 13:16], [0.1, 0.2, 0.3])
    # at the target attitude the error is the identity
    tg[0, 3:7] = q
    assert np.allclose(S.observe(st, tg, 3)[0, 3:7], [1, 0, 0, 0], atol=1e-15)


def test_attitude_error_angle_matches_trace_formula():
    rng = np.random.default_rng(9)
    q = rng.normal(size=(200, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    t = rng.normal(size=(200, 4)); t /= np.linalg.norm(t, axis=1, keepdims=True)
    qe = S.attitude_error(q, t)
    assert np.all(qe[:, 0] >= 0)
    ang = 2 * np.arccos(np.clip(qe[:, 0], -1, 1))
    Rt, R = S.rot(t), S.rot(q)
    cos_tr = (np.einsum("nji,nji->n", Rt, R) - 1) / 2   # tr(Rt^T R)
    assert np.allclose(np.cos(ang), cos_tr, atol=1e-12)
    # and the error rotation takes the target frame to the body frame: R = Rt R(qe)
    assert np.allclose(Rt @ S.rot(qe), R, atol=1e-13)


def test_reward_closed_forms():
    d = S.StationDesc(sigma_p=0.5, w_att=0.5, w_act=0.01)
    st = np.zeros((4, 21)); st[:, 3] = 1.0
    tg = np.zeros((4, 7)); tg[:, 3] = 1.0
    st[1, 0] = 0.5                                    # d = sigma_p
    tg[2, 3:7] = [0.0, 0.0, 0.0, 1.0]                 # half a turn of yaw away: q_e,w = 0
    a = np.zeros((4, 6)); a[3] = [1, -1, 0.5, 0, 0, 0]
    r, term = S.reward_done(d, st, tg, a, 6)
    assert r[0] == 1.0
    assert np.isclose(r[1], np.exp(-1.0), rtol=1e-15)
    assert np.isclose(r[2], 1.0 - 0.5, rtol=1e-15)
    assert np.isclose(r[3], 1.0 - 0.01 * 2.25 / 6, rtol=1e-15)
    assert not term.any()


def test_termination_thresholds():
    d = S.StationDesc(d_max=1.0, tilt_max=0.5)
    st = np.zeros((5, 21)); st[:, 3] = 1.0
    tg = np.zeros((5, 7)); tg[:, 3] = 1.0
    st[0, 0] = 0.999; st[1, 0] = 1.001
    st[2, 3:7] = S.quat_axis(np.array(0.49), 0); st[3, 3:7] = S.quat_axis(np.array(0.51), 1)
    st[4, 9] = np.nan
    r, term = S.reward_done(d, st, tg, np.zeros((5, 6)), 6)
    assert list(term) == [False, True, False, True, True]
    assert r[4] == 0.0
    # a pure yaw of any size never terminates
    st2 = np.zeros((1, 21)); st2[0, 3:7] = S.quat_axis(np.array(3.0), 2)
    assert not S.reward_done(d, st2, tg[:1], np.zeros((1, 6)), 6)[1][0]


def small_task(desc, n=8, seed=5):
    w = synth.plain_small(n=n)
    envs = oracle.make_envs(w.classes[0], w.params, w.dt)
    return S.StationOracle(desc, envs, w.classes[0].m), envs


def test_truncation_and_auto_reset():
    desc = S.StationDesc(max_steps=3, d_max=100.0, tilt_max=3.2)
    task, envs = small_task(desc)
    obs0 = task.reset(11)
    s_ref = task.state.copy()
    a = np.full((8, 6), 0.3)
    for k in range(3):
        obs, r, term, trunc, final = task.step(a)
        s_ref, _, _ = oracle.rollout(envs, s_ref, np.broadcast_to(np.pad(a, ((0, 0), (0, 2)))[:, None, :], (8, 1, 8)).copy(), 1, 1)
        assert not term.any()
        assert trunc.all() == (k == 2) and (trunc.any() == (k == 2))
    s1, t1 = S.episode_start(desc, 11, np.arange(8), 1, 6)
    assert np.array_equal(task.episode, np.ones(8)) and np.array_equal(task.t, np.zeros(8))
    assert np.array_equal(obs, S.observe(s1, t1, 6))
    s0, t0 = S.episode_start(desc, 11, np.arange(8), 0, 6)
    assert np.array_equal(final, S.observe(s_ref, t0, 6))
    assert np.array_equal(obs0, S.observe(s0, t0, 6))
    assert not np.array_equal(obs, obs0)


def test_non_finite_state_terminates_and_restarts():
    task, _ = small_task(S.StationDesc())
    task.reset(3)
    task.state[2, 8] = np.nan
    obs, r, term, trunc, final = task.step(np.zeros((8, 6)))
    assert term[2] and r[2] == 0.0 and np.isnan(final[2]).any()
    assert term.sum() == 1 and task.episode[2] == 1 and np.isfinite(obs).all()


def test_substeps_hold_the_command():
    desc = S.StationDesc(substeps=4)
    task, envs = small_task(desc)
    task.reset(8)
    s_ref = task.state.copy()
    a = np.linspace(-1.5, 1.5, 48).reshape(8, 6)
    obs, r, term, trunc, final = task.step(a)
    packed = np.zeros((8, 1, 8)); packed[:, 0, :6] = a
    for _ in range(4):
        s_ref, _, _ = oracle.rollout(envs, s_ref, packed, 1, 1)
    assert np.array_equal(final, S.observe(s_ref, task.target, 6))
    # the penalty uses the clipped command
    rr, _ = S.reward_done(desc, s_ref, task.target, np.clip(a, -1, 1), 6)
    assert np.array_equal(r, rr)
