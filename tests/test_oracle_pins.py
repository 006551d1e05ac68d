"""Pins for the FP64 oracle: closed forms, textbook identities, invariants and
convergence orders that fix each part of the step independently of the oracle's own
formulas. Each test names the part it pins; a dropped term, a wrong sign, index or a
transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth

G0 = 9.81


def env1(m=2, dt=0.01, **kw):
    """One oracle environment with explicit parameters (defaults: a plausible vehicle)."""
    e = np.zeros(1, dtype=oracle.ENV_DTYPE)
    e["m"] = m
    e["dt"] = dt
    e["g0"] = G0
    e["mass"] = 12.0
    e["inertia"] = [0.8, 1.1, 1.3]
    e["added"] = [3.0, 4.5, 5.0, 0.2, 0.35, 0.5]
    e["dlin"] = [4.0, 6.0, 5.0, 2.0, 3.0, 2.5]
    e["dquad"] = [20.0, 30.0, 25.0, 10.0, 12.0, 8.0]
    e["buoy"] = 12.0 * G0
    e["rb"] = [0.0, 0.0, -0.01]
    e["e"][0, :, 0] = 1.0
    e["k"][0, :m] = 30.0
    e["tau"][0, :m] = 0.1
    for key, val in kw.items():
        e[key] = val
    return e


def state1(p=(0, 0, 0), q=(1, 0, 0, 0), nu=(0,) * 6, n=()):
    s = np.zeros((1, oracle.STATE_LEN))
    s[0, 0:3], s[0, 3:7], s[0, 7:13] = p, q, nu
    s[0, 13:13 + len(n)] = n
    return s


def run(env, s, a, steps, hold=None, traj=True):
    """Constant action ``a`` for ``steps`` steps."""
    m = int(env["m"][0])
    acts = np.zeros((1, 1, oracle.MAX_THR))
    acts[0, 0, :m] = a
    st, tr, _ = oracle.rollout(env, s.copy(), acts, hold=steps + 1, n_steps=steps, traj=traj)
    return st, tr


def rand_quat(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


# ----------------------------------------------------------------------------- P1 rotor lag

def test_p1_first_order_lag_closed_form():
    """Constant command: n_k = a + (n0 - a) exp(-k dt / tau) exactly at the sample times."""
    env = env1(m=3)
    env["tau"][0, :3] = [0.05, 0.1, 0.15]
    n0 = np.array([0.3, -0.7, 0.9])
    a = np.array([-0.4, 0.6, 1.7])  # last one is clipped to 1
    _, tr = run(env, state1(n=n0), a, 1000)
    k = np.arange(1, 1001)[:, None]
    ac = np.clip(a, -1, 1)
    expect = ac + (n0 - ac) * np.exp(-k * 0.01 / env["tau"][0, :3])
    got = tr[0, :, 13:16]
    assert np.max(np.abs(got - expect) / np.abs(n0 - ac)) < 1e-12


def test_p1_zero_order_and_euler_lag():
    env = env1(m=2)
    env["tau"][0, :2] = [0.0, 0.1]
    env["flags"] = oracle.FLAG_LAG_EULER
    _, tr = run(env, state1(n=[0.2, 0.2]), [-0.5, 0.8], 3)
    assert tr[0, 0, 13] == -0.5 and tr[0, 2, 13] == -0.5          # zero-order: command itself
    expect = 0.8 + (0.2 - 0.8) * (1 - 0.01 / 0.1) ** np.arange(1, 4)  # Euler factor dt/tau
    assert np.allclose(tr[0, :, 14], expect, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- P2 thrust

def test_p2_symmetric_pair_gives_pure_surge():
    env = env1(m=2)
    env["r"][0, 0] = [0.0, 0.1, 0.0]
    env["r"][0, 1] = [0.0, -0.1, 0.0]
    env["k"][0, :2] = 25.0
    for n in (0.7, -0.3, 0.0):
        tau = oracle.thrust_wrench(env, [n, n])
        assert tau[0] == 2 * 25.0 * n * abs(n)
        assert np.all(tau[1:] == 0.0)


def test_p2_dead_zone_and_direction_normalisation():
    env = env1(m=1)
    env["deadzone"][0, 0] = 0.2
    env["k"][0, 0] = 10.0
    env["e"][0, 0] = [0.0, 2.0, 0.0]          # not unit: the oracle normalises it
    assert np.allclose(oracle.thrust_wrench(env, [0.5])[:3], [0, 10 * 0.3 * 0.3, 0], atol=1e-15)
    assert np.allclose(oracle.thrust_wrench(env, [-0.5])[:3], [0, -10 * 0.09, 0], atol=1e-15)
    assert np.all(oracle.thrust_wrench(env, [0.15]) == 0.0)


def test_p2_power_of_point_forces():
    """Power identity: for any body velocity (v, w), the wrench satisfies
    tau . nu = sum_i f_i e_i . (v + w x r_i) (the velocity of each thruster point)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        m = int(rng.integers(1, 9))
        env = env1(m=m)
        env["r"][0, :m] = rng.uniform(-0.3, 0.3, (m, 3))
        e = rng.normal(size=(m, 3))
        env["e"][0, :m] = e
        env["k"][0, :m] = rng.uniform(20, 40, m)
        n = rng.uniform(-1, 1, m)
        tau = oracle.thrust_wrench(env, n)
        nu = rng.normal(size=6)
        eu = e / np.linalg.norm(e, axis=1, keepdims=True)
        f = env["k"][0, :m] * n * np.abs(n)
        pts = nu[:3] + np.cross(nu[3:], env["r"][0, :m])
        power = np.sum(f * np.sum(eu * pts, axis=1))
        assert abs(tau @ nu - power) < 1e-12 * (1 + abs(power))


def test_p2_reverse_gain_and_reaction_torque():
    """One thruster off the centre line: forward gain 30, reverse gain 18, shaft torque
    0.04 m per unit thrust. Worked by hand: at n = 0.5 the thrust is 30 * 0.25 = 7.5 N
    along x at r = (0, 0.1, 0), so the moment is r x f e = (0, 0, -0.75) plus the shaft
    torque 0.04 * 7.5 = 0.3 about x; at n = -0.5 the reverse gain gives -4.5 N."""
    env = env1(m=1)
    env["r"][0, 0] = [0.0, 0.1, 0.0]
    env["k"][0, 0] = 30.0
    env["k_rev"][0, 0] = 18.0
    env["reaction"][0, 0] = 0.04
    assert np.allclose(oracle.thrust_wrench(env, [0.5]), [7.5, 0, 0, 0.3, 0, -0.75], rtol=0, atol=1e-14)
    assert np.allclose(oracle.thrust_wrench(env, [-0.5]), [-4.5, 0, 0, -0.18, 0, 0.45], rtol=0, atol=1e-14)
    env["k_rev"][0, 0] = 0.0                  # unset: symmetric
    assert np.allclose(oracle.thrust_wrench(env, [-0.5]), [-7.5, 0, 0, -0.3, 0, 0.75], rtol=0, atol=1e-14)


def test_p2_power_with_reverse_gain_and_shaft_torque():
    """Power identity with direction-dependent gains and shaft torques: for any body
    velocity, tau . nu = sum_i f_i e_i . (v + w x r_i) + sum_i c_i f_i e_i . w, with f_i
    taken with the gain of its own direction."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        m = int(rng.integers(1, 9))
        env = env1(m=m)
        env["r"][0, :m] = rng.uniform(-0.3, 0.3, (m, 3))
        e = rng.normal(size=(m, 3))
        env["e"][0, :m] = e
        kf = rng.uniform(20, 40, m)
        kr = kf * rng.uniform(0.5, 0.9, m)
        c = rng.uniform(-0.05, 0.05, m)
        env["k"][0, :m], env["k_rev"][0, :m], env["reaction"][0, :m] = kf, kr, c
        n = rng.uniform(-1, 1, m)
        tau = oracle.thrust_wrench(env, n)
        nu = rng.normal(size=6)
        eu = e / np.linalg.norm(e, axis=1, keepdims=True)
        f = np.where(n >= 0, kf, kr) * n * np.abs(n)
        pts = nu[:3] + np.cross(nu[3:], env["r"][0, :m])
        power = np.sum(f * np.sum(eu * pts, axis=1)) + np.sum(c * f * (eu @ nu[3:]))
        assert abs(tau @ nu - power) < 1e-12 * (1 + abs(power))


# ----------------------------------------------------------------------------- P12 rudder fins

def fin_env(r=(0.0, 0.0, 0.0), span=(0.0, 0.0, 1.0), chord=(1.0, 0.0, 0.0), kl=15.0, kd0=0.3, kd=6.0, dmax=0.5):
    """One fin and nothing else: span axis, chord at zero deflection, lift/drag gains."""
    e = env1(m=1)
    e["k"][0, 0] = 0.0
    e["kind"][0, 0] = oracle.FIN
    e["r"][0, 0], e["span"][0, 0], e["e"][0, 0] = r, span, chord
    e["fin_max"][0, 0], e["fin_lift"][0, 0], e["fin_drag0"][0, 0], e["fin_drag"][0, 0] = dmax, kl, kd0, kd
    return e


def test_p12_fin_worked_example():
    """Worked by hand: a vertical fin (span z, chord x) moving ahead at 2 m/s and turned by
    0.3 rad toward +y meets the water at 0.3 rad. The flat-plate law pushes it toward +y with
    15 sin(0.3)cos(0.3) 2^2 = 16.94 N and back with (0.3 + 6 sin^2(0.3)) 2^2 = 3.30 N; at
    r = (-0.7, 0, 0.1) that force turns the hull by r x F. The propeller law gives nothing
    for a fin, and the fin law nothing for a propeller."""
    env = fin_env(r=(-0.7, 0.0, 0.1))
    tau = oracle.fin_wrench(env, [0.6], [2.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    lift = 15.0 * np.sin(0.3) * np.cos(0.3) * 4.0
    drag = (0.3 + 6.0 * np.sin(0.3) ** 2) * 4.0
    assert abs(lift - 16.9393) < 1e-4 and abs(drag - 3.2960) < 1e-4
    F = np.array([-drag, lift, 0.0])
    assert np.allclose(tau[:3], F, rtol=0, atol=1e-12)
    assert np.allclose(tau[3:], np.cross([-0.7, 0.0, 0.1], F), rtol=0, atol=1e-12)
    assert np.all(oracle.thrust_wrench(env, [0.6]) == 0.0)
    prop = env1(m=1)
    assert np.all(oracle.fin_wrench(prop, [0.6], [2.0, 0.0, 0.0], [0.0, 0.0, 0.0]) == 0.0)


def _rand_fin(rng):
    span = rng.normal(size=3)
    chord = rng.normal(size=3)
    return fin_env(r=rng.uniform(-0.8, 0.8, 3), span=span, chord=chord, kl=rng.uniform(5, 30),
                   kd0=rng.uniform(0.1, 1.0), kd=rng.uniform(1, 10), dmax=rng.uniform(0.2, 0.7))


def _in_plane_flow(env, vr, w):
    s = env["span"][0, 0] / np.linalg.norm(env["span"][0, 0])
    u = vr + np.cross(w, env["r"][0, 0])
    return u - (u @ s) * s


def test_p12_fin_lift_does_no_work_and_drag_dissipates():
    """Power identities: lift is normal to the in-plane flow, so a fin with only lift does
    no work on the body (tau . [v_r; w] = 0); with only the angle-independent drag the power
    is -K_D0 |u_p|^3, u_p the flow at the fin point without its span component."""
    rng = np.random.default_rng(21)
    for _ in range(30):
        env = _rand_fin(rng)
        vr, w, n = rng.normal(0, 1, 3), rng.normal(0, 1, 3), rng.uniform(-1, 1)
        nur = np.concatenate([vr, w])
        lift_only = env.copy()
        lift_only["fin_drag0"], lift_only["fin_drag"] = 0.0, 0.0
        t = oracle.fin_wrench(lift_only, [n], vr, w)
        assert np.abs(t).max() > 1e-3
        assert abs(t @ nur) < 1e-12 * np.abs(t).max() * np.abs(nur).max()
        drag0 = env.copy()
        drag0["fin_lift"], drag0["fin_drag"] = 0.0, 0.0
        up = _in_plane_flow(env, vr, w)
        t = oracle.fin_wrench(drag0, [n], vr, w)
        ref = -env["fin_drag0"][0, 0] * np.linalg.norm(up) ** 3
        assert abs(t @ nur - ref) < 1e-12 * abs(ref)


def test_p12_fin_angle_of_attack_is_deflection_minus_flow_angle():
    """A fin turned to the flow's own in-plane direction meets it edge-on: no lift, drag
    K_D0 |u_p|^2 exactly against the flow. Flow along the span gives no force at all."""
    rng = np.random.default_rng(22)
    for _ in range(20):
        beta = rng.uniform(-0.45, 0.45)
        env = fin_env(dmax=0.5)
        U = rng.uniform(0.5, 2.0)
        vr = np.array([U * np.cos(beta), U * np.sin(beta), rng.normal()])   # z is the span
        t = oracle.fin_wrench(env, [beta / 0.5], vr, np.zeros(3))
        F = -0.3 * U * U * np.array([np.cos(beta), np.sin(beta), 0.0])
        assert np.allclose(t[:3], F, rtol=0, atol=1e-12)
    assert np.all(oracle.fin_wrench(fin_env(), [0.7], [0.0, 0.0, 1.3], [0.0, 0.0, 0.0]) == 0.0)


def test_p12_fin_small_angle_lift_slope_and_mirror():
    """Thin-fin limit: moving along the chord at U with a small deflection delta, the lift
    tends to K_L delta U^2 (relative error O(delta^2)). Mirroring the deflection and the
    cross flow mirrors the normal force and keeps the chordwise one."""
    env = fin_env(kl=12.0, dmax=0.5)
    for d in (1e-2, 1e-3):
        t = oracle.fin_wrench(env, [d / 0.5], [1.5, 0.0, 0.0], np.zeros(3))
        assert abs(t[1] / (12.0 * d * 1.5 ** 2) - 1) < 2 * d * d
    rng = np.random.default_rng(23)
    for _ in range(10):
        n = rng.uniform(-1, 1)
        vr = np.array([rng.uniform(0.3, 2), rng.normal(), rng.normal()])
        a = oracle.fin_wrench(env, [n], vr, np.zeros(3))
        b = oracle.fin_wrench(env, [-n], vr * [1, -1, 1], np.zeros(3))
        assert np.allclose([a[0], a[1]], [b[0], -b[1]], rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------- P13 payload

def _general_kirchhoff(env, x):
    M = oracle.mass_matrix(env)
    nu = x[7:13]
    Pv = M @ nu
    P, L = Pv[:3], Pv[3:]
    R = oracle.rotation(x[3:7])
    return np.array([0.5 * nu @ Pv, P @ P, P @ L, *(R @ P)])


def test_p13_mass_matrix_with_a_payload():
    """M_RB with the CoG at r_g: symmetric, positive definite, the origin inertia is the
    CoG inertia moved by the parallel-axis theorem, and its kinetic energy is that of the
    CoG's motion plus the spin about the CoG."""
    rng = np.random.default_rng(31)
    env = env1(m=1, added=np.zeros(6), rg=[0.05, -0.03, 0.08])
    M = oracle.mass_matrix(env)
    assert np.allclose(M, M.T, atol=0) and np.all(np.linalg.eigvalsh(M) > 0)
    for _ in range(10):
        nu = rng.normal(size=6)
        v_cg = nu[:3] + np.cross(nu[3:], env["rg"][0])
        T = 0.5 * env["mass"][0] * v_cg @ v_cg + 0.5 * nu[3:] @ (env["inertia"][0] * nu[3:])
        assert abs(0.5 * nu @ M @ nu - T) < 1e-12 * T


def test_p13_kirchhoff_invariants_with_a_payload():
    """Kirchhoff's invariants hold for any symmetric inertia: with a payload (CoG off the
    origin), added mass, and no thrust, damping, restoring or current, RK4 conserves
    T = nu^T M nu / 2, |P|^2, P.L and the world impulse R P to its own error."""
    rng = np.random.default_rng(32)
    x0 = state1(q=rand_quat(rng), nu=[0.4, -0.3, 0.2, 0.3, -0.5, 0.4])
    env = _free_env(0.01, rg=[0.06, -0.04, 0.09])
    env["rb"] = env["rg"]
    inv0 = _general_kirchhoff(env, x0[0])
    ref = oracle.rk4_smooth(env, x0, np.zeros((1, 24)), 1e-3, 1000)
    assert np.max(np.abs(_general_kirchhoff(env, ref[0]) - inv0)) < 1e-10


def test_p13_spin_about_the_centre_of_gravity():
    """Torque-free spin about the CoG: isotropic CoG inertia, no added mass, CoB at the
    CoG of a neutral body, no damping. With v = -w x r_g the CoG is at rest; the Coriolis
    terms then cancel exactly, so the discrete map leaves nu unchanged."""
    rg = np.array([0.05, -0.02, 0.07])
    env = env1(m=1, added=np.zeros(6), dlin=np.zeros(6), dquad=np.zeros(6), inertia=[0.9, 0.9, 0.9], rg=rg,
               k=np.zeros(8))
    env["rb"] = rg
    w = np.array([0.7, -1.1, 0.4])
    nu = np.concatenate([-np.cross(w, rg), w])
    _, tr = run(env, state1(nu=nu), [0.0], 200)
    assert np.max(np.abs(tr[0, :, 7:13] - nu)) < 1e-13


def test_p13_payload_tilts_the_equilibrium():
    """A neutral body with the CoB 3 cm above the origin and a payload moving the CoG 2 cm
    forward and 1 cm down rests pitched so that the CoG hangs straight below the CoB:
    tan(theta) = x_g / (z_g - z_b) (nose down). Started there at rest it stays there."""
    rg, rb = np.array([0.02, 0.0, 0.01]), np.array([0.0, 0.0, -0.03])
    env = env1(m=1, rg=rg, rb=rb, k=np.zeros(8))
    th = -np.arctan2(rg[0], rg[2] - rb[2])
    q = np.array([np.cos(th / 2), 0.0, np.sin(th / 2), 0.0])
    _, tr = run(env, state1(q=q), [0.0], 2000)
    assert np.max(np.abs(tr[0, :, 7:13])) < 1e-12
    # and at zero pitch the same body starts to pitch nose down
    _, tr = run(env, state1(), [0.0], 10)
    assert tr[0, -1, 11] < -1e-4


# ----------------------------------------------------------------------------- P3 kinematics

def euler_zyx_matrix(phi, th, psi):
    """Textbook body -> NED rotation for roll phi, pitch th, yaw psi (z-y-x convention)."""
    c, s = np.cos, np.sin
    return np.array([
        [c(psi) * c(th), -s(psi) * c(phi) + c(psi) * s(th) * s(phi), s(psi) * s(phi) + c(psi) * c(phi) * s(th)],
        [s(psi) * c(th), c(psi) * c(phi) + s(phi) * s(th) * s(psi), -c(psi) * s(phi) + s(th) * s(psi) * c(phi)],
        [-s(th), c(th) * s(phi), c(th) * c(phi)]])


def euler_zyx_quat(phi, th, psi):
    c, s = np.cos, np.sin
    cr, sr, cp, sp, cy, sy = c(phi / 2), s(phi / 2), c(th / 2), s(th / 2), c(psi / 2), s(psi / 2)
    return np.array([cr * cp * cy + sr * sp * sy, sr * cp * cy - cr * sp * sy,
                     cr * sp * cy + sr * cp * sy, cr * cp * sy - sr * sp * cy])


def test_p3_rotation_identities():
    rng = np.random.default_rng(2)
    for _ in range(50):
        q = rand_quat(rng)
        R = oracle.rotation(q)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        assert np.allclose(oracle.rotation(-q), R, atol=0)
        phi, th, psi = rng.uniform(-np.pi, np.pi), rng.uniform(-1.5, 1.5), rng.uniform(-np.pi, np.pi)
        assert np.allclose(oracle.rotation(euler_zyx_quat(phi, th, psi)), euler_zyx_matrix(phi, th, psi),
                           atol=1e-14)


def test_p3_quaternion_product():
    i, j, k, one = np.eye(4)[1], np.eye(4)[2], np.eye(4)[3], np.eye(4)[0]
    assert np.array_equal(oracle.quat_mul(i, j), k)
    assert np.array_equal(oracle.quat_mul(j, k), i)
    assert np.array_equal(oracle.quat_mul(k, i), j)
    assert np.array_equal(oracle.quat_mul(i, i), -one)
    rng = np.random.default_rng(3)
    a, b = rand_quat(rng), rand_quat(rng)
    assert np.allclose(oracle.rotation(oracle.quat_mul(a, b)), oracle.rotation(a) @ oracle.rotation(b),
                       atol=1e-14)


# ----------------------------------------------------------------------------- P4 Coriolis

def test_p4_coriolis_terms_do_no_work():
    """nu^T C_RB(nu) nu = 0 and nu_r^T C_A(nu_r) nu_r = 0 (skew-symmetric forms)."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        env = env1(m=1, current=rng.normal(0, 0.3, 3), inertia=rng.uniform(0.5, 2, 3),
                   added=rng.uniform(0.1, 5, 6))
        q, nu = rand_quat(rng), rng.normal(size=6)
        t = oracle.terms(env, q, nu, [0.0])
        R = oracle.rotation(q)
        vr = nu[:3] - R.T @ env["current"][0]
        nur = np.concatenate([vr, nu[3:]])
        assert abs(nu @ t["crb"]) < 1e-13 * (1 + np.abs(t["crb"]).sum())
        assert abs(nur @ t["ca"]) < 1e-13 * (1 + np.abs(t["ca"]).sum())
        assert np.abs(t["crb"]).max() > 1e-3 and np.abs(t["ca"]).max() > 1e-3


def _free_env(dt, **kw):
    """No damping, no restoring (W = B, r_b = 0), no current, no thrust."""
    return env1(m=1, dt=dt, dlin=np.zeros(6), dquad=np.zeros(6), rb=[0, 0, 0], k=np.zeros(8), **kw)


def _kirchhoff(env, x):
    m, I, A = env["mass"][0], env["inertia"][0], env["added"][0]
    v, w = x[7:10], x[10:13]
    P = (m + A[:3]) * v
    L = (I + A[3:]) * w
    R = oracle.rotation(x[3:7])
    return np.array([0.5 * (P @ v + L @ w), P @ P, P @ L, *(R @ P)])


def test_p4_kirchhoff_invariants():
    """With no thrust, damping, restoring or current, the flow conserves kinetic energy,
    |P|^2, P.L and the world-frame impulse R P (Kirchhoff's equations for a body with
    added mass). RK4 conserves them to its own error; the first-order step drifts by
    O(dt) and the drift halves with dt."""
    rng = np.random.default_rng(5)
    x0 = state1(q=rand_quat(rng), nu=[0.4, -0.3, 0.2, 0.3, -0.5, 0.4])
    env = _free_env(0.01)
    inv0 = _kirchhoff(env, x0[0])
    smooth = np.zeros((1, 24))
    ref = oracle.rk4_smooth(env, x0, smooth, 1e-3, 1000)
    assert np.max(np.abs(_kirchhoff(env, ref[0]) - inv0)) < 1e-11
    drift = []
    for dt in (0.01, 0.005, 0.0025):
        e = _free_env(dt)
        st, _ = run(e, x0, [0.0], int(round(1.0 / dt)), traj=False)
        drift.append(np.abs(_kirchhoff(e, st[0]) - inv0))
    for a, b in zip(drift, drift[1:]):
        ratio = a[0] / b[0]
        assert 1.8 <= ratio <= 2.2, ratio
        assert np.all(a > 1e-8)


# ----------------------------------------------------------------------------- P5 damping

def _surge_env(dt=0.01, dl=4.0, dq=0.0):
    e = env1(m=1, dt=dt, k=np.zeros(8))
    e["dlin"][0, 0] = dl
    e["dquad"][0, 0] = dq
    return e


def test_p5_linear_damping_discrete_closed_form():
    env = _surge_env(dl=7.0)
    _, tr = run(env, state1(nu=[0.5, 0, 0, 0, 0, 0]), [0.0], 1000)
    M = 12.0 + 3.0
    expect = 0.5 * (1 - 0.01 * 7.0 / M) ** np.arange(1, 1001)
    assert np.max(np.abs(tr[0, :, 7] - expect) / np.abs(expect)) < 1e-12
    assert np.all(tr[0, :, 8:13] == 0.0)


def test_p5_position_uses_updated_velocity():
    """Semi-implicit step: position advances with the velocity after the update, so under
    pure linear surge damping p_k = dt u0 r (1 - r^k) / (1 - r), r = 1 - dt d_L / M."""
    env = _surge_env(dl=7.0)
    _, tr = run(env, state1(nu=[0.5, 0, 0, 0, 0, 0]), [0.0], 500)
    r = 1 - 0.01 * 7.0 / 15.0
    k = np.arange(1, 501)
    expect = 0.01 * 0.5 * r * (1 - r ** k) / (1 - r)
    assert np.max(np.abs(tr[0, :, 0] - expect) / expect) < 1e-12


def test_p5_thrust_acts_on_the_lagged_rotor_state():
    """Lag first, then thrust: from rest, the first step's surge velocity is
    dt * 2 k s|s| / M with s the rotor state after this step's lag (zero-order: the
    command itself; first-order: alpha times the command)."""
    for tau, factor in ((0.0, 1.0), (0.1, 1 - np.exp(-0.1))):
        env = env1(m=2)
        env["r"][0, 0] = [0.0, 0.1, 0.0]
        env["r"][0, 1] = [0.0, -0.1, 0.0]
        env["tau"][0, :2] = tau
        _, tr = run(env, state1(), [0.5, 0.5], 1)
        s = 0.5 * factor
        assert abs(tr[0, 0, 7] - 0.01 * 2 * 30.0 * s * s / 15.0) < 1e-15


@pytest.mark.parametrize("a", [0.8, -0.8])
def test_p5_surge_and_roll_from_one_propeller_closed_form(a):
    """One zero-order propeller at the CoG along x with a dead zone, a reverse gain and a
    shaft torque; neutral, CoB at the CoG, linear damping only, no current. Surge and roll
    then stay decoupled (every Coriolis and restoring term vanishes for v and w both along
    x) and the map reduces to two scalar recurrences with exact solutions:
    u_k = u* (1 - r_u^k), u* = f / d_u, r_u = 1 - dt d_u / (m + A_11); the same for the roll
    rate with torque c f and I_x + A_44; x_k = dt sum_{j<=k} u_j and
    q_k = (cos(phi_k / 2), sin(phi_k / 2), 0, 0) with phi_k = dt sum_{j<=k} p_j."""
    dt, steps = 0.01, 400
    env = env1(m=1, dt=dt, dquad=np.zeros(6), rb=[0, 0, 0])
    env["tau"][0, 0] = 0.0
    env["deadzone"][0, 0] = 0.1
    env["k"][0, 0], env["k_rev"][0, 0], env["reaction"][0, 0] = 30.0, 19.0, 0.035
    assert env["buoy"][0] == env["mass"][0] * G0
    gain = 30.0 if a > 0 else 19.0
    f = gain * np.sign(a) * (abs(a) - 0.1) ** 2
    du, dp = env["dlin"][0, 0], env["dlin"][0, 3]
    Mu, Mp = env["mass"][0] + env["added"][0, 0], env["inertia"][0, 0] + env["added"][0, 3]
    k = np.arange(1, steps + 1)
    u = f / du * (1 - (1 - dt * du / Mu) ** k)
    pr = 0.035 * f / dp * (1 - (1 - dt * dp / Mp) ** k)
    x = dt * np.cumsum(u)
    phi = dt * np.cumsum(pr)
    _, tr = run(env, state1(), [a], steps)
    g = tr[0]
    scale = np.abs(g).max(axis=0) + 1e-300
    assert np.max(np.abs(g[:, 7] - u) / np.abs(u).max()) < 1e-12
    assert np.max(np.abs(g[:, 10] - pr) / np.abs(pr).max()) < 1e-12
    assert np.max(np.abs(g[:, 0] - x) / np.abs(x).max()) < 1e-12
    assert np.max(np.abs(g[:, 3] - np.cos(phi / 2))) < 1e-12
    assert np.max(np.abs(g[:, 4] - np.sin(phi / 2))) < 1e-12
    assert np.all(g[:, [1, 2, 5, 6, 8, 9, 11, 12]] == 0.0), scale


def test_p5_damping_continuous_decay_first_order():
    """Exponential decay under pure linear damping, 1/(1 + c t) under pure quadratic
    damping; the discrete map approaches both at first order in dt."""
    M = 15.0
    for dl, dq, exact in ((7.0, 0.0, lambda t: 0.5 * np.exp(-7.0 * t / M)),
                          (0.0, 30.0, lambda t: 0.5 / (1 + 30.0 * 0.5 * t / M))):
        errs = []
        for dt in (0.01, 0.005, 0.0025):
            env = _surge_env(dt, dl, dq)
            st, _ = run(env, state1(nu=[0.5, 0, 0, 0, 0, 0]), [0.0], int(round(2.0 / dt)), traj=False)
            errs.append(abs(st[0, 7] - exact(2.0)))
        assert 1.8 <= errs[0] / errs[1] <= 2.2 and 1.8 <= errs[1] / errs[2] <= 2.2, errs


# ----------------------------------------------------------------------------- P6 restoring

def fossen_restoring(W, B, rb, phi, th):
    """Textbook restoring vector g(eta) for ZYX Euler angles, weight at the origin."""
    c, s = np.cos, np.sin
    xb, yb, zb = rb
    return np.array([(W - B) * s(th), -(W - B) * c(th) * s(phi), -(W - B) * c(th) * c(phi),
                     yb * B * c(th) * c(phi) - zb * B * c(th) * s(phi),
                     -zb * B * s(th) - xb * B * c(th) * c(phi),
                     xb * B * c(th) * s(phi) + yb * B * s(th)])


def test_p6_restoring_matches_euler_angle_form():
    rng = np.random.default_rng(6)
    for _ in range(50):
        rb = rng.uniform(-0.05, 0.05, 3)
        W, B = 120.0, rng.uniform(100, 140)
        env = env1(m=1, rb=rb, buoy=B, mass=W / G0)
        phi, th, psi = rng.uniform(-np.pi, np.pi), rng.uniform(-1.5, 1.5), rng.uniform(-np.pi, np.pi)
        t = oracle.terms(env, euler_zyx_quat(phi, th, psi), np.zeros(6), [0.0])
        assert np.allclose(t["restore"], fossen_restoring(W, B, rb, phi, th), atol=1e-12)


def test_p6_static_equilibrium_is_exact():
    """Neutrally buoyant, CoB straight above CoG, upright, at rest, no command, no current:
    a fixed point of the map, value-for-value constant for 10^4 steps."""
    env = env1(m=2, rb=[0, 0, -0.02])
    x0 = state1()
    st, _ = run(env, x0, [0.0, 0.0], 10000, traj=False)
    assert np.all(st == x0)


def test_p6_small_roll_frequency():
    """Without damping, small roll oscillates at sqrt(B h / (I_x + A_44))."""
    h, phi0 = 0.02, 0.01
    env = env1(m=1, rb=[0, 0, -h], dlin=np.zeros(6), dquad=np.zeros(6), k=np.zeros(8))
    wn = np.sqrt(env["buoy"][0] * h / (env["inertia"][0, 0] + env["added"][0, 3]))
    dt = 0.001
    env["dt"] = dt
    T = 2 * np.pi / wn
    n = int(3.2 * T / dt)
    _, tr = run(env, state1(q=[np.cos(phi0 / 2), np.sin(phi0 / 2), 0, 0]), [0.0], n)
    p = tr[0, :, 10]
    idx = np.where((p[:-1] > 0) & (p[1:] <= 0))[0]
    tz = (idx + 1 + p[idx] / (p[idx] - p[idx + 1])) * dt   # interpolated downward crossings
    period = np.mean(np.diff(tz))
    assert abs(period - T) / T < 1e-3, (period, T)


def _energy(env, x):
    m, I, A = env["mass"][0], env["inertia"][0], env["added"][0]
    Mdiag = np.array([m, m, m, *I]) + A
    nu = x[7:13]
    gb = oracle.rotation(x[3:7])[2]
    W, B = m * G0, env["buoy"][0]
    return 0.5 * nu @ (Mdiag * nu) - (W - B) * x[2] + B * env["rb"][0] @ gb


def test_p6_energy_with_restoring():
    """No damping, thrust or current: kinetic energy plus the potential
    -(W - B) z + B r_b . g_b is conserved by the flow; the step drifts at O(dt)."""
    rng = np.random.default_rng(7)
    kw = dict(dlin=np.zeros(6), dquad=np.zeros(6), k=np.zeros(8), rb=[0.01, -0.02, -0.03],
              buoy=12.3 * G0)
    x0 = state1(q=rand_quat(rng), nu=[0.3, -0.2, 0.1, 0.4, -0.3, 0.2])
    env = env1(m=1, **kw)
    e0 = _energy(env, x0[0])
    ref = oracle.rk4_smooth(env, x0, np.zeros((1, 24)), 1e-3, 2000)
    assert abs(_energy(env, ref[0]) - e0) < 1e-10
    drift = []
    for dt in (0.01, 0.005, 0.0025):
        e = env1(m=1, dt=dt, **kw)
        st, _ = run(e, x0, [0.0], int(round(2.0 / dt)), traj=False)
        drift.append(abs(_energy(e, st[0]) - e0))
    assert 1.8 <= drift[0] / drift[1] <= 2.2 and 1.8 <= drift[1] / drift[2] <= 2.2, drift


# ----------------------------------------------------------------------------- P7-P9 fixed points

def test_p7_terminal_surge_under_thrust():
    env = env1(m=2)
    env["r"][0, 0] = [0.0, 0.1, 0.0]
    env["r"][0, 1] = [0.0, -0.1, 0.0]
    a = 0.6
    F = 2 * 30.0 * a * a
    dl, dq = env["dlin"][0, 0], env["dquad"][0, 0]
    u_inf = (-dl + np.sqrt(dl * dl + 4 * dq * F)) / (2 * dq)
    st, _ = run(env, state1(), [a, a], 5000, traj=False)
    assert abs(st[0, 7] - u_inf) / u_inf < 1e-12
    assert np.all(np.abs(st[0, 8:13]) < 1e-14)


def test_p8_terminal_heave_under_net_buoyancy():
    env = env1(m=1, k=np.zeros(8), buoy=12.0 * G0 * 1.02)
    W, B = 12.0 * G0, env["buoy"][0]
    dl, dq = env["dlin"][0, 2], env["dquad"][0, 2]
    w_inf = -(-dl + np.sqrt(dl * dl + 4 * dq * (B - W))) / (2 * dq)
    st, _ = run(env, state1(), [0.0], 5000, traj=False)
    assert abs(st[0, 9] - w_inf) / abs(w_inf) < 1e-12
    assert w_inf < 0          # rises (NED: negative z is up)


def test_p9_body_drifts_to_the_current():
    """Isotropic linear added mass, neutral, CoB at the CoG, no thrust, not rotating: the
    world-frame velocity R v tends to the current V_c exactly (v_r -> 0), for any fixed
    attitude. Pins the sign of v_r and the direction of the body projection."""
    rng = np.random.default_rng(9)
    Vc = np.array([0.3, -0.2, 0.1])
    env = env1(m=1, k=np.zeros(8), rb=[0, 0, 0], added=[3.0, 3.0, 3.0, 0.2, 0.3, 0.4], current=Vc,
               dlin=[20.0, 25.0, 30.0, 2.0, 3.0, 2.5])
    q0 = rand_quat(rng)
    st, _ = run(env, state1(q=q0), [0.0], 6000, traj=False)
    R = oracle.rotation(st[0, 3:7])
    assert np.allclose(st[0, 3:7], q0, atol=1e-15)
    assert np.max(np.abs(R @ st[0, 7:10] - Vc)) < 1e-12


def test_p9_spinning_body_carried_by_the_current():
    """A body moving with the water (v_r = 0) while spinning about any axis with
    isotropic I + A_2 stays with the water in continuous time only if the added-mass term
    from the rotating current projection is present: RK4 keeps |v_r| at its own error
    with the term and loses it without."""
    rng = np.random.default_rng(10)
    Vc = np.array([0.4, -0.3, 0.2])
    base = dict(k=np.zeros(8), rb=[0, 0, 0], inertia=[0.8, 1.0, 1.2], added=[3, 4, 5, 0.7, 0.5, 0.3],
                current=Vc, dlin=[4, 6, 5, 0, 0, 0], dquad=[20, 30, 25, 0, 0, 0])
    q0 = rand_quat(rng)
    w0 = np.array([0.5, -0.4, 0.3])
    v0 = oracle.rotation(q0).T @ Vc
    x0 = state1(q=q0, nu=[*v0, *w0])

    def vr_after(flags):
        env = env1(m=1, flags=flags, **base)
        x = oracle.rk4_smooth(env, x0, np.zeros((1, 24)), 1e-3, 2000)
        return np.linalg.norm(x[0, 7:10] - oracle.rotation(x[0, 3:7]).T @ Vc)

    assert vr_after(0) < 1e-10
    assert vr_after(oracle.FLAG_NO_AMC) > 1e-3


# ----------------------------------------------------------------------------- P10 attitude

def test_p10_constant_spin_attitude_is_exact():
    """Torque-free spin with isotropic I + A_2: q_k = q_0 (x) exp(k w dt / 2) exactly."""
    rng = np.random.default_rng(11)
    env = env1(m=1, k=np.zeros(8), rb=[0, 0, 0], inertia=[1.0, 2.0, 3.0], added=[3, 4, 5, 3.0, 2.0, 1.0],
               dlin=[4, 6, 5, 0, 0, 0], dquad=[20, 30, 25, 0, 0, 0])
    w = np.array([0.7, -0.5, 0.4])
    q0 = rand_quat(rng)
    _, tr = run(env, state1(q=q0, nu=[0, 0, 0, *w]), [0.0], 1000)
    wn = np.linalg.norm(w)
    for k in (1, 10, 100, 1000):
        th = k * wn * 0.01
        d = np.array([np.cos(th / 2), *(np.sin(th / 2) * w / wn)])
        assert np.max(np.abs(tr[0, k - 1, 3:7] - oracle.quat_mul(q0, d))) < 1e-12
    assert np.max(np.abs(tr[0, :, 10:13] - w)) < 1e-13
    assert np.max(np.abs(tr[0, :, 7:10])) < 1e-13


# ----------------------------------------------------------------------------- P11 whole map

def _smooth(rng, n):
    sp = np.zeros((n, 24))
    sp[:, :8] = 0.8
    sp[:, 8:16] = rng.uniform(0.2, 1.0, (n, 8))
    sp[:, 16:24] = rng.uniform(0, 2 * np.pi, (n, 8))
    return sp


@pytest.mark.parametrize("with_current", [False, True])
def test_p11_step_halving_first_order(with_current):
    """Whole map against a fine RK4 solution of the continuous model over 1 s: the error
    halves with dt (first-order scheme) for dt = 0.02, 0.01, 0.005."""
    n = 8
    cls = synth.draw_class(6, 0, dt=0.02)
    if with_current:
        params = synth.randomised_params(cls, n, dt=0.02)
    else:
        params = synth.nominal_params(cls, n)
    st0 = synth.initial_state(n, 6)
    x0 = oracle.pack_state(st0.p, st0.q, st0.nu, st0.n)
    sp = _smooth(np.random.default_rng(12), n)
    ref = oracle.rk4_smooth(oracle.make_envs(cls, params, 0.02), x0, sp, 0.005 / 64, 64 * 200)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        envs = oracle.make_envs(cls, params, dt)
        x = oracle.rollout_smooth(envs, x0, sp, int(round(1.0 / dt)))
        errs.append(np.linalg.norm(x - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 <= r1 <= 2.2 and 1.8 <= r2 <= 2.2, (errs, r1, r2)


def test_rk4_reference_is_fourth_order():
    """Self-convergence of the continuous reference on a smooth instance: quadratic damping
    and thrust off, since |x| x has a kink in its second derivative that lowers the order
    near zero crossings."""
    n = 4
    cls = synth.draw_class(6, 0)
    envs = oracle.make_envs(cls, synth.randomised_params(cls, n), 0.01)
    envs["dquad"] = 0.0
    envs["k"] = 0.0
    st0 = synth.initial_state(n, 6)
    x0 = oracle.pack_state(st0.p, st0.q, st0.nu, st0.n)
    sp = _smooth(np.random.default_rng(13), n)
    xs = [oracle.rk4_smooth(envs, x0, sp, 0.2 / 2 ** j, 2 ** j * 5) for j in range(3, 7)]
    e = [np.linalg.norm(a - b) for a, b in zip(xs, xs[1:])]
    assert 12 <= e[0] / e[1] <= 20 and 12 <= e[1] / e[2] <= 20, e


# ----------------------------------------------------------------------------- force readout

def test_forces_readout_closes_the_rigid_body_balance():
    """M_RB d(nu)/dt + C_RB(nu) nu + g_RB = actuator wrench + hydrodynamic wrench (Eq. (2)
    with the hydrodynamic part moved to the right as in Eq. (3))."""
    rng = np.random.default_rng(14)
    cls = synth.draw_class(6, 0)
    params = synth.randomised_params(cls, 4)
    envs = oracle.make_envs(cls, params, 0.01)
    st0 = synth.initial_state(4, 6)
    x0 = oracle.pack_state(st0.p, st0.q, st0.nu, st0.n)
    x0[:, 13:19] = rng.uniform(-1, 1, (4, 6))
    for i in range(4):
        a = rng.uniform(-1, 1, 6)
        x1, f = oracle.step(envs[i:i + 1], x0[i], a, want_forces=True)
        nudot = (x1[7:13] - x0[i, 7:13]) / 0.01
        m, I = envs["mass"][i], envs["inertia"][i]
        t = oracle.terms(envs[i:i + 1], x0[i, 3:7], x0[i, 7:13], x1[13:19])
        gb = oracle.rotation(x0[i, 3:7])[2]
        g_rb = np.concatenate([-m * G0 * gb, np.zeros(3)])
        lhs = np.array([m, m, m, *I]) * nudot + t["crb"] + g_rb
        assert np.allclose(lhs, f[:6] + f[6:], rtol=1e-9, atol=1e-9)


def test_action_row_indexing():
    """Step t uses row floor(t / hold) - row0 of the action buffer."""
    env = env1(m=1, k=np.zeros(8))
    env["tau"][0, 0] = 0.0   # zero-order: n equals the command
    acts = np.zeros((1, 5, oracle.MAX_THR))
    acts[0, :, 0] = [0.1, 0.2, 0.3, 0.4, 0.5]
    _, tr, _ = oracle.rollout(env, state1(), acts, hold=3, n_steps=9, t0=7, row0=2, traj=True)
    got = tr[0, :, 13]
    expect = [acts[0, (7 + k) // 3 - 2, 0] for k in range(9)]
    assert np.array_equal(got, expect)
    with pytest.raises(IndexError):
        oracle.rollout(env, state1(), acts, hold=3, n_steps=15, t0=7, row0=2)


# ----------------------------------------------------------------------------- P13 rollout loss

def _loss(env, s0, acts, wp, weight=1e-3):
    """Per-environment loss of one environment; acts [H, 8], wp [3]."""
    H = acts.shape[0]
    return oracle.rollout_loss(env, s0, acts[None], H, np.asarray(wp, float)[None], weight)[0]


def test_p13_loss_static_equilibrium_is_horizon_times_distance():
    """A neutral vehicle at rest with its CoB above the CoG and zero commands stays at the
    origin (pin P6(ii)), so every one of the H terms is |w|^2 and the loss is H |w|^2."""
    env = env1(m=2)
    wp = [0.7, -1.3, 2.1]
    for H in (1, 7, 256):
        L = _loss(env, state1(), np.zeros((H, oracle.MAX_THR)), wp)
        assert L == pytest.approx(H * (0.49 + 1.69 + 4.41), rel=1e-13, abs=0)  # summation order only


def _surge_closed_form(u0, dl, M, dt, H):
    """Positions after steps 1..H under pure linear surge damping (no thrust): the
    velocity after step j is u0 r^j, r = 1 - dt d_L / M, and the semi-implicit position is
    p_k = dt sum_{j=1..k} u_j = dt u0 r (1 - r^k) / (1 - r)."""
    r = 1.0 - dt * dl / M
    k = np.arange(1, H + 1)
    return dt * u0 * r * (1.0 - r ** k) / (1.0 - r), r


def test_p13_loss_surge_decay_closed_form():
    """Surge-only linear damping: the loss sums the distance from the waypoint of the
    position AFTER each of the steps 1..H. A loss that scores the position before the
    step (k = 0..H-1), drops the last step or mixes the waypoint axes fails here."""
    env = _surge_env(dl=7.0)
    H, u0, wp = 200, 0.5, np.array([0.9, -0.4, 0.25])
    p, _ = _surge_closed_form(u0, 7.0, 15.0, 0.01, H)
    expect = np.sum((p - wp[0]) ** 2) + H * (wp[1] ** 2 + wp[2] ** 2)
    L = _loss(env, state1(nu=[u0, 0, 0, 0, 0, 0]), np.zeros((H, oracle.MAX_THR)), wp)
    assert abs(L - expect) / expect < 1e-13
    before = np.sum((np.concatenate([[0.0], p[:-1]]) - wp[0]) ** 2) + H * (wp[1] ** 2 + wp[2] ** 2)
    assert abs(before - expect) / expect > 1e-3   # the two readings are far apart here


def test_p13_damping_derivative_closed_form_against_finite_differences():
    """P13's closed form: under pure linear surge damping du_k/dd_L = -k (dt/M) u0 r^(k-1),
    so dp_k/dd_L = dt sum_{j<=k} du_j/dd_L and dL/dd_L = sum_k 2 (p_k - w_x) dp_k/dd_L.
    Central differences (h = 1e-4) of the oracle's loss and of its velocity agree with it."""
    dl, dt, M, H, u0 = 7.0, 0.01, 15.0, 256, 0.5
    wp = np.array([0.9, -0.4, 0.25])
    p, r = _surge_closed_form(u0, dl, M, dt, H)
    k = np.arange(1, H + 1)
    du = -k * (dt / M) * u0 * r ** (k - 1)
    dp = dt * np.cumsum(du)
    dL = np.sum(2.0 * (p - wp[0]) * dp)
    h = 1e-4
    s0 = state1(nu=[u0, 0, 0, 0, 0, 0])
    acts = np.zeros((H, oracle.MAX_THR))
    fd = (_loss(_surge_env(dl=dl + h), s0, acts, wp) - _loss(_surge_env(dl=dl - h), s0, acts, wp)) / (2 * h)
    assert abs(fd - dL) / abs(dL) < 1e-7, (fd, dL)
    _, tp = run(_surge_env(dl=dl + h), s0, [0.0], H)
    _, tm = run(_surge_env(dl=dl - h), s0, [0.0], H)
    fd_u = (tp[0, :, 7] - tm[0, :, 7]) / (2 * h)
    assert np.max(np.abs(fd_u - du)) / np.abs(du).max() < 1e-7


def test_p13_action_weight_uses_the_raw_commands_of_the_class_thrusters():
    """With zero thrust gains the commands move nothing, so L = H |w|^2 + lambda sum_k
    sum_{i<m} a_{k,i}^2: the raw commands (values beyond [-1, 1] are not clipped in the
    penalty), only the class's m thrusters (the padding of the action rows is ignored)."""
    rng = np.random.default_rng(3)
    m, H, lam = 3, 40, 2.5e-3
    env = env1(m=m, k=np.zeros(8))
    acts = np.full((H, oracle.MAX_THR), 7.0)       # padding entries must not count
    acts[:, :m] = rng.uniform(-1.5, 1.5, size=(H, m))
    wp = [0.3, 0.2, -0.6]
    L = _loss(env, state1(), acts, wp, weight=lam)
    expect = H * 0.49 + lam * np.sum(acts[:, :m] ** 2)
    assert L == pytest.approx(expect, rel=1e-14)


def test_p13_step_k_is_driven_by_action_row_k():
    """Two zero-order thrusters of equal gain at (0, +-0.1, 0) along +x give pure surge
    (pin P2) from force F_k = 2 g s_k |s_k|, s_k = clip(a_k); with linear surge damping the
    map is u_{k+1} = r u_k + (dt/M) F_k and p_{k+1} = p_k + dt u_{k+1}, so the loss follows
    from a scalar recurrence driven by row k at step k (a shifted row fails)."""
    rng = np.random.default_rng(11)
    H, dt, g, lam = 60, 0.01, 30.0, 1e-3
    env = _surge_env(dl=7.0)
    env["m"] = 2
    env["k"][0, :2] = g
    env["tau"][0, :2] = 0.0
    env["r"][0, 0] = [0.0, 0.1, 0.0]
    env["r"][0, 1] = [0.0, -0.1, 0.0]
    cmd = rng.uniform(-1.2, 1.2, size=H)
    acts = np.zeros((H, oracle.MAX_THR))
    acts[:, 0] = acts[:, 1] = cmd
    wp = np.array([0.05, 0.1, -0.2])
    r = 1.0 - dt * 7.0 / 15.0
    u, x, L = 0.0, 0.0, 0.0
    for kk in range(H):
        s = np.clip(cmd[kk], -1.0, 1.0)
        u = r * u + dt / 15.0 * 2.0 * g * s * abs(s)
        x += dt * u
        L += (x - wp[0]) ** 2 + wp[1] ** 2 + wp[2] ** 2 + lam * 2.0 * cmd[kk] ** 2
    got = _loss(env, state1(), acts, wp, weight=lam)
    assert abs(got - L) / L < 1e-12, (got, L)
