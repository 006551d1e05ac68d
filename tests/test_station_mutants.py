"""Planted mistakes in the station-keeping task oracle (``oracle/station.py``): each mutant
is a copy of the module with one plausible error (a transposed rotation, a missing
conjugate, a dropped or re-signed reward term, an off-by-one in the episode bookkeeping, a
swapped Euler order, a wrong generator counter). The pins of ``test_station_pins.py``
must fail on every one; a survivor means that part of the task oracle is not pinned."""
import importlib.util
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "station.py")
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import test_station_pins as P  # noqa: E402

MUTANTS = {
    "observe_uses_R_not_RT": ('np.einsum("nji,nj->ni", R, target[:, 0:3] - p)',
                              'np.einsum("nij,nj->ni", R, target[:, 0:3] - p)'),
    "observe_sign": ("target[:, 0:3] - p)", "p - target[:, 0:3])"),
    "error_without_conjugate": ("conj = q_target * np.array([1.0, -1.0, -1.0, -1.0])", "conj = q_target"),
    "error_order": ("qe = quat_mul(conj, q)", "qe = quat_mul(q, conj)"),
    "error_no_sign_fix": ("return np.where(qe[..., :1] < 0, -qe, qe)", "return qe"),
    "hamilton_sign": ("aw * bz + ax * by - ay * bx + az * bw", "aw * bz - ax * by + ay * bx + az * bw"),
    "rotation_transposed": ("np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)",
                            "np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], -1)"),
    "half_angle": ("q[..., 0] = np.cos(0.5 * angle)", "q[..., 0] = np.cos(angle)"),
    "euler_order": ("q0 = quat_mul(quat_mul(quat_axis(np.pi * (2.0 * u[:, 4] - 1.0), 2),\n"
                    "                           quat_axis(desc.tilt0 * (2.0 * u[:, 6] - 1.0), 1)),\n"
                    "                  quat_axis(desc.tilt0 * (2.0 * u[:, 5] - 1.0), 0))",
                    "q0 = quat_mul(quat_axis(desc.tilt0 * (2.0 * u[:, 5] - 1.0), 0),\n"
                    "              quat_mul(quat_axis(desc.tilt0 * (2.0 * u[:, 6] - 1.0), 1),\n"
                    "                       quat_axis(np.pi * (2.0 * u[:, 4] - 1.0), 2)))"),
    "target_yaw_axis": ("tgt[:, 3:7] = quat_axis(np.pi * (2.0 * u[:, 3] - 1.0), 2)",
                        "tgt[:, 3:7] = quat_axis(np.pi * (2.0 * u[:, 3] - 1.0), 0)"),
    "counter_episode_slot": ("ctr[..., 1] = (ep & np.uint64(0xFFFFFFFF))[:, None]", "ctr[..., 3] = (ep & np.uint64(0xFFFFFFFF))[:, None]"),
    "stream": ("STREAM_TASK = 8", "STREAM_TASK = 7"),
    "word_pairs": ("u[:, 1::2] = u53(w[..., 2], w[..., 3])", "u[:, 1::2] = u53(w[..., 3], w[..., 2])"),
    "reward_no_attitude": ("- desc.w_att * (1.0 - qe[:, 0] ** 2)", ""),
    "reward_sigma": ("np.exp(-d / desc.sigma_p)", "np.exp(-d * desc.sigma_p)"),
    "reward_unclipped_sum": ("np.mean(a_clipped[:, :m] ** 2, axis=1)", "np.sum(a_clipped[:, :m] ** 2, axis=1)"),
    "nonfinite_reward": ("r = np.where(finite, r, 0.0)", "r = r"),
    "tilt_column": ("up = rot(s[:, 3:7])[:, 2, 2]", "up = rot(s[:, 3:7])[:, 0, 0]"),
    "tilt_cos": ("(up < np.cos(desc.tilt_max))", "(up < desc.tilt_max)"),
    "distance_ge": ("(d > desc.d_max)", "(d > 2 * desc.d_max)"),
    "truncation_off_by_one": ("trunc = self.t >= d.max_steps", "trunc = self.t > d.max_steps"),
    "episode_not_advanced": ("self.episode[done] += 1", "self.episode[done] += 0"),
    "step_counter_not_reset": ("self.t[done] = 0", "self.t[done] = self.t[done]"),
    "final_after_reset": ("final = observe(self.state, self.target, m)\n        done = term | trunc",
                          "done = term | trunc"),
    "substeps_ignored": ("a, d.substeps, d.substeps)", "a, 1, 1)"),
    "start_velocity_scale": ("s[:, 7:13] = desc.v0 * (2.0 * u[:, 7:13] - 1.0)", "s[:, 7:13] = desc.v0 * u[:, 7:13]"),
}


def _load_mutant(name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutant {name}: pattern must occur once"
    text = text.replace(old, new)
    if name == "final_after_reset":
        text = text.replace("obs = observe(self.state, self.target, m)\n        return obs, r, term, trunc, final",
                            "obs = observe(self.state, self.target, m)\n        final = obs\n"
                            "        return obs, r, term, trunc, final")
    spec = importlib.util.spec_from_loader(f"station_mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod  # dataclasses look their module up there
    exec(compile(text, f"<station mutant {name}>", "exec"), mod.__dict__)
    return mod


PIN_TESTS = [
    lambda: P.test_hamilton_basis_products(),
    lambda: [P.test_rotation_of_axis_quaternion_is_textbook_matrix(a) for a in (0, 1, 2)],
    lambda: P.test_rotation_composes_like_the_product(),
    lambda: P.test_episode_start_is_zyx_euler_of_the_draws(),
    lambda: P.test_start_draw_distributions(),
    lambda: P.test_start_uniforms_use_the_published_generator(),
    lambda: P.test_observation_worked_example(),
    lambda: P.test_attitude_error_angle_matches_trace_formula(),
    lambda: P.test_reward_closed_forms(),
    lambda: P.test_termination_thresholds(),
    lambda: P.test_truncation_and_auto_reset(),
    lambda: P.test_non_finite_state_terminates_and_restarts(),
    lambda: P.test_substeps_hold_the_command(),
]


def test_unmutated_module_passes_the_pins():
    orig = P.S
    try:
        P.S = _load_mutant("none", "STREAM_TASK = 8", "STREAM_TASK = 8")
        for t in PIN_TESTS:
            t()
    finally:
        P.S = orig


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    orig = P.S
    P.S = _load_mutant(name, old, new)
    try:
        caught = False
        for t in PIN_TESTS:
            try:
                t()
            except (AssertionError, ValueError, IndexError, FloatingPointError):
                caught = True
                break
        assert caught, f"mutant {name} survived every pin"
    finally:
        P.S = orig
