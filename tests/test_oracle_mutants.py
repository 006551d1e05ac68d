"""Planted mistakes: each mutant is a copy of the oracle with one plausible error (a
dropped term, a flipped sign, a swapped index, a transposed operand). The pin suite must
fail on every one of them; a mutant that survives means a part of the oracle is not
pinned. Runs on the CPU only; mutants are built in a temporary directory."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mgx_oracle.c")

MUTANTS = {
    "crb_sign": ("cross3(w, vw, t3);", "cross3(vw, w, t3);"),
    "payload_coriolis_order": ("cross3(env->rg, wxv, t5);", "cross3(wxv, env->rg, t5);"),
    "crb_rot_sign": ("cross3(w, Iw, t4);", "cross3(Iw, w, t4);"),
    "ca_lin_sign": ("cross3(w, A1vr, c1);", "cross3(A1vr, w, c1);"),
    "ca_ang_sign": ("cross3(vr, A1vr, c2);", "cross3(A1vr, vr, c2);"),
    "ca_uses_v_not_vr": ("A1vr[j] = env->added[j] * vr[j];", "A1vr[j] = env->added[j] * v[j];"),
    "damp_no_abs": ("fabs(nur[j])) * nur[j]", "nur[j]) * nur[j]"),
    "restore_sign": ("out->restore[j] = -(W - env->buoy) * gb[j];", "out->restore[j] = (W - env->buoy) * gb[j];"),
    "restore_moment_order": ("cross3(env->rb, gb, rbxg);\n    cross3(env->rg", "cross3(gb, env->rb, rbxg);\n    cross3(env->rg"),
    "gravity_row": ("gb[j] = R[2][j];", "gb[j] = R[j][2];"),
    "current_transposed": ("vc[j] = R[0][j] * env->current[0] + R[1][j] * env->current[1] + R[2][j] * env->current[2];",
                           "vc[j] = R[j][0] * env->current[0] + R[j][1] * env->current[1] + R[j][2] * env->current[2];"),
    "vr_sign": ("vr[j] = v[j] - vc[j];", "vr[j] = v[j] + vc[j];"),
    "no_hadd": ("int amc = !(env->flags & ORC_FLAG_NO_AMC);", "int amc = 0;"),
    "hadd_order": ("cross3(w, vc, wxvc);", "cross3(vc, w, wxvc);"),
    "mass_no_added": ("for (int j = 0; j < 6; ++j) M[6 * j + j] += env->added[j];", ""),
    "inertia_index": ("(i == j ? env->inertia[i] + env->mass * r2 : 0.0)",
                      "(i == j ? env->inertia[(i + 1) % 3] + env->mass * r2 : 0.0)"),
    "payload_rotation_order": ("cross3(w, env->rg, wxr);", "cross3(env->rg, w, wxr);"),
    "payload_restoring_sign": ("env->buoy * rbxg[j] - W * rgxg[j]", "env->buoy * rbxg[j] + W * rgxg[j]"),
    "parallel_axis_sign": ("- env->mass * r[i] * r[j];", "+ env->mass * r[i] * r[j];"),
    "mass_coupling_sign": ("M[6 * i + 3 + j] = -m * S[i][j];", "M[6 * i + 3 + j] = m * S[i][j];"),
    "payload_coriolis_dropped": ("out->crb[3 + j] = env->mass * t5[j] + t4[j];", "out->crb[3 + j] = t4[j];"),
    "position_transposed": ("s->p[j] += env->dt * (R[j][0] * nun[0] + R[j][1] * nun[1] + R[j][2] * nun[2]);",
                            "s->p[j] += env->dt * (R[0][j] * nun[0] + R[1][j] * nun[1] + R[2][j] * nun[2]);"),
    "position_old_velocity": ("s->p[j] += env->dt * (R[j][0] * nun[0] + R[j][1] * nun[1] + R[j][2] * nun[2]);",
                              "s->p[j] += env->dt * (R[j][0] * s->nu[0] + R[j][1] * s->nu[1] + R[j][2] * s->nu[2]);"),
    "attitude_left_mult": ("orc_quat_mul(s->q, dq, qn);", "orc_quat_mul(dq, s->q, qn);"),
    "attitude_full_angle": ("double half = 0.5 * wn * env->dt;", "double half = wn * env->dt;"),
    "rotation_sign": ("R[0][1] = 2.0 * (x * y - w * z);", "R[0][1] = 2.0 * (x * y + w * z);"),
    "thrust_moment_order": ("cross3(env->r[i], e, mom);", "cross3(e, env->r[i], mom);"),
    "thrust_no_sign": ("double f = gain * s * fabs(s);", "double f = gain * s * s;"),
    "reverse_gain_ignored": ("if (s < 0.0 && env->k_rev[i] > 0.0) gain = env->k_rev[i];", ""),
    "reverse_gain_forward": ("if (s < 0.0 && env->k_rev[i] > 0.0) gain = env->k_rev[i];",
                             "if (s > 0.0 && env->k_rev[i] > 0.0) gain = env->k_rev[i];"),
    "shaft_torque_sign": ("tau[3 + j] += f * mom[j] + env->reaction[i] * f * e[j];",
                          "tau[3 + j] += f * mom[j] - env->reaction[i] * f * e[j];"),
    "shaft_torque_dropped": ("tau[3 + j] += f * mom[j] + env->reaction[i] * f * e[j];", "tau[3 + j] += f * mom[j];"),
    "fin_alpha_sign": ("double alpha = env->fin_max[i] * n[i] - atan2(un, uc);",
                       "double alpha = env->fin_max[i] * n[i] + atan2(un, uc);"),
    "fin_lift_direction": ("cross3(s, up, lift_dir);", "cross3(up, s, lift_dir);"),
    "fin_drag_sign": ("F[j] = L * lift_dir[j] - D * up[j];", "F[j] = L * lift_dir[j] + D * up[j];"),
    "fin_ignores_rotation": ("u[j] = vr[j] + wxr[j];", "u[j] = vr[j];"),
    "fin_rotation_order": ("cross3(w, env->r[i], wxr);", "cross3(env->r[i], w, wxr);"),
    "fin_moment_order": ("cross3(env->r[i], F, mom);", "cross3(F, env->r[i], mom);"),
    "fin_keeps_span_flow": ("double speed2 = uc * uc + un * un;",
                            "double speed2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];"),
    "fin_not_deflected": ("double alpha = env->fin_max[i] * n[i] - atan2(un, uc);",
                          "double alpha = -atan2(un, uc);"),
    "shaft_torque_unsigned": ("tau[3 + j] += f * mom[j] + env->reaction[i] * f * e[j];",
                              "tau[3 + j] += f * mom[j] + env->reaction[i] * fabs(f) * e[j];"),
    "lag_euler_always": ("return 1.0 - exp(-env->dt / env->tau[i]);", "return env->dt / env->tau[i];"),
    "lag_before_clip": ("nl[i] = env->tau[i] > 0.0 ? s->n[i] + orc_lag_factor(env, i) * (c - s->n[i]) : c;",
                        "nl[i] = env->tau[i] > 0.0 ? s->n[i] + orc_lag_factor(env, i) * (a[i] - s->n[i]) : c;"),
    "thrust_from_old_rotor": ("orc_terms_eval(env, s->q, s->nu, nl, &t);", "orc_terms_eval(env, s->q, s->nu, s->n, &t);"),
    "quat_product_sign": ("out[1 + j] = a[0] * bv[j] + b[0] * av[j] + c[j];", "out[1 + j] = a[0] * bv[j] + b[0] * av[j] - c[j];"),
    "loss_position_before_step": ("orc_step(&envs[e], &s, a, 0);\n            double d0 = s.p[0] - w[0], d1 = s.p[1] - w[1], d2 = s.p[2] - w[2];",
                                  "double d0 = s.p[0] - w[0], d1 = s.p[1] - w[1], d2 = s.p[2] - w[2];\n            orc_step(&envs[e], &s, a, 0);"),
    "loss_drops_last_step": ("for (int32_t k = 0; k < horizon; ++k) {\n            const double* a = actions + (e * horizon + k)",
                             "for (int32_t k = 0; k < horizon - 1; ++k) {\n            const double* a = actions + (e * horizon + k)"),
    "loss_waypoint_axis": ("d1 = s.p[1] - w[1]", "d1 = s.p[1] - w[0]"),
    "loss_penalty_all_rows": ("for (int i = 0; i < envs[e].m; ++i) aa += a[i] * a[i];",
                              "for (int i = 0; i < ORC_MAX_THR; ++i) aa += a[i] * a[i];"),
    "loss_penalty_clipped": ("for (int i = 0; i < envs[e].m; ++i) aa += a[i] * a[i];",
                             "for (int i = 0; i < envs[e].m; ++i) aa += fmin(a[i] * a[i], 1.0);"),
    "loss_action_row_shift": ("const double* a = actions + (e * horizon + k) * ORC_MAX_THR;",
                              "const double* a = actions + (e * horizon + (k + 1) % horizon) * ORC_MAX_THR;"),
}


def _build(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant {name}: pattern not unique"
    mdir = os.path.join(tmp, name)
    os.makedirs(mdir)
    path = os.path.join(mdir, "mgx_oracle.c")
    open(path, "w").write(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "mgx_oracle.h")
    lib = os.path.join(mdir, "lib.so")
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                           "-fPIC", "-shared", "-D_GNU_SOURCE", "-I", os.path.dirname(hdr), path, "-o", lib,
                           "-lm"])
    return lib


def test_every_planted_mistake_is_caught(tmp_path):
    from concurrent.futures import ThreadPoolExecutor

    def run(item):
        name, (old, new) = item
        lib = _build(str(tmp_path), name, old, new)
        env = dict(os.environ, MGX_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py")], env=env, cwd=ROOT,
                           capture_output=True, text=True)
        return name, r.returncode

    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(run, MUTANTS.items()))
    survivors = [n for n, rc in results if rc == 0]
    assert not survivors, f"pins did not catch: {survivors}"
