"""Gradients of a rollout loss through the hand-written adjoint kernels, against central
finite differences (h = 1e-4) of the FP64 oracle's loss.

Workload: the 8-thruster class, per-step actions, horizon 256, loss
sum_k |p_k - w|^2 + 1e-3 |a_{k-1}|^2 with a N(0, 2^2) waypoint per environment; gradients
with respect to every action and to each environment's d_L, d_Q and added mass. The loss
separates over environments, so each finite difference perturbs one environment only.
Bar: |g - g_fd| <= tol * max(|g_fd|, rms of that gradient block), tol = 1e-3 in float32
and 1e-5 in float64. The float64 bar is set by the finite differences, not the adjoint:
thrust k n|n| and quadratic damping d_Q |x| x have a kink in their second derivative at
zero, and a central difference of width 2h across such a crossing carries an O(h) error
(observed up to ~1.3e-6 relative on single entries, against ~1e-9 elsewhere)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2503_09203_amd import mgx

from gpu_helpers import torch

pytestmark = pytest.mark.gpu

H = 256
FD_H = 1e-4


def _setup(n, precision, variants=False):
    t = torch()
    from paper_2503_09203_amd.autograd import DiffRollout
    w = synth.differentiable(n=n, horizon=H)
    if variants:
        w.classes[0] = synth.propeller_variants(w.classes[0])
    b = mgx.Batch(w.classes, w.n_envs, w.dt, precision)
    init = t.tensor(b.pack_state([w.state[0].stacked()]), dtype=b.dtype, device=b.device)
    ro = DiffRollout(b, w.params, init, H, hold=1)
    acts_np = w.actions(H)[0]                                     # [H, m, N]
    actions = t.tensor(b.pack_actions([acts_np]), dtype=b.dtype, device=b.device, requires_grad=True)
    dev = b.device
    f = lambda x: t.tensor(np.ascontiguousarray(x), dtype=t.float64, device=dev, requires_grad=True)
    dl, dq, am = f(w.params.dlin), f(w.params.dquad), f(w.params.added)
    return w, b, ro, acts_np, actions, dl, dq, am


def _loss(ro, actions, dl, dq, am, wp):
    t = torch()
    pos = ro.positions(ro(actions, dl, dq, am))                   # [H, 3, N]
    d = pos.to(t.float64) - wp[None]
    return (d * d).sum() + 1e-3 * (actions.to(t.float64) ** 2).sum()


def _fd_oracle(w, acts_np, envs_idx):
    """Central differences of the oracle loss for the listed environments:
    returns (g_actions [len, H, m], g_params [len, 18])."""
    cls = w.classes[0]
    m = cls.m
    wp_all = w.extra["waypoints"]
    st0 = w.state[0]
    x0_all = oracle.pack_state(st0.p, st0.q, st0.nu, st0.n)
    out_a, out_p = [], []
    for e in envs_idx:
        p1 = w.params.subset(np.array([e]))
        base_env = oracle.make_envs(cls, p1, w.dt)
        a0 = np.zeros((H, oracle.MAX_THR))
        a0[:, :m] = acts_np[:, :, e]
        n_dir = H * m + 18
        envs = np.repeat(base_env, 2 * n_dir)
        acts = np.repeat(a0[None], 2 * n_dir, axis=0)
        for d in range(H * m):
            k, i = divmod(d, m)
            acts[2 * d, k, i] += FD_H
            acts[2 * d + 1, k, i] -= FD_H
        for j in range(18):
            r = 2 * (H * m + j)
            field, jj = ("dlin", j) if j < 6 else (("dquad", j - 6) if j < 12 else ("added", j - 12))
            envs[field][r, jj] += FD_H
            envs[field][r + 1, jj] -= FD_H
        x0 = np.repeat(x0_all[e:e + 1], 2 * n_dir, axis=0)
        wps = np.repeat(wp_all[:, e][None], 2 * n_dir, axis=0)
        L = oracle.rollout_loss(envs, x0, acts, H, wps, 1e-3)
        g = (L[0::2] - L[1::2]) / (2 * FD_H)
        out_a.append(g[:H * m].reshape(H, m))
        out_p.append(g[H * m:])
    return np.array(out_a), np.array(out_p)


def _check_block(g, g_fd, tol, mask=None, label=""):
    if mask is not None:
        g, g_fd = g[mask], g_fd[mask]
    rms = np.sqrt(np.mean(g_fd ** 2))
    err = np.abs(g - g_fd) / np.maximum(np.abs(g_fd), rms)
    print(label, f"max rel err {err.max():.2e} (rms {rms:.3e})", flush=True)
    assert err.max() <= tol, (label, err.max())


@pytest.mark.parametrize("precision,tol,variants", [(mgx.FP64, 1e-5, False), (mgx.FP32, 1e-3, False),
                                                    (mgx.FP32, 1e-3, True)])
def test_rollout_gradients_match_oracle_finite_differences(precision, tol, variants):
    """variants: the class with dead zones, reverse gains and shaft torques."""
    t = torch()
    n = 16
    w, b, ro, acts_np, actions, dl, dq, am = _setup(n, precision, variants)
    wp = t.tensor(w.extra["waypoints"], dtype=t.float64, device=b.device)
    loss = _loss(ro, actions, dl, dq, am, wp)
    loss.backward()
    ga = b.unpack_actions(actions.grad.detach().cpu().numpy().astype(np.float64))[0]   # [H, m, N]
    gp = np.concatenate([dl.grad.cpu().numpy(), dq.grad.cpu().numpy(), am.grad.cpu().numpy()])  # [18, N]
    fd_a, fd_p = _fd_oracle(w, acts_np, range(n))
    ok = np.abs(np.transpose(acts_np, (2, 0, 1))) < 1 - 2 * FD_H
    _check_block(np.transpose(ga, (2, 0, 1)), fd_a, tol, ok, f"actions p{precision}")
    for blk, name in ((slice(0, 6), "d_L"), (slice(6, 12), "d_Q"), (slice(12, 18), "M_A")):
        _check_block(gp[blk].T, fd_p[:, blk], tol, None, f"{name} p{precision}")
    # the loss itself agrees with the oracle's
    cls = w.classes[0]
    envs = oracle.make_envs(cls, w.params, w.dt)
    st0 = w.state[0]
    a_orc = np.zeros((n, H, oracle.MAX_THR))
    a_orc[:, :, :cls.m] = np.transpose(acts_np, (2, 0, 1))
    L = oracle.rollout_loss(envs, oracle.pack_state(st0.p, st0.q, st0.nu, st0.n), a_orc, H,
                            w.extra["waypoints"].T, 1e-3)
    assert abs(loss.item() - L.sum()) <= (1e-9 if precision == mgx.FP64 else 1e-4) * abs(L.sum())
    b.close()


def test_full_size_gradients_sampled():
    """8192 environments, horizon 256, float32; 8 sampled environments against the oracle."""
    t = torch()
    w, b, ro, acts_np, actions, dl, dq, am = _setup(8192, mgx.FP32)
    wp = t.tensor(w.extra["waypoints"], dtype=t.float64, device=b.device)
    loss = _loss(ro, actions, dl, dq, am, wp)
    loss.backward()
    idx = np.array([0, 1, 777, 2048, 4095, 5000, 8000, 8191])
    ga = b.unpack_actions(actions.grad.detach().cpu().numpy().astype(np.float64))[0][:, :, idx]
    gp = np.concatenate([dl.grad.cpu().numpy(), dq.grad.cpu().numpy(), am.grad.cpu().numpy()])[:, idx]
    fd_a, fd_p = _fd_oracle(w, acts_np, idx)
    ok = np.abs(np.transpose(acts_np[:, :, idx], (2, 0, 1))) < 1 - 2 * FD_H
    _check_block(np.transpose(ga, (2, 0, 1)), fd_a, 1e-3, ok, "actions 8192")
    for blk, name in ((slice(0, 6), "d_L"), (slice(6, 12), "d_Q"), (slice(12, 18), "M_A")):
        _check_block(gp[blk].T, fd_p[:, blk], 1e-3, None, f"{name} 8192")
    b.close()


def test_backward_requires_a_forward():
    w = synth.differentiable(n=64, horizon=8)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    b.set_params(w.params)
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_rollout_backward(b.h, None, None, None)
    assert e.value.status == mgx.MGX_E_STATE
    b.close()


@pytest.mark.parametrize("make,word", [(synth.rudders, "has fins"), (synth.payload, "payload")])
def test_fin_and_payload_classes_are_refused(make, word):
    t = torch()
    w = make(n=64, steps=8)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    b.set_params(w.params)
    acts = b.gen_actions(8, seed=1)
    pos = t.zeros((8, 3 * b.layout.n_pad_total), dtype=b.dtype, device=b.device)
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_rollout_forward(b.h, acts.data_ptr(), acts.shape[0], 0, 1, 8, 4, pos.data_ptr())
    assert word in str(e.value)
    b.close()


def test_classes_in_one_batch_match_each_class_alone():
    """Two classes in one batch (4 and 8 thrusters; 70 and 200 environments, so ragged
    tiles; horizon 70, so a short last segment) give, bit for bit in float32, the positions
    and gradients of each class run in a batch of its own: each class works in its own block
    of the checkpoint, recompute and tape buffers."""
    t = torch()
    from paper_2503_09203_amd.autograd import DiffRollout
    Hs = 70
    classes = [synth.draw_class(4, 0), synth.draw_class(8, 4)]
    ns = [70, 200]
    w = synth.mixed(classes, ns, steps=Hs, hold=1)
    acts = w.actions(Hs)
    wp_all = synth.waypoints(sum(ns))

    def run(cls_idx):
        cl = [classes[c] for c in cls_idx]
        b = mgx.Batch(cl, [ns[c] for c in cls_idx], w.dt, mgx.FP32)
        offs = np.cumsum([0] + ns)
        idx = np.concatenate([np.arange(offs[c], offs[c + 1]) for c in cls_idx])
        params = w.params.subset(idx)
        init = t.tensor(b.pack_state([w.state[c].stacked() for c in cls_idx]), dtype=b.dtype, device=b.device)
        ro = DiffRollout(b, params, init, Hs, hold=1)
        a = t.tensor(b.pack_actions([acts[c] for c in cls_idx]), dtype=b.dtype, device=b.device, requires_grad=True)
        f = lambda x: t.tensor(np.ascontiguousarray(x), dtype=t.float64, device=b.device, requires_grad=True)
        dl, dq, am = f(params.dlin), f(params.dquad), f(params.added)
        wp = t.tensor(wp_all[:, idx], dtype=t.float64, device=b.device)
        pos = ro.positions(ro(a, dl, dq, am))
        d = pos.to(t.float64) - wp[None]
        ((d * d).sum() + 1e-3 * (a.to(t.float64) ** 2).sum()).backward()
        out = dict(pos=pos.detach().cpu().numpy(),
                   ga=b.unpack_actions(a.grad.detach().cpu().numpy()),
                   gp=np.concatenate([dl.grad.cpu().numpy(), dq.grad.cpu().numpy(), am.grad.cpu().numpy()]))
        b.close()
        return out

    both = run([0, 1])
    off = 0
    for c in range(2):
        alone = run([c])
        sl = slice(off, off + ns[c])
        assert np.array_equal(both["pos"][:, :, sl], alone["pos"]), f"positions of class {c}"
        assert np.array_equal(both["ga"][c], alone["ga"][0]), f"action gradients of class {c}"
        assert np.array_equal(both["gp"][:, sl], alone["gp"]), f"parameter gradients of class {c}"
        assert np.abs(alone["gp"]).max() > 0 and np.abs(alone["ga"][0]).max() > 0
        off += ns[c]
