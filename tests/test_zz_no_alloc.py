"""The allocation-free rollout (mgx_rollout_forward_static): through the C ABI its forward
positions, final state and reverse-mode gradients equal those of mgx_rollout_forward bit for
bit, on two calls in a row with the second smaller; sizes beyond the static array are
refused; a later static forward invalidates an earlier one's checkpoints."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2503_09203_amd import mgx

from gpu_helpers import torch

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _batch(n, horizon):
    t = torch()
    w = synth.differentiable(n=n, horizon=horizon)
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    b.set_params(w.params)
    b.set_state(t.tensor(b.pack_state([s.stacked() for s in w.state]), dtype=b.dtype, device=b.device))
    acts = t.tensor(b.pack_actions(w.actions(horizon)), dtype=b.dtype, device=b.device)
    return b, acts


def _run(static, n, horizon, ckpt):
    t = torch()
    b, acts = _batch(n, horizon)
    pos = t.zeros((horizon, 3 * b.layout.n_pad_total), dtype=b.dtype, device=b.device)
    fwd = mgx.mgx_rollout_forward_static if static else mgx.mgx_rollout_forward
    fwd(b.h, _vp(acts), acts.shape[0], 0, 1, horizon, ckpt, _vp(pos))
    dpos = t.sin(t.arange(pos.numel(), dtype=b.dtype, device=b.device).reshape(pos.shape))
    dact = t.zeros_like(acts)
    dpar = t.zeros((18 * b.layout.n_pad_total,), dtype=b.dtype, device=b.device)
    mgx.mgx_rollout_backward(b.h, _vp(dpos), _vp(dact), _vp(dpar))
    out = [pos, b.get_state(), dact, dpar]
    t.cuda.synchronize()
    assert b.t == horizon
    b.close()
    return out


def test_static_forward_equals_the_allocating_one_on_two_calls():
    t = torch()
    for n, horizon, ckpt in ((4096, 128, 32), (1000, 70, 16)):   # the second call smaller
        ref = _run(False, n, horizon, ckpt)
        got = _run(True, n, horizon, ckpt)
        for name, x, y in zip(("positions", "state", "action gradients", "parameter gradients"), got, ref):
            assert t.equal(x, y), (n, horizon, name)


def test_static_forward_refuses_sizes_beyond_the_array():
    b, acts = _batch(65536, 64)
    t = torch()
    pos = t.zeros((64, 3 * b.layout.n_pad_total), dtype=b.dtype, device=b.device)
    s0 = b.get_state().clone()
    with pytest.raises(mgx.MgxError) as e:
        # 2 x 64 x state_elems x 4 bytes of segment scratch alone is 704 MB
        mgx.mgx_rollout_forward_static(b.h, _vp(acts), acts.shape[0], 0, 1, 64, 64, _vp(pos))
    assert e.value.status == mgx.MGX_E_INVALID and "static scratch" in str(e.value)
    assert t.equal(b.get_state(), s0) and b.t == 0
    b.close()


def test_later_static_forward_invalidates_earlier_checkpoints():
    t = torch()
    b1, a1 = _batch(512, 40)
    b2, a2 = _batch(256, 40)
    p1 = t.zeros((40, 3 * b1.layout.n_pad_total), dtype=b1.dtype, device=b1.device)
    p2 = t.zeros((40, 3 * b2.layout.n_pad_total), dtype=b2.dtype, device=b2.device)
    mgx.mgx_rollout_forward_static(b1.h, _vp(a1), a1.shape[0], 0, 1, 40, 8, _vp(p1))
    mgx.mgx_rollout_forward_static(b2.h, _vp(a2), a2.shape[0], 0, 1, 40, 8, _vp(p2))
    with pytest.raises(mgx.MgxError) as e:
        mgx.mgx_rollout_backward(b1.h, _vp(t.ones_like(p1)), None, None)
    assert e.value.status == mgx.MGX_E_STATE
    mgx.mgx_rollout_backward(b2.h, _vp(t.ones_like(p2)), None, None)   # the latest one is intact
    t.cuda.synchronize()
    b1.close()
    b2.close()
