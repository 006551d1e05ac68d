"""The batch boundary on the device: caller-owned state and record buffers adopted in place,
a caller's allocator for every library buffer, and the device-side parameter check that
refuses an invalid or not positive definite mass matrix without changing the batch."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_2503_09203_amd import mgx

from gpu_helpers import device_actions, make_batch, torch

pytestmark = pytest.mark.gpu


def _packed_state(w):
    b = mgx.Batch(w.classes, w.n_envs, w.dt)
    flat = b.pack_state([s.stacked() for s in w.state])
    b.close()
    return flat


def test_adopted_state_is_stepped_in_place_and_outlives_the_batch():
    """A torch tensor passed as the state is the batch's state: stepping moves it in place,
    bit for bit as a library-owned batch moves, its valid slots survive creation, and
    destroying the batch leaves the tensor alive and unchanged."""
    t = torch()
    w = synth.randomised(n=1000, steps=40)
    acts = w.actions(4)
    plan = mgx.mgx_batch_plan([mgx.mgx_class_define(c) for c in w.classes], w.n_envs, w.dt)
    flat = _packed_state(w)
    assert flat.size == plan.state_elems
    state = t.tensor(flat, dtype=t.float32, device="cuda:0")
    record = t.full((plan.record_elems,), 7.0, dtype=t.float32, device="cuda:0")
    b = mgx.Batch(w.classes, w.n_envs, w.dt, state=state, record=record)
    assert t.equal(state, t.tensor(flat, dtype=t.float32, device="cuda:0"))   # valid slots kept, padding at rest
    b.set_params(w.params)
    b.step(device_actions(b, acts), 40, hold=10)
    ref = make_batch(w)
    ref.step(device_actions(ref, acts), 40, hold=10)
    assert t.equal(b.get_state(), state)          # the batch's state is the caller's tensor
    assert t.equal(state, ref.get_state())        # and moved exactly as a library-owned one
    assert not t.equal(state, t.tensor(flat, dtype=t.float32, device="cuda:0"))
    snap = state.clone()
    b.close()
    ref.close()
    t.cuda.synchronize()
    assert t.equal(state, snap)                   # not freed, not touched by destroy
    assert record[0].item() != 7.0                # the record was built in the caller's buffer


def test_torch_allocator_takes_every_library_buffer():
    """With torch's caching allocator, the batch (including the rollout checkpoints
    allocated on first use) gives the same results, and destroy returns every buffer."""
    t = torch()
    w = synth.differentiable(n=256, horizon=64)
    acts = w.actions(64)
    outs = []
    for use in (False, True):
        b = mgx.Batch(w.classes, w.n_envs, w.dt, torch_allocator=use)
        b.set_params(w.params)
        b.set_state(t.tensor(b.pack_state([s.stacked() for s in w.state]), dtype=b.dtype, device=b.device))
        a = device_actions(b, acts)
        pos = t.zeros((64, 3 * b.layout.n_pad_total), dtype=b.dtype, device=b.device)
        mgx.mgx_rollout_forward(b.h, ctypes.c_void_p(a.data_ptr()), a.shape[0], 0, 1, 64, 32,
                                ctypes.c_void_p(pos.data_ptr()))
        dp = t.ones_like(pos)
        dact = t.zeros_like(a)
        mgx.mgx_rollout_backward(b.h, ctypes.c_void_p(dp.data_ptr()), ctypes.c_void_p(dact.data_ptr()), None)
        outs.append((b.get_state(), pos.clone(), dact.clone()))
        alloc = b._allocator
        if use:
            assert len(alloc.live) >= 10      # state, record, bookkeeping, checkpoints, scratch
        b.close()
        if use:
            assert alloc.live == {}
    for x, y in zip(outs[0], outs[1]):
        assert t.equal(x, y)


def _status(fn):
    with pytest.raises(mgx.MgxError) as e:
        fn()
    return e.value.status


def test_device_parameter_check_refuses_and_leaves_the_batch_unchanged():
    """Device-resident parameters are checked before any record is written: a non-finite
    mass is MGX_E_INVALID, an added-mass entry that makes a diagonal entry of M_RB + M_A
    non-positive is MGX_E_NOT_SPD, and in both cases the stored parameters and the stepping
    are those of the last accepted call."""
    w = synth.randomised(n=300, steps=10)
    b = make_batch(w)
    before = b.get_params()
    bad = w.params.subset(np.arange(300))
    bad.mass = bad.mass.copy()
    bad.mass[17] = np.nan
    assert _status(lambda: b.set_params(bad)) == mgx.MGX_E_INVALID
    bad = w.params.subset(np.arange(300))
    bad.added = bad.added.copy()
    bad.added[3, 5] = -(w.classes[0].inertia[0] + 0.5)
    assert _status(lambda: b.set_params(bad)) == mgx.MGX_E_NOT_SPD
    assert _status(lambda: b.set_params(bad, on_device=False)) == mgx.MGX_E_NOT_SPD
    after = b.get_params()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    # a negative added-mass entry that keeps M positive definite is accepted
    ok = w.params.subset(np.arange(300))
    ok.added = ok.added.copy()
    ok.added[0, 9] = -0.5
    b.set_params(ok)
    assert b.get_params()["added"][0, 9] == np.float32(-0.5)
    b.step(device_actions(b, w.actions(1)), 5, hold=10, flags=mgx.STEP_STATS)
    assert b.check() == (mgx.MGX_OK, 0)
    b.close()


def test_unchecked_device_parameters_report_through_the_error_word():
    """on_device = 2 skips the prior check and the wait: the same invalid added mass is
    accepted by the call, its environment gets a NaN record (non-finite after a step) and
    mgx_batch_check reports MGX_E_NOT_SPD."""
    t = torch()
    w = synth.randomised(n=300, steps=10)
    b = make_batch(w)
    bad = w.params.subset(np.arange(300))
    bad.added = bad.added.copy()
    bad.added[3, 5] = -(w.classes[0].inertia[0] + 0.5)
    keep = {k: t.as_tensor(np.ascontiguousarray(getattr(bad, k), dtype=np.float64), device=b.device)
            for k in ("mass", "added", "dlin", "dquad", "buoy", "current")}
    mgx.mgx_batch_set_params(b.h, {k: v.data_ptr() for k, v in keep.items()}, 2)
    b.step(device_actions(b, w.actions(1)), 5, hold=10, flags=mgx.STEP_STATS)
    st, nf = b.check()
    assert st == mgx.MGX_E_NOT_SPD
    state = b.unpack_state(b.get_state().cpu().numpy())[0]
    finite = np.all(np.isfinite(state), axis=0)
    assert not finite[5] and finite.sum() == 299
    b.close()


def test_payload_mass_matrix_that_is_not_positive_definite_is_refused():
    """With a payload every diagonal entry of M can be positive while M is not positive
    definite (the centre of gravity couples surge and heave with pitch): the Cholesky check
    on the device refuses it with MGX_E_NOT_SPD."""
    w = synth.payload(n=128, steps=10)
    c = w.classes[0]
    b = make_batch(w)
    p = w.params.subset(np.arange(128))
    p.added = p.added.copy()
    e = 40
    m, rg = p.mass[e], c.rg
    couple = (m * rg[2]) ** 2 / (m + p.added[0, e]) + (m * rg[0]) ** 2 / (m + p.added[2, e])
    p.added[4, e] = -(c.inertia[1] + m * (rg[0] ** 2 + rg[2] ** 2)) + 0.5 * couple
    M = oracle.mass_matrix(oracle.make_envs(c, p.subset(np.array([e])), w.dt))
    assert np.all(np.diag(M) > 0) and np.linalg.eigvalsh(M).min() < 0    # the case meant
    assert _status(lambda: b.set_params(p)) == mgx.MGX_E_NOT_SPD
    b.step(device_actions(b, w.actions(1)), 5, hold=10, flags=mgx.STEP_STATS)
    assert b.check() == (mgx.MGX_OK, 0)         # still the valid parameters of make_batch
    b.close()
