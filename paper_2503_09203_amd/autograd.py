"""Differentiable rollouts through the hand-written adjoint kernels.

``RolloutFunction`` is a ``torch.autograd.Function`` whose forward runs
``mgx_rollout_forward`` (positions after every step; checkpoints every 32 steps) and whose
backward runs ``mgx_rollout_backward`` (per-segment recomputation and the reverse sweep
on the device). Gradients flow to the actions and to the per-environment linear and
quadratic damping and added mass.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import mgx


class DiffRollout:
    """Differentiable H-step rollouts of one batch from a fixed initial state.

    base_params: object with mass[N], added[6,N], dlin[6,N], dquad[6,N], buoy[N],
    current[3,N] (numpy float64); mass, buoyancy and current stay fixed.
    init_state: flat state tensor in the batch layout.
    """

    def __init__(self, batch: mgx.Batch, base_params, init_state, H, hold=1, ckpt=32):
        self.b = batch
        self.H, self.hold, self.ckpt = int(H), int(hold), int(ckpt)
        dev = batch.device
        f64 = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=dev)
        self.mass, self.buoy, self.current = f64(base_params.mass), f64(base_params.buoy), f64(base_params.current)
        self.init = init_state
        L = batch.layout
        npad_tot = L.n_pad_total
        # index maps from (padded, class-segmented) layouts to class-concatenated env order
        pos_idx, par_idx = [], []
        pad_off = 0
        for c in range(len(batch.m)):
            npad, n = batch.n_pad[c], batch.n[c]
            e = np.arange(n)
            pos_idx.append(np.stack([3 * pad_off + j * npad + e for j in range(3)]))
            par_idx.append(np.stack([18 * pad_off + j * npad + e for j in range(18)]))
            pad_off += npad
        self.pos_idx = torch.as_tensor(np.concatenate(pos_idx, axis=1), device=dev)   # [3, N]
        self.par_idx = torch.as_tensor(np.concatenate(par_idx, axis=1), device=dev)   # [18, N]
        self.pos_row = 3 * npad_tot
        self.par_len = 18 * npad_tot

    def set_params(self, dlin, dquad, added):
        self._p = [t.detach().to(torch.float64).contiguous() for t in (self.mass, added, dlin, dquad, self.buoy,
                                                                       self.current)]
        ptrs = dict(zip(("mass", "added", "dlin", "dquad", "buoy", "current"), (t.data_ptr() for t in self._p)))
        mgx.mgx_batch_set_params(self.b.h, ptrs, 1)

    def positions(self, pos):
        """[H, 3 * n_pad_total] -> [H, 3, N] (differentiable gather)."""
        return pos[:, self.pos_idx]

    def __call__(self, actions, dlin, dquad, added):
        return RolloutFunction.apply(actions, dlin, dquad, added, self)


class RolloutFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, actions, dlin, dquad, added, ro: DiffRollout):
        b = ro.b
        assert actions.dtype == b.dtype and actions.is_contiguous() and actions.shape[1] == b.layout.row_elems
        ro.set_params(dlin, dquad, added)
        b.set_state(ro.init)
        b.t = 0
        pos = torch.empty((ro.H, ro.pos_row), dtype=b.dtype, device=b.device)
        mgx.mgx_rollout_forward(b.h, ctypes.c_void_p(actions.data_ptr()), actions.shape[0], 0, ro.hold, ro.H, ro.ckpt,
                                ctypes.c_void_p(pos.data_ptr()))
        ctx.ro = ro
        ctx.actions = actions  # the kernels read it again in backward
        ctx.param_dtype = dlin.dtype
        return pos

    @staticmethod
    def backward(ctx, dpos):
        ro = ctx.ro
        b = ro.b
        dpos = dpos.to(b.dtype).contiguous()
        dact = torch.zeros_like(ctx.actions)
        dpar = torch.zeros(ro.par_len, dtype=b.dtype, device=b.device)
        mgx.mgx_rollout_backward(b.h, ctypes.c_void_p(dpos.data_ptr()), ctypes.c_void_p(dact.data_ptr()),
                                 ctypes.c_void_p(dpar.data_ptr()))
        g = dpar[ro.par_idx].to(ctx.param_dtype)   # [18, N]
        return dact, g[0:6], g[6:12], g[12:18], None
