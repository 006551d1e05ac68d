"""Shared set-up for GPU tests: builds a device batch and the matching oracle inputs from
one synthetic workload, and runs both over the same steps."""
import numpy as np

import oracle
import synth
from paper_2503_09203_amd import mgx


def torch():
    import torch as _t
    return _t


def make_batch(w, precision=mgx.FP32, flags=0):
    t = torch()
    b = mgx.Batch(w.classes, w.n_envs, w.dt, precision, flags)
    b.set_params(w.params)
    init = b.pack_state([s.stacked() for s in w.state])
    b.set_state(t.tensor(init, dtype=b.dtype, device=b.device))
    return b


def oracle_inputs(w, flags=0):
    """Per-class (envs, AoS state) for the oracle."""
    out, off = [], 0
    for c, n, st in zip(w.classes, w.n_envs, w.state):
        envs = oracle.make_envs(c, w.params.subset(np.arange(off, off + n)), w.dt, flags)
        out.append((envs, oracle.pack_state(st.p, st.q, st.nu, st.n)))
        off += n
    return out


def device_actions(b, per_class):
    t = torch()
    return t.tensor(b.pack_actions(per_class), dtype=b.dtype, device=b.device)


def run_pair(w, per_class_actions, hold, checkpoints, precision=mgx.FP32, flags=0, sample=None, chunk=None,
             shape=None, final_state=None):
    """Advance the device batch and the oracle to each checkpoint step; return a list of
    (k, [(gpu [C,n], ref [C,n]) per class]). ``sample``: per-class env indices given to
    the oracle (all if None). ``chunk``: split each device call into launches of this many
    steps (the launch configuration of the benchmark). ``shape``: arguments of
    ``Batch.set_shape`` (launch mode, K, block, blocks per CU). ``final_state``: a list that
    receives the device state (flat layout, on the host) after the last checkpoint."""
    b = make_batch(w, precision, flags)
    if shape is not None:
        b.set_shape(*shape)
    acts = device_actions(b, per_class_actions)
    rows = acts.shape[0]
    ins = oracle_inputs(w, flags)
    if sample is not None:
        ins = [(e[s], st[s]) for (e, st), s in zip(ins, sample)]
    ora_actions = [oracle.pack_actions(a) for a in per_class_actions]
    if sample is not None:
        ora_actions = [a[s] for a, s in zip(ora_actions, sample)]
    states = [st.copy() for _, st in ins]
    out, t = [], 0
    for k in checkpoints:
        n = k - t
        done = 0
        while done < n:
            kk = n - done if chunk is None else min(chunk, n - done)
            b.step(acts, kk, hold=hold)
            done += kk
        for c, (envs, _) in enumerate(ins):
            states[c], _, _ = oracle.rollout(envs, states[c], ora_actions[c], hold, n, t0=t)
        t = k
        flat = b.get_state().cpu().numpy().astype(np.float64)
        gpu = b.unpack_state(flat)
        pairs = []
        for c in range(len(ins)):
            g = gpu[c] if sample is None else gpu[c][:, sample[c]]
            pairs.append((g, oracle.unpack_state(states[c], w.classes[c].m)))
        out.append((k, pairs))
    if final_state is not None:
        final_state.append(flat)
    b.close()
    return out
