"""Domain-randomisation sampler, plain numpy (Sec. III-C: each parameter drawn from a
uniform, Gaussian or custom piecewise distribution, resampled for chosen environments, with
ranges that may change between calls for a curriculum).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the device sampler is checked
against it; the product never imports it.

Convention shared with the device (both implement it from this description):
- generator: Philox4x32-10 (the published counter-based generator) with key
  (seed mod 2^32, 7 << 24) and counter (global env id, epoch mod 2^32, call j, 0) for
  j = 0..22; each call gives two uniforms on [0, 1) of 53 bits, (w0, w1) then (w2, w3).
- uniform slots: mass 0-1, added mass entry i 2+2i, 3+2i, linear damping 14+2i, 15+2i,
  quadratic damping 26+2i, 27+2i, buoyancy 38-39, current axis a 40+2a, 41+2a; a shared
  vector group uses its first entry's pair for every entry.
- uniform: lo + (hi - lo) u1. Gaussian: mean + std sqrt(-2 ln(1 - u1)) cos(2 pi u2),
  clipped to [lo, hi]. Piecewise (bins [e_k, e_k+1) with weights w_k): t = u1 W with W the
  sum of the weights, the first bin k with t < S_k+1 (S the running sums from the left;
  the last bin of positive weight if none), x = min(e_k + (t - S_k) / w_k (e_k+1 - e_k),
  e_k+1). Fixed: the nominal itself.
- relative groups multiply the class nominal by the draw; absolute ones take the draw.
"""
from __future__ import annotations

import numpy as np

from synth.philox import philox4x32, u53

STREAM_DR = 7
FIXED, UNIFORM, GAUSSIAN, PIECEWISE = 0, 1, 2, 3
GROUPS = (("mass", 1, 0), ("added", 6, 2), ("dlin", 6, 14), ("dquad", 6, 26), ("buoy", 1, 38), ("current", 3, 40))
NOMINAL_OFFSET = {"mass": 0, "added": 1, "dlin": 7, "dquad": 13, "buoy": 19, "current": 20}


def uniforms(seed: int, epoch: int, env_ids) -> np.ndarray:
    """[n, 46] uniforms for global env ids."""
    ids = np.asarray(env_ids, dtype=np.uint64)
    ctr = np.zeros((ids.size, 23, 4), dtype=np.uint64)
    ctr[..., 0] = ids[:, None]
    ctr[..., 1] = np.uint64(epoch & 0xFFFFFFFF)
    ctr[..., 2] = np.arange(23, dtype=np.uint64)[None, :]
    key = np.array([seed & 0xFFFFFFFF, STREAM_DR << 24], dtype=np.uint64)
    w = philox4x32(ctr, key)
    u = np.empty((ids.size, 46))
    u[:, 0::2] = u53(w[..., 0], w[..., 1])
    u[:, 1::2] = u53(w[..., 2], w[..., 3])
    return u


def draw(dist: dict, u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    """The distribution's value for uniforms u1, u2 (arrays)."""
    kind = dist["kind"]
    if kind == UNIFORM:
        return dist["lo"] + (dist["hi"] - dist["lo"]) * u1
    if kind == GAUSSIAN:
        z = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)
        return np.minimum(np.maximum(dist["mean"] + dist["std"] * z, dist["lo"]), dist["hi"])
    if kind == PIECEWISE:
        e = np.asarray(dist["edges"], dtype=np.float64)
        w = np.asarray(dist["weights"], dtype=np.float64)
        n = w.size
        S = np.zeros(n + 1)
        for k in range(n):
            S[k + 1] = S[k] + w[k]
        t = u1 * S[n]
        last = max(k for k in range(n) if w[k] > 0)
        out = np.empty_like(u1)
        for idx, tv in np.ndenumerate(t):
            k = next((k for k in range(n) if tv < S[k + 1]), last)
            out[idx] = min(e[k] + (tv - S[k]) / w[k] * (e[k + 1] - e[k]), e[k + 1])
        return out
    raise ValueError(f"unknown distribution kind {kind}")


def sample(spec: dict, nominal, env_ids, seed: int, epoch: int) -> dict:
    """Parameters of the listed environments (one class, nominal = its 23 values: mass,
    added[6], dlin[6], dquad[6], buoy, current[3]) as float64 arrays, component-major."""
    nominal = np.asarray(nominal, dtype=np.float64)
    u = uniforms(seed, epoch, env_ids)
    out = {}
    for name, size, slot in GROUPS:
        dist = spec.get(name, {"kind": FIXED})
        nom = nominal[NOMINAL_OFFSET[name]:NOMINAL_OFFSET[name] + size]
        vals = np.empty((size, u.shape[0]))
        for i in range(size):
            if dist["kind"] == FIXED:
                vals[i] = nom[i]
                continue
            s = slot if dist.get("shared", 0) else slot + 2 * i
            x = draw(dist, u[:, s], u[:, s + 1])
            vals[i] = nom[i] * x if dist.get("relative", 1) else x
        out[name] = vals[0] if size == 1 else vals
    return out
