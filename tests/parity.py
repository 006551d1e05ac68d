"""Parity metric between the device path (float32 or float64) and the FP64 oracle."""
import numpy as np


def component_errors(gpu, ref):
    """gpu, ref: [C, N] one step's state components. Per component c:
    max_env |x_gpu - x_ref| / max(|x_ref|, rms_c), rms_c the batch RMS of the reference."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref * ref, axis=1, keepdims=True))
    floor = np.maximum(np.abs(ref), np.maximum(rms, 1e-30))
    return np.max(np.abs(gpu - ref) / floor, axis=1)


def geodesic(qa, qb):
    """Rotation angle between quaternion columns [4, N] (sign-insensitive)."""
    d = np.abs(np.sum(np.asarray(qa, dtype=np.float64) * np.asarray(qb, dtype=np.float64), axis=0))
    return 2 * np.arccos(np.clip(d, 0, 1))


# Rudder-workload environments (of 65,536) whose trajectories amplify rounding the most:
# the ten largest drifts of the FP64 oracle with its state rounded to float32 after every
# step, against itself, after 1000 steps (recomputed by tests/test_conditioning.py).
RUDDER_SENSITIVE = np.array([39754, 26752, 49185, 13584, 29825, 21597, 5733, 64156, 26187, 14274])
