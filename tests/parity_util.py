"""Helpers for GPU-vs-oracle parity (test infrastructure).

Tolerance (FP32 GPU vs FP64 oracle): |a - b| <= 1e-4 * max(|b|, floor) per
state component with floors 2 cm (position), 1 (quaternion), 0.1 m/s
(velocity), 1 rad/s (angular velocity); sensor force magnitudes use a 1 N
floor.  A step (or a segment of steps) of one simulation is *non-chaotic*
when the oracle run from the double-precision state and the run from its
float32-rounded copy agree to 1e-6 (same floors) with identical contact
sets; parity is asserted there, and contact sets must then match exactly,
except at a tie of the contact cap: when the oracle's last kept and first
dropped candidates have gaps within CAP_TIE (below the float32 resolution of
a gap, about 1e-8 m at these sizes) either choice is a correct result, and
the sets may differ by those candidates.

Sensor forces are compared on the scale of the simulation's contact forces:
|a - b| <= 1e-4 * F with F = max(1 N, largest sensor force of that
simulation).  With redundant contacts the split of force between links
(internal squeeze) is set by the compliance and is conditioned like the
whole contact solve, not like each link's own magnitude.
"""
import numpy as np

FLOORS = np.array([0.02] * 3 + [1.0] * 4 + [0.1] * 3 + [1.0] * 3)
TOL = 1e-4
CHAOS_TOL = 1e-6
FORCE_FLOOR = 1.0
CAP_TIE = 1e-7


def keys_match(gpu_keys, ora_keys, diag=None):
    """Per-env: contact sets equal, or differing by at most one swapped pair
    at a cap tie reported by the oracle."""
    out = []
    for i, (a, b) in enumerate(zip(key_sets(gpu_keys), key_sets(ora_keys))):
        if a == b:
            out.append(True)
            continue
        tie = diag is not None and (diag["d_first_dropped"][i] - diag["d_last_kept"][i]) < CAP_TIE
        out.append(bool(tie and len(a) == len(b) and len(a ^ b) <= 2))
    return np.array(out)


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), FLOORS)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def key_sets(wkey):
    return [frozenset(int(k) for k in row if k >= 0) for row in wkey]


def obs_from_gpu(obs_t):
    """[4][L][K] tensor -> [K][L][4] numpy (float64)."""
    return obs_t.detach().cpu().numpy().transpose(2, 1, 0).astype(np.float64)


def obs_close(a, b, tau):
    """Per-env boolean: sensor observations agree within the tolerance; the
    direction (error about 2 |dc| / |c|) is compared only where both sides
    are clearly on the same side of the contact threshold tau."""
    scale = np.maximum(np.abs(b[..., 0]).max(axis=-1, keepdims=True), FORCE_FLOOR)   # [K,1]
    tol = TOL * scale
    mag_ok = np.abs(a[..., 0] - b[..., 0]) <= tol
    clear = np.abs(b[..., 0] - tau) > tol
    dir_tol = np.minimum(2.0 * tol / np.maximum(np.abs(b[..., 0]), 1e-30), 2.0)
    dir_ok = np.all(np.abs(a[..., 1:] - b[..., 1:]) <= dir_tol[..., None], axis=-1) | ~clear
    return np.all(mag_ok & dir_ok, axis=-1)
