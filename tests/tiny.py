"""Hand-made tiny scenes for closed-form checks (test helper)."""
import math

import numpy as np

from paper_2002_12160_amd.scene import HAND_STRIDE, ModelConsts


def link_row(a, b, radius, parent=-1, joint=-1, axis=(0.0, 1.0, 0.0)):
    """A capsule link from a to b (no parent, optional joint about `axis` in
    the link's rest frame)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = b - a
    length = float(np.linalg.norm(d))
    x = d / length
    # rotation taking e_x to x
    ex = np.array([1.0, 0.0, 0.0])
    c = float(np.dot(ex, x))
    ax = np.cross(ex, x)
    s = float(np.linalg.norm(ax))
    if s < 1e-15:
        q = np.array([1.0, 0, 0, 0]) if c > 0 else np.array([0.0, 0, 0, 1.0])
    else:
        ang = math.atan2(s, c)
        ax = ax / s
        q = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * ax)])
    row = np.zeros(HAND_STRIDE)
    row[0] = parent
    row[1] = joint
    row[2] = -1
    row[3:6] = axis
    row[9:12] = a
    row[12:16] = q
    row[16] = length
    row[17] = radius
    return row


def far_link():
    """One capsule link far away from everything (a hand that never touches)."""
    return link_row((10.0, 10.0, 10.0), (10.1, 10.0, 10.0), 0.008)


def single_sphere(radius, inv_inertia=(0.0, 0.0, 0.0), offset=(0.0, 0.0, 0.0)):
    sph = np.array([[[offset[0], offset[1], offset[2], radius]]], dtype=np.float64)
    return sph, np.array([1], dtype=np.int32), np.array([inv_inertia], dtype=np.float64)


def consts(**kw):
    return ModelConsts(**kw)


def state(x=(0, 0, 0), q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    return np.array([*x, *q, *v, *w], dtype=np.float64)


def params(m, mu, f=(0, 0, 0)):
    return np.array([m, mu, *f], dtype=np.float64)
