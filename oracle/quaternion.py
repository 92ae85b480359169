"""Quaternion product (Sec. 2.1, eq. qprule).  Oracle module (test infrastructure only).

A quaternion f = (f0, f) is stored as the last axis of length 4; components may
be complex (the complexified quaternions of Theorems thm:dlp1form and
thm:cslp1form, where Im is taken component by component).
"""
import numpy as np


def qmul(f, g):
    """fg = (f0 g0 - f.g, f0 g + g0 f + f x g)."""
    f = np.asarray(f)
    g = np.asarray(g)
    f0, fv = f[..., 0], f[..., 1:]
    g0, gv = g[..., 0], g[..., 1:]
    s = f0 * g0 - np.sum(fv * gv, axis=-1)
    v = f0[..., None] * gv + g0[..., None] * fv + np.cross(fv, gv)
    return np.concatenate([s[..., None], v], axis=-1)


def pure(v):
    """(0, v) for a 3-vector v."""
    v = np.asarray(v)
    return np.concatenate([np.zeros(v.shape[:-1] + (1,), dtype=v.dtype), v], axis=-1)
