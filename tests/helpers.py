"""Shared test helpers: relative-error metric and solver set-up from seeded inputs."""
import numpy as np

POSITIVE = {"rho", "p", "D", "tau"}


def rel_err(a, b, name):
    """Per-zone relative error: positive fields |a-b|/|b|, signed fields
    |a-b|/max|b| over the field."""
    a = np.asarray(a)
    b = np.asarray(b)
    if name in POSITIVE:
        return np.abs(a - b) / np.abs(b)
    scale = np.max(np.abs(b))
    if scale == 0.0:
        return np.abs(a - b)
    return np.abs(a - b) / scale


def max_rel(a_dict, b_dict, names, sl=None):
    out = {}
    for n in names:
        a, b = a_dict[n], b_dict[n]
        if sl is not None:
            a, b = a[sl], b[sl]
        out[n] = float(np.max(rel_err(a, b, n)))
    return out


def interior(a, g=5):
    return a[g:-g, g:-g, g:-g]
