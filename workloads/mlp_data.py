"""Seeded primitive samples for training the learned Newton guess.

Log-uniform rho in [1e-6, 10], p/rho in [1e-4, 10], Lorentz factor W in
[1, 10], plasma beta = 2 p / b^2 in [1e-2, 1e3]; independent isotropic
directions of the velocity and of the field; flat local frame.  Returns
float64 arrays (n, 8): rho, u^1, u^2, u^3, p, B^1, B^2, B^3 with u = W v.
The field magnitude follows from beta through b^2 = B^2/W^2 + (v.B)^2.
Also the initial network weights (seeded, scaled uniform per layer).
"""
import numpy as np

SEED_DATA = 1810
SEED_INIT = 1811
WIDTHS = (8, 64, 64, 64, 5)


def sample_prims(n, seed=SEED_DATA):
    rng = np.random.default_rng(seed)
    rho = 10.0 ** rng.uniform(-6.0, 1.0, n)
    theta = 10.0 ** rng.uniform(-4.0, 1.0, n)
    w = 10.0 ** rng.uniform(0.0, 1.0, n)
    beta = 10.0 ** rng.uniform(-2.0, 3.0, n)
    dv = rng.normal(size=(n, 3))
    dv /= np.linalg.norm(dv, axis=1, keepdims=True)
    db = rng.normal(size=(n, 3))
    db /= np.linalg.norm(db, axis=1, keepdims=True)
    p = theta * rho
    v = np.sqrt(1.0 - 1.0 / (w * w))
    vb = v * np.sum(dv * db, axis=1)
    bsq = 2.0 * p / beta
    bmag = np.sqrt(bsq / (1.0 / (w * w) + vb * vb))
    out = np.empty((n, 8))
    out[:, 0] = rho
    out[:, 1:4] = (w * v)[:, None] * dv
    out[:, 4] = p
    out[:, 5:8] = bmag[:, None] * db
    return out


def init_weights(seed=SEED_INIT):
    """Per layer: W (out x in) uniform in +-sqrt(6/(in+out)), b = 0."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(WIDTHS[:-1], WIDTHS[1:]):
        lim = np.sqrt(6.0 / (a + b))
        params.append((rng.uniform(-lim, lim, size=(b, a)), np.zeros(b)))
    return params
