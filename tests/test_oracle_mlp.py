"""Pins of the oracle's learned-guess reference: gradients against central
finite differences, features/targets against their definitions on closed-form
states, and the guess reproducing y = rho h W^2 when the network is exact."""
import numpy as np

from oracle import mlp
from workloads.mlp_data import sample_prims, init_weights

GAM = 4.0 / 3.0


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = init_weights()
    x = rng.normal(size=(32, 8))
    y = rng.normal(size=(32, 5))
    loss, grads = mlp.loss_and_grads(params, x, y)
    h = 1e-6
    for li in range(4):
        w, b = params[li]
        for _ in range(6):
            i, j = rng.integers(w.shape[0]), rng.integers(w.shape[1])
            wp = [(a.copy(), c.copy()) for a, c in params]
            wm = [(a.copy(), c.copy()) for a, c in params]
            wp[li][0][i, j] += h
            wm[li][0][i, j] -= h
            fd = (mlp.loss_and_grads(wp, x, y)[0] - mlp.loss_and_grads(wm, x, y)[0]) / (2 * h)
            assert abs(fd - grads[li][0][i, j]) <= 1e-6 * max(1.0, abs(fd)), (li, fd, grads[li][0][i, j])
        i = rng.integers(b.shape[0])
        wp = [(a.copy(), c.copy()) for a, c in params]
        wm = [(a.copy(), c.copy()) for a, c in params]
        wp[li][1][i] += h
        wm[li][1][i] -= h
        fd = (mlp.loss_and_grads(wp, x, y)[0] - mlp.loss_and_grads(wm, x, y)[0]) / (2 * h)
        assert abs(fd - grads[li][1][i]) <= 1e-6 * max(1.0, abs(fd))


def test_features_targets_closed_form():
    prims = np.zeros((1, 8))
    prims[0, 0], prims[0, 4] = 2.0, 0.5          # at rest, no field
    f, t = mlp.features_targets(prims, GAM)
    tau = 0.5 / (GAM - 1)                          # D = rho
    assert np.isclose(f[0, 0], np.log10(2.0))
    assert np.isclose(f[0, 1], np.log10(tau / 2.0))
    assert np.allclose(f[0, 2:], 0.0)
    # y = rho h = rho + Gamma/(Gamma-1) p, U = rho + p/(Gamma-1)
    y, U = 2.0 + 4.0 * 0.5, 2.0 + 3.0 * 0.5
    assert np.isclose(t[0, 0], np.log10(y / U)) and np.isclose(t[0, 1], np.log10(0.25))


def test_exact_targets_give_exact_guess():
    prims = sample_prims(1000, seed=3)
    f, t = mlp.features_targets(prims, GAM)
    mean, std = mlp.standardise_stats(t)
    out = (t - mean) / std
    from oracle.physics import state
    m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0}
    for i in range(3):
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
            m["gu%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
    st = state(prims[:, 0], tuple(prims[:, 1 + i] for i in range(3)), prims[:, 4],
               tuple(prims[:, 5 + i] for i in range(3)), m, GAM)
    y0 = mlp.guess_y0(out, mean, std, st["tau"] + st["D"])
    assert np.allclose(y0, st["y"], rtol=1e-10)


def test_sampler_ranges_and_beta():
    prims = sample_prims(20000)
    rho, p = prims[:, 0], prims[:, 4]
    assert rho.min() >= 1e-6 and rho.max() <= 10
    th = p / rho
    assert th.min() >= 1e-4 * (1 - 1e-12) and th.max() <= 10 * (1 + 1e-12)
    w = np.sqrt(1 + np.sum(prims[:, 1:4] ** 2, axis=1))
    assert w.max() <= 10 * (1 + 1e-9)
    v = prims[:, 1:4] / w[:, None]
    b = prims[:, 5:8]
    bsq = np.sum(b * b, axis=1) / w ** 2 + np.sum(v * b, axis=1) ** 2
    beta = 2 * p / bsq
    assert beta.min() >= 1e-2 * (1 - 1e-9) and beta.max() <= 1e3 * (1 + 1e-9)
