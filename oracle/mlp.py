"""Learned Newton initial guess: FP64 reference (oracle).

The learned part is a training-system pattern added on top of the method (no
counterpart in the paper): an MLP 8 -> 64 -> 64 -> 64 -> 5 with tanh hidden
activations and a linear output, trained with mean-squared error on
(conserved -> primitive) pairs produced by the method's own prim -> cons map.

Features (8), in the Eulerian orthonormal frame (Cholesky gamma = L L^T:
S_hat = L^-1 S, B_hat = L^T B), from undensitised D, S_i, tau, B^i:
  [log10 D, log10(tau/D), S_hat/(tau+D) (3), B_hat/sqrt(tau+D) (3)]
Targets (5): [log10(y/U), log10(p/D), u_hat (3)] with y = rho h W^2 (the
Newton variable), U = tau + D and u_hat = L^T u.  Both are standardised with
the training-set mean and standard deviation.  Guess: y0 = U 10^t0 (the
first target is the Newton variable itself because p is ill-conditioned in
cold, magnetised states, which made a guess assembled from rho, p and u
worse than the cold start).
"""
import numpy as np

from .physics import state


def features_targets(prims, gam, m=None):
    """prims (n, 8) in a flat frame (m None) -> (features (n, 8), targets (n, 5))."""
    n = prims.shape[0]
    if m is None:
        m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0}
        for i in range(3):
            for j in range(i, 3):
                m["g%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
                m["gu%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
    rho, p = prims[:, 0], prims[:, 4]
    u = tuple(prims[:, 1 + i] for i in range(3))
    b = tuple(prims[:, 5 + i] for i in range(3))
    st = state(rho, u, p, b, m, gam)
    dd, tau = st["D"], st["tau"]
    s = np.stack(st["S"], axis=1)
    bb = np.stack(b, axis=1)
    uu = np.stack(u, axis=1)
    e = dd + tau
    f = np.empty((n, 8))
    f[:, 0] = np.log10(dd)
    f[:, 1] = np.log10(tau / dd)
    f[:, 2:5] = s / e[:, None]          # flat frame: L = identity
    f[:, 5:8] = bb / np.sqrt(e)[:, None]
    t = np.empty((n, 5))
    t[:, 0] = np.log10(st["y"] / e)
    t[:, 1] = np.log10(p / dd)
    t[:, 2:5] = uu
    return f, t


def standardise_stats(x):
    return x.mean(axis=0), x.std(axis=0)


def forward(params, x):
    """params: [(W (out, in), b (out))] x 4; x (n, 8) -> (out (n, 5), activations)."""
    acts = [x]
    h = x
    for li, (w, b) in enumerate(params):
        z = h @ w.T + b
        h = np.tanh(z) if li < len(params) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grads(params, x, y):
    """Mean squared error over samples and outputs, and its gradients."""
    out, acts = forward(params, x)
    n = x.shape[0]
    diff = out - y
    loss = float(np.mean(diff * diff))
    d = 2.0 * diff / (n * y.shape[1])
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        w, _ = params[li]
        a_prev = acts[li]
        grads[li] = (d.T @ a_prev, d.sum(axis=0))
        if li > 0:
            da = d @ w
            d = da * (1.0 - acts[li] ** 2)
    return loss, grads


def guess_y0(out, mean_t, std_t, utot):
    """Newton guess from standardised network outputs and U = tau + D."""
    t = out * std_t + mean_t
    return utot * 10.0 ** t[:, 0]
