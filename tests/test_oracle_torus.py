"""Oracle pins in curved spacetime: the unmagnetised constant-l torus in
Kerr-Schild is an exact stationary solution, so the discrete right-hand side
inside the torus must shrink with resolution (the metric sources balance
the flux divergence)."""
import numpy as np
import pytest

from oracle.scheme import Solver
from workloads.torus import torus


def _torus_residual(n1, n2, n3):
    g, d, tab = torus(n1, n2, n3, noise=0.0, beta=np.inf)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    L = s.rhs()
    sg = s.centre_metric()["sqrtg"]
    x1 = g.x0[0] + (np.arange(n1) + 0.5) * g.dx[0]
    th = g.x0[1] + (np.arange(n2) + 0.5) * g.dx[1]
    r = np.exp(x1)
    # deep inside the torus: 8 <= r <= 12, |theta - pi/2| <= 0.2
    mi = (r >= 8.0) & (r <= 12.0)
    mj = np.abs(th - np.pi / 2) <= 0.2
    P = s.interior(s.P["rho"])
    out = {}
    for k in ("S1", "S2", "tau"):
        v = (L[k] / sg)[:, mj][:, :, mi]
        out[k] = float(np.max(np.abs(v)))
    return out, float(P[:, mj][:, :, mi].min())


def test_unmagnetised_torus_equilibrium_converges():
    r1, rho1 = _torus_residual(48, 48, 4)
    r2, rho2 = _torus_residual(96, 96, 4)
    assert rho1 > 0.1 and rho2 > 0.1
    for k in ("S1", "S2"):
        order = np.log2(r1[k] / r2[k])
        assert order >= 4.5, (k, r1, r2, order)


def test_torus_no_field_without_potential():
    g, d, tab = torus(16, 12, 4, noise=0.0, beta=np.inf)
    assert np.all(d["A3"] == 0.0)


def test_torus_initial_data_sane():
    g, d, tab = torus(32, 16, 8)
    assert np.all(d["rho"] > 0) and np.all(d["p"] > 0)
    assert abs(g.meta["ell"] - 3.6307) < 1e-3
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    assert s.diagnostics()["max_divb"] < 1e-12 * np.max(np.abs(s.interior(s.U["Bf1"]))) / g.dx[0] + 1e-12
