"""Pins of the oracle's state diagnostics (Solver.diagnostics): sums of the
conserved fields, the divergence measure and its normalised form, extrema,
the largest Lorentz factor and field strength, and the count of non-finite
primitives.  The expected values are closed forms written out here:

  * uniform flow with a uniform field (flat box): every cell holds the same
    D = rho W, S_1 = (rho h W^2 + B^2) v_1 - (v.B) B_1, so the sums are n^3
    times those; the divergence of a uniform face field is exactly zero;
  * a face field B^1 = sin(k x) on the x^1 faces of a flat box: the staggered
    sixth-order derivative and midpoint interpolation act on a Fourier mode
    by their symbols (the sum of the stencil's sines and cosines), so
    div B = s_D cos(k x_c) and B^1 = s_I sin(k x_c) at centres x_c;
  * Kerr-Schild torus grid with u^2 only: W = sqrt(1 + gamma_22 (u^2)^2).
"""
import math

import numpy as np

from oracle.scheme import Solver
from workloads.grid import box, torus_grid
from workloads import metric as wmetric

GAM = 4.0 / 3.0


def _uniform(n, rho, v1, p, b):
    g = box(n)
    s = Solver(g)
    w = 1.0 / math.sqrt(1.0 - v1 * v1)
    sh = (n, n, n)
    data = {"rho": np.full(sh, rho), "u1": np.full(sh, w * v1), "u2": np.zeros(sh),
            "u3": np.zeros(sh), "p": np.full(sh, p)}
    gs = g.shape
    data.update({"B1f": np.full(gs, b[0]), "B2f": np.full(gs, b[1]), "B3f": np.full(gs, b[2])})
    s.set_face_fields(data)
    s.set_primitives(data)
    return g, s, w


def test_uniform_state_sums_extrema_and_zero_divergence():
    n, rho, v1, p, b = 6, 1.3, 0.6, 0.2, (0.3, 0.4, 0.0)
    g, s, w = _uniform(n, rho, v1, p, b)
    out = s.diagnostics()
    h = 1.0 + GAM / (GAM - 1.0) * p / rho
    y = rho * h * w * w
    b2 = b[0] ** 2 + b[1] ** 2
    vb = v1 * b[0]
    e2 = b2 * v1 * v1 - vb * vb
    D = rho * w
    S1 = (y + b2) * v1 - vb * b[0]
    S2 = -vb * b[1]
    tau = y - p + 0.5 * (b2 + e2) - D
    N = n ** 3
    for key, want in (("sum_D", N * D), ("sum_S1", N * S1), ("sum_S2", N * S2), ("sum_S3", 0.0),
                      ("sum_tau", N * tau), ("sum_Bf1", N * b[0]), ("sum_Bf2", N * b[1]),
                      ("sum_Bf3", 0.0)):
        assert abs(out[key] - want) <= 1e-12 * max(abs(want), 1.0), (key, out[key], want)
    assert out["max_divb"] == 0.0 and out["max_divb_norm"] == 0.0
    assert abs(out["w_max"] - 1.25) < 1e-14          # v = 0.6: W = 5/4
    assert abs(out["b_max"] - 0.5) < 1e-14           # |(0.3, 0.4, 0)| = 1/2
    assert out["rho_min"] == out["rho_max"] and abs(out["rho_min"] - rho) < 1e-13
    assert abs(out["p_min"] - p) < 1e-12 and abs(out["p_max"] - p) < 1e-12
    assert out["n_nonfinite"] == 0


def _symbols(kh, order=6):
    """Symbols of the staggered derivative (times h) and midpoint interpolation
    on exp(i k x), from the stencil weights of each order."""
    if order == 6:
        dw = ((75.0 / 64.0, 0.5), (-25.0 / 384.0, 1.5), (3.0 / 640.0, 2.5))
        iw = ((150.0 / 256.0, 0.5), (-25.0 / 256.0, 1.5), (3.0 / 256.0, 2.5))
    else:
        dw = ((27.0 / 24.0, 0.5), (-1.0 / 24.0, 1.5))
        iw = ((9.0 / 16.0, 0.5), (-1.0 / 16.0, 1.5))
    sd = sum(c * 2.0 * math.sin(o * kh) for c, o in dw)
    si = sum(c * 2.0 * math.cos(o * kh) for c, o in iw)
    return sd, si


def test_planted_divergence_and_normalised_measure():
    """B^1 = sin(2 pi m x) on the x^1 faces of a flat box (B^2 = B^3 = 0): the
    divergence is that of one Fourier mode, read off at the cell centres."""
    n, mode = 16, 3
    g = box(n)
    s = Solver(g)
    k = 2.0 * math.pi * mode
    xf = np.array(g.faces(0))
    xc = np.array(g.centres(0))[g.ng:-g.ng]
    bf1 = np.broadcast_to(np.sin(k * xf)[None, None, :], g.shape).copy()
    s.set_face_fields({"B1f": bf1, "B2f": np.zeros(g.shape), "B3f": np.zeros(g.shape)})
    sh = (n, n, n)
    s.set_primitives({"rho": np.ones(sh), "u1": np.zeros(sh), "u2": np.zeros(sh), "u3": np.zeros(sh),
                      "p": np.full(sh, 0.1)})
    out = s.diagnostics()
    h = g.dx[0]
    sd, si = _symbols(k * h)
    div_max = abs(sd / h) * np.max(np.abs(np.cos(k * xc)))
    b_max = abs(si) * np.max(np.abs(np.sin(k * xc)))
    assert abs(out["max_divb"] / div_max - 1.0) < 1e-12, (out["max_divb"], div_max)
    assert abs(out["b_max"] / b_max - 1.0) < 1e-13
    assert abs(out["max_divb_norm"] / (div_max * h / b_max) - 1.0) < 1e-12
    # the sums see only the face field
    assert abs(out["sum_Bf1"] - n * n * np.sum(np.sin(k * xf[g.ng:-g.ng]))) < 1e-11
    # a planted mistake in the derivative's weights or its face indices would
    # move the measure far from this value: the fourth-order symbol differs
    sd4, _ = _symbols(k * h, 4)
    assert abs(sd4 / sd - 1.0) > 1e-3


def test_lorentz_factor_with_metric_and_nonfinite_count():
    gr = torus_grid(8, 6, 4)
    tab = wmetric.kerr_schild_tables(gr)
    s = Solver(gr, tab)
    shp = (4, 6, 8)
    rng = np.random.default_rng(21)
    u2 = rng.uniform(-0.3, 0.3, shp)
    vals = {"rho": rng.uniform(0.5, 2.0, shp), "p": rng.uniform(0.05, 0.2, shp),
            "u1": np.zeros(shp), "u2": u2, "u3": np.zeros(shp),
            "B1": np.zeros(shp), "B2": np.zeros(shp), "B3": np.zeros(shp)}
    for k, v in vals.items():
        s.set_interior(s.P[k], v)
    for f in ("Bf1", "Bf2", "Bf3"):
        s.U[f] = np.zeros(gr.shape)
    for f in ("D", "S1", "S2", "S3", "tau"):
        s.U[f] = np.zeros(gr.shape)
    g = gr.ng
    g22 = wmetric.unpack(tab)[0]["C"]["g22"][g:-g, g:-g][None]
    w = np.sqrt(1.0 + g22 * u2 * u2)
    out = s.diagnostics()
    assert abs(out["w_max"] / np.max(w) - 1.0) < 1e-14
    assert out["b_max"] == 0.0 and out["max_divb_norm"] == 0.0
    # non-finite primitives are counted; extrema skip them
    rho_ok = vals["rho"].copy()
    s.P["rho"][g + 1, g + 2, g + 3] = np.nan
    s.P["p"][g + 0, g + 1, g + 2] = np.inf
    s.P["u3"][g + 2, g + 2, g + 2] = np.nan
    rho_ok[1, 2, 3] = np.nan
    out = s.diagnostics()
    assert out["n_nonfinite"] == 3
    assert out["rho_min"] == np.nanmin(rho_ok) and out["rho_max"] == np.nanmax(rho_ok)
