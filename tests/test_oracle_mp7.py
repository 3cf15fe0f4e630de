"""Pins of the oracle's MP7 reconstruction (oracle/recon.py) and of the
six-ghost-layer grids it runs on.

  * the unlimited value is the degree-6 interpolant of the seven point
    values, so it is exact on polynomials of degree <= 6 and not on degree 7;
  * the limiter is MP5's: the limited value keeps a gentle monotone
    polynomial, creates no new extremum on monotone data, is equivariant
    under sign, translation and positive scaling, and the left and right
    states coincide on data symmetric about the face;
  * the scheme with MP7 and the sixth-order derivative: the right-hand side
    of a smooth entropy wave converges at sixth order (the derivative's);
    conserved sums stay constant and div B at round-off over ten steps;
  * six ghost layers change nothing for the other reconstructions: a grid
    with ng = 6 gives the ng = 5 right-hand side bit for bit.
"""
import numpy as np
import pytest

from oracle import recon
from oracle.scheme import Solver
from workloads import box


def _poly(coef, h=1.0):
    x = np.arange(-3, 4, dtype=float) * h
    return np.polyval(coef, x), np.polyval(coef, 0.5 * h)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5, 6])
def test_mp7_unlimited_exact_to_degree6(deg):
    rng = np.random.default_rng(60 + deg)
    coef = rng.normal(size=deg + 1)
    q, exact = _poly(coef)
    assert abs(recon.mp7_unlimited(*q) - exact) < 1e-12 * max(1.0, abs(exact))


def test_mp7_unlimited_not_exact_degree7():
    q, exact = _poly([1.0, 0, 0, 0, 0, 0, 0, 0])
    assert abs(recon.mp7_unlimited(*q) - exact) > 1e-3


def test_mp7_keeps_smooth_monotone_polynomials():
    for coef in ([0.3, -0.1, 1.0, 0.2], [0.0, 0.0, 2.0, -1.0], [0.01, 0.05, 0.1, 1.0, 0.0]):
        q, exact = _poly(coef, h=0.05)
        assert abs(recon.mp7(*q) - exact) < 1e-13


def test_mp7_no_new_extrema_on_monotone_data():
    rng = np.random.default_rng(65)
    q = np.sort(rng.normal(size=(20000, 7)), axis=1)
    q[::2] = q[::2, ::-1]
    out = recon.mp7(*q.T)
    lo = np.minimum(q[:, 3], q[:, 4])
    hi = np.maximum(q[:, 3], q[:, 4])
    assert np.all(out >= lo - 1e-14) and np.all(out <= hi + 1e-14)


def test_mp7_equivariance_and_step():
    rng = np.random.default_rng(66)
    q = rng.normal(size=(7, 5000))
    base = recon.mp7(*q)
    assert np.allclose(recon.mp7(*(-q)), -base, atol=1e-14)
    assert np.allclose(recon.mp7(*(q + 3.0)), base + 3.0, atol=1e-12)
    assert np.allclose(recon.mp7(*(2.5 * q)), 2.5 * base, atol=1e-13)
    # a step between cells j and j+1 stays inside the data
    out = recon.mp7(*np.array([0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0]))
    assert 0.0 <= out <= 1.0


def test_mp7_face_states_mirror_on_symmetric_data():
    row = np.array([0.1, 0.4, 0.2, 0.9, 0.3, 1.0, 1.0, 0.3, 0.9, 0.2, 0.4, 0.1])
    q = row[None, None, :]
    take = lambda a, d, lo, hi, g: a[..., lo + g:hi + g]
    left, right = recon.face_states(q, 0, 5, 6, 0, take, "mp7")
    assert left[0, 0, 0] == right[0, 0, 0]


def test_mp7_needs_six_ghost_layers():
    g, d = box.turbulent_box(8)
    with pytest.raises(ValueError):
        Solver(g, recon="mp7")


def test_rhs_operator_sixth_order_with_mp7():
    errs = []
    for n in (16, 32, 64):
        g, d = box.entropy_wave_1d(n, axis=0, ng=6)
        s = Solver(g, recon="mp7")
        s.set_face_fields(d)
        s.set_primitives(d)
        L = s.rhs()
        x = (np.arange(n) + 0.5) / n
        v = np.array([0.3, 0.2, 0.1])
        w = 1 / np.sqrt(1 - v @ v)
        exact = w * (-v[0] * 0.2 * 2 * np.pi * np.cos(2 * np.pi * x))
        errs.append(np.max(np.abs(L["D"][0, 0] - exact)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] >= 5.7, (errs, orders)


def test_conservation_and_divb_with_mp7():
    g, d = box.turbulent_box(12, ng=6)
    s = Solver(g, recon="mp7")
    s.curl_potential(d)
    s.set_primitives(d)
    d0 = s.diagnostics()
    for _ in range(10):
        s.rk_step()
    d1 = s.diagnostics()
    for k in ("sum_D", "sum_S1", "sum_S2", "sum_S3", "sum_tau", "sum_Bf1", "sum_Bf2", "sum_Bf3"):
        assert abs(d1[k] - d0[k]) < 1e-12 * max(1.0, abs(d0[k])), (k, d0[k], d1[k])
    assert d1["max_divb"] <= 1e-12


@pytest.mark.parametrize("method", ["mp5", "weno5", "plm"])
def test_six_ghost_layers_change_nothing(method):
    out = {}
    for ng in (5, 6):
        g, d = box.turbulent_box(12, ng=ng)
        s = Solver(g, recon=method)
        s.curl_potential(d)
        s.set_primitives(d)
        out[ng] = s.rhs()
    for k in out[5]:
        assert np.array_equal(out[5][k], out[6][k]), k
