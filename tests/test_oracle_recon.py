"""Pins of the oracle's alternative reconstructions (WENO5 point-value form,
PLM with the monotonized-central limiter).

WENO5: each candidate is the quadratic through its three points, so every
convex combination of them -- the reconstruction for any weights -- is exact
on polynomials of degree <= 2; with equal smoothness indicators (linear data,
or eps -> infinity) the weights are the linear ones and the value is the
degree-4 interpolant (3, -20, 90, 60, -5)/128, checked against the separately
written MP5 module; on smooth data away from critical points the error falls
at fifth order; across a step it stays within the data's range up to a small
multiple of the jump.  PLM-MC: exact on linear data, never leaves the range
of its two neighbours (no new extrema), equivariant under sign, translation
and positive scaling, second order on smooth monotone data, first order
(the cell value) at an extremum.  Both: the left and right states of a face
coincide on data symmetric about it.
"""
import numpy as np
import pytest

from oracle import recon, mp5


def _stencil_poly(coef, h=1.0):
    x = np.arange(-2, 3, dtype=float) * h
    return np.polyval(coef, x), np.polyval(coef, 0.5 * h)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_weno5_candidates_exact_on_quadratics(deg):
    rng = np.random.default_rng(40 + deg)
    coef = rng.normal(size=deg + 1)
    q, exact = _stencil_poly(coef)
    for p in recon.weno5_candidates(*q):
        assert abs(p - exact) < 1e-13


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_weno5_exact_on_quadratics_for_any_weights(deg):
    rng = np.random.default_rng(50 + deg)
    coef = rng.normal(size=deg + 1)
    q, exact = _stencil_poly(coef)
    for eps in (1e-6, 1e-30, 1.0):
        assert abs(recon.weno5(*q, eps=eps) - exact) < 1e-12


def test_weno5_candidates_not_exact_on_cubics():
    q, exact = _stencil_poly([1.0, 0.0, 0.0, 0.0])
    assert all(abs(p - exact) > 1e-3 for p in recon.weno5_candidates(*q))


def test_weno5_linear_weights_give_the_degree4_interpolant():
    rng = np.random.default_rng(8)
    q = rng.normal(size=(5, 1000))
    # eps -> infinity: alpha_k proportional to d_k (b_k / eps below rounding)
    got = recon.weno5(*q, eps=1e20)
    assert np.allclose(got, mp5.unlimited(*q), rtol=0, atol=1e-12)
    # linear data: all three indicators are equal, so the weights are linear
    s = rng.normal(size=200)
    lin = np.outer(np.arange(-2, 3, dtype=float), s)
    b = recon.weno5_indicators(*lin)
    assert np.allclose(b[0], b[1], rtol=1e-13) and np.allclose(b[1], b[2], rtol=1e-13)
    assert np.allclose(recon.weno5(*lin), 0.5 * s, rtol=0, atol=1e-13)


def test_weno5_fifth_order_on_smooth_monotone_data():
    # q = sin(x) on a monotone stretch; error at x + h/2 falls as h^5
    errs = []
    hs = [0.04, 0.02, 0.01]
    for h in hs:
        x0 = 0.3
        q = np.sin(x0 + np.arange(-2, 3) * h)
        errs.append(abs(recon.weno5(*q, eps=1e-40) - np.sin(x0 + 0.5 * h)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 4.5, orders


def test_weno5_step_nearly_bounded():
    # jumps whose indicators dwarf eps (the weights are scale dependent: a
    # jump of order sqrt(eps) is treated as smooth)
    for jump in (0.1, 1.0, 10.0):
        for q in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [0, 1, 1, 1, 1], [0, 0, 0, 0, 1]):
            v = recon.weno5(*(jump * np.array(q, float)))
            assert -1e-3 * jump <= v <= jump * (1 + 1e-3), (q, v)


def test_weno5_equivariance_sign_translation():
    rng = np.random.default_rng(9)
    q = rng.normal(size=(5, 3000))
    base = recon.weno5(*q)
    assert np.allclose(recon.weno5(*(-q)), -base, atol=1e-13)
    assert np.allclose(recon.weno5(*(q + 3.0)), base + 3.0, atol=1e-12)


def test_plm_exact_on_linear_and_bounded():
    rng = np.random.default_rng(10)
    s = rng.normal(size=500)
    c = rng.normal(size=500)
    assert np.allclose(recon.plm(c - s, c, c + s), c + 0.5 * s, rtol=0, atol=1e-14)
    q = rng.normal(size=(3, 20000))
    v = recon.plm(*q)
    lo = np.minimum(q[1], q[2])
    hi = np.maximum(q[1], q[2])
    assert np.all(v >= lo - 1e-14) and np.all(v <= hi + 1e-14)


def test_plm_extremum_gives_cell_value():
    assert recon.plm(0.0, 1.0, 0.0) == 1.0
    assert recon.plm(2.0, 1.0, 3.0) == 1.0


def test_plm_equivariance():
    rng = np.random.default_rng(11)
    q = rng.normal(size=(3, 3000))
    base = recon.plm(*q)
    assert np.allclose(recon.plm(*(-q)), -base, atol=1e-14)
    assert np.allclose(recon.plm(*(q + 3.0)), base + 3.0, atol=1e-13)
    assert np.allclose(recon.plm(*(2.5 * q)), 2.5 * base, atol=1e-13)


def test_plm_second_order_on_smooth_monotone_data():
    errs = []
    for h in (0.04, 0.02, 0.01):
        x0 = 0.3
        q = np.sin(x0 + np.arange(-1, 2) * h)
        errs.append(abs(recon.plm(*q) - np.sin(x0 + 0.5 * h)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.8 < min(orders) and max(orders) < 2.2, orders


@pytest.mark.parametrize("method", ["mp5", "weno5", "plm"])
def test_face_states_mirror_on_symmetric_data(method):
    # one row of cells symmetric about the face between cells 5 and 6
    row = np.array([0.1, 0.4, 0.2, 0.9, 0.3, 1.0, 1.0, 0.3, 0.9, 0.2, 0.4, 0.1])
    q = row[None, None, :]
    take = lambda a, d, lo, hi, g: a[..., lo + g:hi + g]
    left, right = recon.face_states(q, 0, 5, 6, 0, take, method)
    assert left[0, 0, 0] == right[0, 0, 0]


def test_unknown_method_rejected():
    q = np.zeros((1, 1, 12))
    take = lambda a, d, lo, hi, g: a[..., lo + g:hi + g]
    with pytest.raises(ValueError):
        recon.face_states(q, 0, 3, 6, 0, take, "ppm")
