"""Pins of the oracle's finite-difference operators and MP5 reconstruction.

D_d must be exact on polynomials of degree <= 6 (its truncation error is
O(Delta^6) times the 7th derivative) and I_d on degree <= 5; the unlimited
MP5 interpolant is exact on degree <= 4.  The limiter is pinned by the
properties that define it: no new extrema on monotone data, equivariance
under sign, translation and positive scaling, and continuity.
"""
import numpy as np
import pytest

from oracle import fd, mp5

G = 5


def _poly_faces(coef, n, dx, face=True):
    """Polynomial sampled at faces (m + 1) dx or centres (m + 1/2) dx."""
    m = np.arange(-G, n + G)
    x = (m + (1.0 if face else 0.5)) * dx
    return np.polyval(coef, x), m


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5, 6])
def test_deriv_exact_on_polynomials(deg):
    rng = np.random.default_rng(deg)
    coef = rng.normal(size=deg + 1)
    n, dx = 12, 0.1
    f, m = _poly_faces(coef, n, dx)
    a = np.broadcast_to(f, (1, 1, f.size)).copy()
    d = fd.deriv(a, 0, 0, n, dx, G)[0, 0]
    xc = (np.arange(n) + 0.5) * dx
    exact = np.polyval(np.polyder(coef), xc)
    assert np.max(np.abs(d - exact)) <= 1e-11 * max(1.0, np.abs(exact).max())


def test_deriv_not_exact_degree7():
    coef = np.zeros(8); coef[0] = 1.0
    n, dx = 12, 0.1
    f, _ = _poly_faces(coef, n, dx)
    a = f[None, None, :]
    d = fd.deriv(a, 0, 0, n, dx, G)[0, 0]
    xc = (np.arange(n) + 0.5) * dx
    assert np.max(np.abs(d - 7 * xc ** 6)) > 1e-9


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5])
def test_interp_exact_on_polynomials(deg):
    rng = np.random.default_rng(10 + deg)
    coef = rng.normal(size=deg + 1)
    n, dx = 12, 0.1
    f, _ = _poly_faces(coef, n, dx)
    v = fd.interp(f[None, None, :], 0, 0, n, G)[0, 0]
    exact = np.polyval(coef, (np.arange(n) + 0.5) * dx)
    assert np.max(np.abs(v - exact)) <= 1e-12 * max(1.0, np.abs(exact).max())


def test_deriv_telescopes_on_periodic_data():
    rng = np.random.default_rng(3)
    n = 16
    f = rng.normal(size=n)
    a = np.pad(f, G, mode="wrap")[None, None, :]
    d = fd.deriv(a, 0, 0, n, 1.0, G)
    assert abs(d.sum()) < 1e-13


def test_deriv_along_each_axis():
    rng = np.random.default_rng(4)
    coef = rng.normal(size=4)
    n, dx = 8, 0.2
    f, _ = _poly_faces(coef, n, dx)
    for d, shp in ((0, (1, 1, -1)), (1, (1, -1, 1)), (2, (-1, 1, 1))):
        a = f.reshape(shp)
        r = fd.deriv(a, d, 0, n, dx, G).ravel()
        exact = np.polyval(np.polyder(coef), (np.arange(n) + 0.5) * dx)
        assert np.allclose(r, exact, rtol=0, atol=1e-11)


# ---------------------------------------------------------------- MP5
@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_unlimited_interpolant_exact(deg):
    rng = np.random.default_rng(20 + deg)
    coef = rng.normal(size=deg + 1)
    x = np.arange(-2, 3, dtype=float)          # cells j-2..j+2 at integer points
    q = np.polyval(coef, x)
    got = mp5.unlimited(*q)
    assert abs(got - np.polyval(coef, 0.5)) < 1e-13


def test_unlimited_not_exact_degree5():
    x = np.arange(-2, 3, dtype=float)
    q = x ** 5
    assert abs(mp5.unlimited(*q) - 0.5 ** 5) > 1e-3


def test_mp5_keeps_smooth_monotone_polynomials():
    # gentle monotone cubic: the limiter must accept the interpolant
    x = np.arange(-2, 3, dtype=float) * 0.05
    for coef in ([0.3, -0.1, 1.0, 0.2], [0.0, 0.0, 2.0, -1.0], [0.0, 0.1, 1.0, 0.0]):
        q = np.polyval(coef, x)
        assert abs(mp5.mp5(*q) - np.polyval(coef, 0.025)) < 1e-13


def test_mp5_no_new_extrema_on_monotone_data():
    rng = np.random.default_rng(5)
    q = np.sort(rng.normal(size=(20000, 5)), axis=1)
    q[::2] = q[::2, ::-1]
    out = mp5.mp5(*q.T)
    lo = np.minimum(q[:, 2], q[:, 3])
    hi = np.maximum(q[:, 2], q[:, 3])
    assert np.all(out >= lo - 1e-14) and np.all(out <= hi + 1e-14)


def test_mp5_step_data_bounded():
    # discontinuity between j and j+1
    q = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    out = mp5.mp5(*q)
    assert 0.0 <= out <= 1.0
    q = np.array([0.0, 0.0, 1.0, 1.0, 1.0])
    assert mp5.mp5(*q) == 1.0


def test_mp5_equivariance():
    rng = np.random.default_rng(6)
    q = rng.normal(size=(5, 5000))
    base = mp5.mp5(*q)
    assert np.allclose(mp5.mp5(*(-q)), -base, atol=1e-14)
    assert np.allclose(mp5.mp5(*(q + 3.0)), base + 3.0, atol=1e-12)
    assert np.allclose(mp5.mp5(*(2.5 * q)), 2.5 * base, atol=1e-13)


def test_mp5_continuity():
    rng = np.random.default_rng(7)
    q = rng.normal(size=(5, 20000))
    eps = 1e-9
    dq = rng.uniform(-1, 1, size=q.shape) * eps
    a = mp5.mp5(*q)
    b = mp5.mp5(*(q + dq))
    # Lipschitz: a small input change gives a change of the same order
    assert np.max(np.abs(a - b)) < 50 * eps


def test_mp5_mirror_states_on_symmetric_data():
    # symmetric data about a face: left and right states coincide
    q = np.array([0.3, 0.7, 1.0, 1.0, 0.7, 0.3])
    left = mp5.mp5(q[0], q[1], q[2], q[3], q[4])
    right = mp5.mp5(q[5], q[4], q[3], q[2], q[1])
    assert left == right


# ---------------------------------------------------------------- fourth-order D and I
@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_deriv4_exact_on_polynomials(deg):
    rng = np.random.default_rng(60 + deg)
    coef = rng.normal(size=deg + 1)
    n, dx = 12, 0.1
    f, _ = _poly_faces(coef, n, dx)
    d = fd.deriv(f[None, None, :], 0, 0, n, dx, G, order=4)[0, 0]
    exact = np.polyval(np.polyder(coef), (np.arange(n) + 0.5) * dx)
    assert np.max(np.abs(d - exact)) <= 1e-11 * max(1.0, np.abs(exact).max())


def test_deriv4_not_exact_degree5_and_differs_from_deriv6():
    coef = np.zeros(6); coef[0] = 1.0
    n, dx = 12, 0.1
    f, _ = _poly_faces(coef, n, dx)
    d4 = fd.deriv(f[None, None, :], 0, 0, n, dx, G, order=4)[0, 0]
    d6 = fd.deriv(f[None, None, :], 0, 0, n, dx, G)[0, 0]
    xc = (np.arange(n) + 0.5) * dx
    assert np.max(np.abs(d4 - 5 * xc ** 4)) > 1e-6
    assert np.max(np.abs(d6 - 5 * xc ** 4)) < 1e-11


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_interp4_exact_on_polynomials(deg):
    rng = np.random.default_rng(70 + deg)
    coef = rng.normal(size=deg + 1)
    n, dx = 12, 0.1
    f, _ = _poly_faces(coef, n, dx)
    v = fd.interp(f[None, None, :], 0, 0, n, G, order=4)[0, 0]
    exact = np.polyval(coef, (np.arange(n) + 0.5) * dx)
    assert np.max(np.abs(v - exact)) <= 1e-12 * max(1.0, np.abs(exact).max())


def test_interp4_not_exact_degree4():
    n, dx = 12, 0.1
    f, _ = _poly_faces([1.0, 0, 0, 0, 0], n, dx)
    v = fd.interp(f[None, None, :], 0, 0, n, G, order=4)[0, 0]
    assert np.max(np.abs(v - ((np.arange(n) + 0.5) * dx) ** 4)) > 1e-7


def test_deriv4_telescopes_and_converges_at_fourth_order():
    rng = np.random.default_rng(12)
    a = np.pad(rng.normal(size=16), G, mode="wrap")[None, None, :]
    assert abs(fd.deriv(a, 0, 0, 16, 1.0, G, order=4).sum()) < 1e-13
    errs = []
    for n in (16, 32, 64):
        dx = 1.0 / n
        xf = (np.arange(-G, n + G) + 1.0) * dx
        d = fd.deriv(np.sin(2 * np.pi * xf)[None, None, :], 0, 0, n, dx, G, order=4)[0, 0]
        errs.append(np.max(np.abs(d - 2 * np.pi * np.cos(2 * np.pi * (np.arange(n) + 0.5) * dx))))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.9 and max(orders) < 4.1, orders
