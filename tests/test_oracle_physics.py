"""Pins of the oracle's pointwise algebra, HLL flux, speeds and inversion.

The 3+1 conserved variables and fluxes are checked against the covariant
stress-energy tensor T^{mu nu} = (rho h + b^2) u^mu u^nu + (p + b^2/2) g^{mu nu}
- b^mu b^nu built from the full 4-metric, an independent route to the same
quantities: D = rho alpha u^0, S_i = alpha T^0_i, U = alpha^2 T^00,
F[D] = alpha sqrt(gamma) rho u^d, F[S_i] = alpha sqrt(gamma) T^d_i,
F[U] = sqrt(gamma) alpha^2 T^{0d}.
"""
import numpy as np
import pytest

from oracle import physics, hll, c2p

GAM = 4.0 / 3.0


def random_metric(rng, n):
    """Random lapse, shift and SPD spatial metric (as location dict)."""
    a = rng.normal(size=(n, 3, 3)) * 0.3
    g = np.einsum("nij,nkj->nik", a, a) + np.eye(3) * rng.uniform(0.5, 2.0, size=(n, 1, 1))
    gi = np.linalg.inv(g)
    m = {"alpha": rng.uniform(0.5, 1.5, n), "sqrtg": np.sqrt(np.linalg.det(g))}
    beta = rng.normal(size=(n, 3)) * 0.2
    for i in range(3):
        m["beta%d" % (i + 1)] = beta[:, i]
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = g[:, i, j]
            m["gu%d%d" % (i + 1, j + 1)] = gi[:, i, j]
    return m, g, gi, beta


def random_prims(rng, n, vmax=0.8, bmax=1.0):
    rho = rng.uniform(0.1, 2.0, n)
    p = rng.uniform(0.01, 1.0, n)
    u = tuple(rng.normal(size=n) * vmax for _ in range(3))
    b = tuple(rng.normal(size=n) * bmax for _ in range(3))
    return rho, u, p, b


def covariant(rho, u, p, b, m, g3, gi3, beta):
    n = rho.size
    al = m["alpha"]
    # 4-metric
    bl = np.einsum("nij,nj->ni", g3, beta)
    g4 = np.zeros((n, 4, 4))
    g4[:, 0, 0] = -al ** 2 + np.einsum("ni,ni->n", bl, beta)
    g4[:, 0, 1:] = bl
    g4[:, 1:, 0] = bl
    g4[:, 1:, 1:] = g3
    gi4 = np.linalg.inv(g4)
    U3 = np.stack(u, axis=1)
    B3 = np.stack(b, axis=1)
    ul = np.einsum("nij,nj->ni", g3, U3)
    W = np.sqrt(1 + np.einsum("ni,ni->n", ul, U3))
    v = U3 / W[:, None]
    u4 = np.zeros((n, 4))
    u4[:, 0] = W / al
    u4[:, 1:] = U3 - W[:, None] * beta / al[:, None]
    bv = np.einsum("ni,ni->n", np.einsum("nij,nj->ni", g3, v), B3)
    b4 = np.zeros((n, 4))
    b4[:, 0] = W * bv / al
    b4[:, 1:] = B3 / W[:, None] + al[:, None] * b4[:, :1] * (v - beta / al[:, None])
    b4l = np.einsum("nij,nj->ni", g4, b4)
    bsq = np.einsum("ni,ni->n", b4, b4l)
    h = 1 + GAM / (GAM - 1) * p / rho
    T = ((rho * h + bsq)[:, None, None] * np.einsum("ni,nj->nij", u4, u4)
         + (p + 0.5 * bsq)[:, None, None] * gi4 - np.einsum("ni,nj->nij", b4, b4))
    Tmix = np.einsum("nij,njk->nik", T, g4)     # T^mu_nu
    return u4, T, Tmix, bsq


def test_conserved_and_fluxes_match_covariant_form():
    rng = np.random.default_rng(11)
    n = 500
    m, g3, gi3, beta = random_metric(rng, n)
    rho, u, p, b = random_prims(rng, n)
    st = physics.state(rho, u, p, b, m, GAM)
    u4, T, Tmix, bsq = covariant(rho, u, p, b, m, g3, gi3, beta)
    al, sg = m["alpha"], m["sqrtg"]
    assert np.allclose(st["D"], rho * al * u4[:, 0], rtol=1e-12)
    for i in range(3):
        assert np.allclose(st["S"][i], al * Tmix[:, 0, i + 1], rtol=1e-10, atol=1e-12)
    assert np.allclose(st["Utot"], al ** 2 * T[:, 0, 0], rtol=1e-10)
    assert np.allclose(st["B2"] / st["W"] ** 2 + st["vB"] ** 2, bsq, rtol=1e-10)
    for d in range(3):
        f = physics.flux(st, m, d)
        assert np.allclose(f[0], al * sg * rho * u4[:, d + 1], rtol=1e-10, atol=1e-12)
        for i in range(3):
            assert np.allclose(f[1 + i], al * sg * Tmix[:, d + 1, i + 1], rtol=1e-9, atol=1e-11)
        fu = f[4] + f[0]
        assert np.allclose(fu, sg * al ** 2 * T[:, 0, d + 1], rtol=1e-9, atol=1e-11)


def test_flat_static_closed_forms():
    m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0,
         "g11": 1.0, "g12": 0.0, "g13": 0.0, "g22": 1.0, "g23": 0.0, "g33": 1.0,
         "gu11": 1.0, "gu12": 0.0, "gu13": 0.0, "gu22": 1.0, "gu23": 0.0, "gu33": 1.0}
    rho, p = 1.3, 0.4
    z = (0.0, 0.0, 0.0)
    st = physics.state(rho, z, p, z, m, GAM)
    assert np.isclose(st["tau"], p / (GAM - 1))
    b = (0.2, -0.1, 0.3)
    st = physics.state(rho, z, p, b, m, GAM)
    assert np.isclose(st["tau"], p / (GAM - 1) + 0.5 * (0.04 + 0.01 + 0.09))
    f = physics.flux(st, m, 0)
    # static magnetised state: momentum flux = total pressure - B_x B_x
    assert np.isclose(f[1], p + 0.5 * 0.14 - 0.04)
    assert np.isclose(f[2], 0.02) and np.isclose(f[3], -0.06)


def test_speeds_reduce_to_velocity_addition():
    m = {"alpha": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0, "g11": 1.0, "g12": 0.0,
         "g13": 0.0, "g22": 1.0, "g23": 0.0, "g33": 1.0, "gu11": 1.0, "gu12": 0.0,
         "gu13": 0.0, "gu22": 1.0, "gu23": 0.0, "gu33": 1.0, "sqrtg": 1.0}
    rng = np.random.default_rng(3)
    for _ in range(50):
        v = rng.uniform(-0.9, 0.9)
        rho, p = rng.uniform(0.1, 2), rng.uniform(0.01, 2)
        w = 1 / np.sqrt(1 - v * v)
        st = physics.state(rho, (w * v, 0.0, 0.0), p, (0.0, 0.0, 0.0), m, GAM)
        lp, lm = physics.speeds(st, m, 0, GAM)
        cs = np.sqrt(GAM * p / (rho * st["h"]))
        assert np.isclose(lp, (v + cs) / (1 + v * cs), rtol=1e-12)
        assert np.isclose(lm, (v - cs) / (1 - v * cs), rtol=1e-12)


def test_speeds_static_gr():
    rng = np.random.default_rng(5)
    m, *_ = random_metric(rng, 200)
    rho, _, p, b = random_prims(rng, 200)
    z = tuple(np.zeros(200) for _ in range(3))
    st = physics.state(rho, z, p, b, m, GAM)
    rhoh = rho * st["h"]
    cs2 = GAM * p / rhoh
    va2 = st["B2"] / (rhoh + st["B2"])
    a = np.sqrt(cs2 + va2 - cs2 * va2)
    for d in range(3):
        lp, lm = physics.speeds(st, m, d, GAM)
        gdd = m["gu%d%d" % (d + 1, d + 1)]
        bd = m["beta%d" % (d + 1)]
        assert np.allclose(lp, m["alpha"] * a * np.sqrt(gdd) - bd, rtol=1e-12)
        assert np.allclose(lm, -m["alpha"] * a * np.sqrt(gdd) - bd, rtol=1e-12)


def test_hll_consistency_and_upwinding():
    rng = np.random.default_rng(2)
    f = rng.normal(size=100)
    u = rng.normal(size=100)
    ap, am = rng.uniform(0.1, 1, 100), rng.uniform(0.1, 1, 100)
    assert np.allclose(hll.hll_flux(f, f, u, u, ap, am), f, rtol=1e-14)
    fl, fr, ur = rng.normal(size=100), rng.normal(size=100), rng.normal(size=100)
    assert np.allclose(hll.hll_flux(fl, fr, u, ur, ap, 0.0 * am), fl, rtol=1e-14)
    assert np.allclose(hll.hll_flux(fl, fr, u, ur, 0.0 * ap, am), fr, rtol=1e-14)
    ap2, am2 = hll.hll_speeds(np.array([0.5]), np.array([0.2]), np.array([0.7]), np.array([0.1]))
    assert ap2[0] == 0.7 and am2[0] == 0.0


def sample_box(rng, n):
    """Log-uniform primitive sampling box of the learned-guess training set."""
    rho = 10 ** rng.uniform(-6, 1, n)
    theta = 10 ** rng.uniform(-4, 1, n)
    p = theta * rho
    w = 10 ** rng.uniform(0, 1, n)
    beta = 10 ** rng.uniform(-2, 3, n)
    dirs = rng.normal(size=(2, n, 3))
    dirs /= np.linalg.norm(dirs, axis=2, keepdims=True)
    umag = np.sqrt(w * w - 1)
    u = tuple(umag * dirs[0, :, i] for i in range(3))
    return rho, u, p, beta, dirs[1], w


def test_round_trip_sampling_box():
    rng = np.random.default_rng(7)
    n = 20000
    rho, u, p, beta, bdir, w = sample_box(rng, n)
    m = {"alpha": np.ones(n), "sqrtg": np.ones(n)}
    for i in range(3):
        m["beta%d" % (i + 1)] = np.zeros(n)
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = np.full(n, 1.0 if i == j else 0.0)
            m["gu%d%d" % (i + 1, j + 1)] = np.full(n, 1.0 if i == j else 0.0)
    # b^2 from beta = 2 p / b^2, field along bdir: solve |B| from b^2 = B^2/W^2 + (vB)^2
    z = tuple(np.zeros(n) for _ in range(3))
    st0 = physics.state(rho, u, p, tuple(bdir[:, i] for i in range(3)), m, GAM)
    bb_unit = st0["B2"] / st0["W"] ** 2 + st0["vB"] ** 2
    scale = np.sqrt(2 * p / beta / bb_unit)
    b = tuple(scale * bdir[:, i] for i in range(3))
    st = physics.state(rho, u, p, b, m, GAM)
    D, S, tau = st["D"], st["S"], st["tau"]
    res = c2p.newton(D, S, tau, b, m, GAM, GAM * (tau + D))
    assert res["ok"].mean() > 0.999
    ok = res["ok"]
    # backward error: cons(prim(U)) = U
    st2 = physics.state(res["rho"], res["u"], res["p"], b, m, GAM)
    utot = tau + D
    assert np.max(np.abs(st2["D"] - D)[ok] / D[ok]) < 1e-12
    assert np.max(np.abs(st2["tau"] + st2["D"] - utot)[ok] / utot[ok]) < 1e-12
    smag = np.sqrt(S[0] ** 2 + S[1] ** 2 + S[2] ** 2) + 1e-300
    for i in range(3):
        assert np.max(np.abs(st2["S"][i] - S[i])[ok] / (smag + utot)[ok]) < 1e-12
    # forward error on rho is well conditioned
    assert np.max(np.abs(res["rho"] / rho - 1)[ok]) < 1e-9


def test_inversion_closed_forms():
    n = 10
    m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0}
    for i in range(3):
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
            m["gu%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
    D = np.linspace(0.5, 2.0, n)
    tau = np.linspace(0.1, 3.0, n)
    z = tuple(np.zeros(n) for _ in range(3))
    r = c2p.newton(D, z, tau, z, m, GAM, GAM * (tau + D))
    assert np.allclose(r["p"], (GAM - 1) * tau, rtol=1e-13)
    assert np.allclose(r["rho"], D, rtol=1e-14)
    b = (np.full(n, 0.3), np.full(n, -0.2), np.full(n, 0.1))
    tau_b = tau + 0.5 * 0.14
    r = c2p.newton(D, z, tau_b, b, m, GAM, GAM * (tau_b + D))
    assert np.allclose(r["p"], (GAM - 1) * (tau_b - 0.07), rtol=1e-12)


def test_inversion_flags_unphysical_states():
    m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0}
    for i in range(3):
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
            m["gu%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
    D = np.array([1.0, -1.0, 1.0, 1.0])
    tau = np.array([-2.0, 1.0, 1.0, np.nan])
    S = (np.array([0.0, 0.0, 50.0, 0.0]), np.zeros(4), np.zeros(4))
    z = tuple(np.zeros(4) for _ in range(3))
    r = c2p.newton(D, S, tau, z, m, GAM, GAM * (tau + D))
    assert not r["ok"].any()


def test_newton_warm_start_converges_fast():
    rng = np.random.default_rng(9)
    n = 5000
    rho, u, p, beta, bdir, w = sample_box(rng, n)
    m = {"alpha": 1.0, "sqrtg": 1.0, "beta1": 0.0, "beta2": 0.0, "beta3": 0.0}
    for i in range(3):
        for j in range(i, 3):
            m["g%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
            m["gu%d%d" % (i + 1, j + 1)] = 1.0 if i == j else 0.0
    b = tuple(0.1 * np.sqrt(p) * bdir[:, i] for i in range(3))
    st = physics.state(rho, u, p, b, m, GAM)
    y_true = st["y"]
    r = c2p.newton(st["D"], st["S"], st["tau"], b, m, GAM, y_true * (1 + 1e-3))
    assert r["ok"].all()
    assert np.percentile(r["iters"], 99) <= 5
