"""Scheme-level pins of the oracle: conservation, div B, convergence order,
time integrator, metric tables, flat curvilinear equilibrium, boundaries."""
import numpy as np
import pytest

from oracle import scheme, fd
from oracle.scheme import Solver, SSPRK3, rk_combine
from workloads import box
from workloads.grid import GridSpec, torus_grid, LOGSPH, BC_OUTFLOW, BC_AXIS, BC_PERIODIC
from workloads import metric as wmetric


def _box_solver(n):
    g, d = box.turbulent_box(n)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    return s


def test_ssprk3_linear_amplification():
    # dU/dt = lam U: one step must give 1 + z + z^2/2 + z^3/6
    for z in (0.3, -1.2, 0.5 + 0.7j, -0.1 - 2.0j):
        lam, dt = z, 1.0
        un = 1.0 + 0j
        u = un
        for a, b in SSPRK3:
            u = rk_combine(un, u, lam * u, a, b, dt)
        assert abs(u - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14


def test_conservation_and_divb_periodic_box():
    s = _box_solver(16)
    d0 = s.diagnostics()
    for _ in range(10):
        s.rk_step()
    d1 = s.diagnostics()
    for k in ("D", "tau"):
        assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * abs(d0["sum_" + k])
    scale = sum(np.abs(s.interior(s.U[k])).sum() for k in ("S1", "S2", "S3"))
    for k in ("S1", "S2", "S3"):
        assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * scale
    bscale = sum(np.abs(s.interior(s.U[k])).sum() for k in ("Bf1", "Bf2", "Bf3"))
    for k in ("Bf1", "Bf2", "Bf3"):
        assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * bscale
    assert d0["max_divb"] <= 1e-12
    assert d1["max_divb"] <= 1e-12
    bmax = max(np.abs(s.interior(s.P[k])).max() for k in ("B1", "B2", "B3"))
    assert d1["max_divb"] * s.grid.dx[0] / bmax <= 1e-12


def test_shaped_box_generator_equals_cubic_one():
    """The non-cubic box generator (direct sum over the modes) reproduces the
    cubic generator (inverse FFT for n >= 9) when the three sizes agree."""
    g1, d1 = box.turbulent_box(12)
    g2, d2 = box.turbulent_box_shape(12, 12, 12)
    assert g1.n == g2.n and g1.dx == g2.dx and g1.bc == g2.bc
    for k in d1:
        assert np.allclose(d1[k], d2[k], rtol=0, atol=1e-13), k


def test_conservation_and_divb_non_cubic_box():
    """On a ragged non-cubic periodic box (13 x 9 x 11) the oracle keeps the
    totals of D, S, tau and the face fields and div B at round-off."""
    g, d = box.turbulent_box_shape(13, 9, 11)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    d0 = s.diagnostics()
    for _ in range(3):
        s.rk_step()
    d1 = s.diagnostics()
    for grp in (("D",), ("tau",), ("S1", "S2", "S3"), ("Bf1", "Bf2", "Bf3")):
        scale = sum(np.abs(s.interior(s.U[k])).sum() for k in grp)
        for k in grp:
            assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * scale, k
    assert d0["max_divb"] <= 1e-12 and d1["max_divb"] <= 1e-12


def test_uniform_state_stays_uniform_and_b_unchanged():
    g, d = box.entropy_wave(8, amp=0.0)
    s = Solver(g)
    s.set_face_fields(d)
    s.set_primitives(d)
    u0 = {k: s.interior(v).copy() for k, v in s.U.items()}
    s.rk_step()
    for k in ("Bf1", "Bf2", "Bf3"):
        assert np.max(np.abs(s.interior(s.U[k]) - u0[k])) < 1e-15
    for k in ("D", "S1", "S2", "S3", "tau"):
        assert np.max(np.abs(s.interior(s.U[k]) - u0[k])) < 1e-14


def _run_wave(n, axis, t_end):
    g, d = box.entropy_wave_1d(n, axis=axis)
    s = Solver(g)
    s.set_face_fields(d)
    s.set_primitives(d)
    dt0 = 0.4 * (1.0 / 16) * (16.0 / n) ** (5.0 / 3.0)
    nsteps = int(np.ceil(t_end / dt0))
    dt = t_end / nsteps
    for _ in range(nsteps):
        s.rk_step(dt)
    _, de = box.entropy_wave_1d(n, axis=axis, t=t_end)
    return np.mean(np.abs(s.interior(s.P["rho"]) - de["rho"]))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fifth_order_convergence_entropy_wave(axis):
    errs = [_run_wave(n, axis, 0.2) for n in (16, 32, 64)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] >= 4.7, (errs, orders)


def test_rhs_operator_fifth_order():
    # || L(U_exact) - dU/dt_exact || for the 1-D entropy wave: d/dt D = -v dD/dx
    errs = []
    for n in (16, 32, 64):
        g, d = box.entropy_wave_1d(n, axis=0)
        s = Solver(g)
        s.set_face_fields(d)
        s.set_primitives(d)
        L = s.rhs()
        x = (np.arange(n) + 0.5) / n
        v = np.array([0.3, 0.2, 0.1])
        w = 1 / np.sqrt(1 - v @ v)
        drho_dt = -v[0] * 0.2 * 2 * np.pi * np.cos(2 * np.pi * x)
        exact = w * drho_dt          # dD/dt with uniform W
        errs.append(np.max(np.abs(L["D"][0, 0] - exact)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] >= 4.7, (errs, orders)


def _rhs_errors(recon, ns):
    linf, l1 = [], []
    for n in ns:
        g, d = box.entropy_wave_1d(n, axis=0)
        s = Solver(g, recon=recon)
        s.set_face_fields(d)
        s.set_primitives(d)
        L = s.rhs()
        x = (np.arange(n) + 0.5) / n
        v = np.array([0.3, 0.2, 0.1])
        w = 1 / np.sqrt(1 - v @ v)
        e = L["D"][0, 0] - w * (-v[0] * 0.2 * 2 * np.pi * np.cos(2 * np.pi * x))
        linf.append(np.max(np.abs(e)))
        l1.append(np.mean(np.abs(e)))
    order = lambda a: [np.log2(a[i] / a[i + 1]) for i in range(len(a) - 1)]
    return order(linf), order(l1)


def test_rhs_operator_order_weno5():
    # WENO5's nonlinear weights keep fifth order on the smooth wave
    linf, l1 = _rhs_errors("weno5", (16, 32, 64))
    assert linf[-1] >= 4.7 and l1[-1] >= 4.7, (linf, l1)


def test_rhs_operator_order_plm():
    # second order in L1; first order in the maximum norm, because the MC
    # limiter reduces the reconstruction to the cell value at the extrema
    linf, l1 = _rhs_errors("plm", (16, 32, 64))
    assert l1[-1] >= 1.9, l1
    assert 0.9 < linf[-1] < 1.1, linf


@pytest.mark.parametrize("recon", ["weno5", "plm"])
def test_conservation_and_divb_other_reconstructions(recon):
    g, d = box.turbulent_box(12)
    s = Solver(g, recon=recon)
    s.curl_potential(d)
    s.set_primitives(d)
    d0 = s.diagnostics()
    for _ in range(3):
        s.rk_step()
    d1 = s.diagnostics()
    for grp in (("D",), ("tau",), ("S1", "S2", "S3"), ("Bf1", "Bf2", "Bf3")):
        scale = sum(np.abs(s.interior(s.U[k])).sum() for k in grp)
        for k in grp:
            assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * scale, k
    assert d1["max_divb"] <= 1e-12


def test_rhs_operator_fourth_order_with_d4():
    """With the fourth-order D and I the RHS of the smooth wave converges at
    fourth order (MP5 is fifth order, D4 sets the rate)."""
    errs = []
    for n in (16, 32, 64):
        g, d = box.entropy_wave_1d(n, axis=0)
        s = Solver(g, deriv_order=4)
        s.set_face_fields(d)
        s.set_primitives(d)
        L = s.rhs()
        x = (np.arange(n) + 0.5) / n
        v = np.array([0.3, 0.2, 0.1])
        w = 1 / np.sqrt(1 - v @ v)
        errs.append(np.max(np.abs(L["D"][0, 0] - w * (-v[0] * 0.2 * 2 * np.pi * np.cos(2 * np.pi * x)))))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 3.8 < orders[-1] < 4.3, (errs, orders)


def test_conservation_and_divb_with_d4():
    g, d = box.turbulent_box(12)
    s = Solver(g, deriv_order=4)
    s.curl_potential(d)
    s.set_primitives(d)
    d0 = s.diagnostics()
    for _ in range(3):
        s.rk_step()
    d1 = s.diagnostics()
    for grp in (("D",), ("tau",), ("S1", "S2", "S3"), ("Bf1", "Bf2", "Bf3")):
        scale = sum(np.abs(s.interior(s.U[k])).sum() for k in grp)
        for k in grp:
            assert abs(d1["sum_" + k] - d0["sum_" + k]) <= 1e-13 * scale, k
    assert d0["max_divb"] <= 1e-12 and d1["max_divb"] <= 1e-12
    # the sixth-order divergence of the D4-built field is not zero
    s6 = Solver(g)
    s6.U = s.U
    assert s6.div_b().max() > 1e-6


def test_unknown_reconstruction_rejected():
    g, _ = box.turbulent_box(8)
    with pytest.raises(ValueError):
        Solver(g, recon="ppm")


# ------------------------------------------------------------ metric tables
def test_kerr_schild_tables_pins():
    gr = torus_grid(16, 12, 4)
    tab = wmetric.kerr_schild_tables(gr, a=0.9)
    loc, der = wmetric.unpack(tab)
    g = gr.ng
    for L in wmetric.LOCS:
        m = loc[L]
        sinth_nonzero = m["gu33"] != 0.0
        G = np.array([[m["g11"], m["g12"], m["g13"]], [m["g12"], m["g22"], m["g23"]],
                      [m["g13"], m["g23"], m["g33"]]])
        Gi = np.array([[m["gu11"], m["gu12"], m["gu13"]], [m["gu12"], m["gu22"], m["gu23"]],
                       [m["gu13"], m["gu23"], m["gu33"]]])
        prod = np.einsum("ijab,jkab->ikab", G, Gi)
        for i in range(3):
            for k in range(3):
                want = 1.0 if i == k else 0.0
                assert np.allclose(prod[i, k][sinth_nonzero], want, atol=1e-12)
        det = np.linalg.det(np.moveaxis(G, (0, 1), (-2, -1)))
        assert np.allclose(np.sqrt(np.maximum(det, 0)), m["sqrtg"], rtol=1e-10, atol=1e-12)
    # alpha sqrt(gamma) = r Sigma |sin theta| at centres
    i = np.arange(-g, gr.n[0] + g)
    j = np.arange(-g, gr.n[1] + g)
    r = np.exp(gr.x0[0] + (i + 0.5) * gr.dx[0])[None, :]
    th = (gr.x0[1] + (j + 0.5) * gr.dx[1])[:, None]
    sig = r * r + 0.81 * np.cos(th) ** 2
    assert np.allclose(loc["C"]["alpha"] * loc["C"]["sqrtg"], r * sig * np.abs(np.sin(th)), rtol=1e-12)
    # complex-step derivatives against 4th-order central differences
    h = 1e-4
    x1 = gr.x0[0] + (i + 0.5) * gr.dx[0]
    for k, axis in (("d1", 0), ("d2", 1)):
        for nm in ("alpha", "beta1", "g11", "g13", "g22", "g33"):
            def f(dx1, dth):
                X1, TH = np.meshgrid(x1 + dx1, np.abs(th[:, 0]) + dth)
                return np.asarray(wmetric._ks_fields(X1, TH, 0.9, 1.0)[nm]) * np.ones_like(X1)
            e = [(0, 0)] * 4
            if axis == 0:
                pts = [f(s * h, 0) for s in (-2, -1, 1, 2)]
            else:
                pts = [f(0, s * h) for s in (-2, -1, 1, 2)]
            fd4 = (pts[0] - 8 * pts[1] + 8 * pts[2] - pts[3]) / (12 * h)
            inner = slice(g, g + gr.n[1])
            # central differences carry round-off of order eps |f| / h
            tol = 1e-11 * np.abs(pts[2]).max() / h + 1e-12
            assert np.max(np.abs(der[k + "_" + nm][inner] - fd4[inner])) <= tol


def test_flat_spherical_static_state_residual_converges():
    """Uniform static gas in flat log-spherical coordinates is an exact
    equilibrium: the geometric sources balance the flux divergence, so the
    discrete RHS must vanish at the scheme's order."""
    res = []
    for n in (16, 32):
        gr = GridSpec(n=(n, n, 4), coord=LOGSPH, x0=(np.log(2.0), 0.6, 0.0),
                      dx=(np.log(4.0) / n, 1.2 / n, 0.1),
                      bc=(BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC))
        tab = wmetric.kerr_schild_tables(gr, a=0.0, m=0.0)
        s = Solver(gr, tab)
        d = box.uniform_state(gr, rho=1.0, p=0.1)
        s.set_face_fields(d)
        s.set_primitives(d)
        L = s.rhs()
        sg = s.centre_metric()["sqrtg"]
        # away from the outflow boundaries (the copy there is not an equilibrium)
        c = slice(6, -6)
        res.append(max(np.max(np.abs((L[k] / sg)[:, c, c])) for k in ("S1", "S2", "tau")))
    order = np.log2(res[0] / res[1])
    assert order >= 4.5, (res, order)


def test_gr_path_with_flat_tables_equals_default():
    s1 = _box_solver(8)
    g, d = box.turbulent_box(8)
    s2 = Solver(g, wmetric.minkowski_tables(g))
    s2.curl_potential(d)
    s2.set_primitives(d)
    s1.rk_step(1e-3)
    s2.rk_step(1e-3)
    for k in ("D", "S1", "tau", "Bf2"):
        assert np.array_equal(s1.interior(s1.U[k]), s2.interior(s2.U[k]))


def test_axis_boundary_reflection():
    gr = torus_grid(8, 6, 8)
    s = Solver(gr, wmetric.kerr_schild_tables(gr))
    rng = np.random.default_rng(1)
    for k in s.P:
        s.set_interior(s.P[k], rng.normal(size=(8, 6, 8)))
    from oracle.boundary import fill_centred
    fill_centred(s.P, gr)
    g = gr.ng
    # ghost row j=-1 equals row 0 at phi + pi, u2 flipped
    for k in range(8):
        kk = (k + 4) % 8
        assert np.array_equal(s.P["rho"][k + g, g - 1, g:g + 8], s.P["rho"][kk + g, g, g:g + 8])
        assert np.array_equal(s.P["u2"][k + g, g - 1, g:g + 8], -s.P["u2"][kk + g, g, g:g + 8])
        assert np.array_equal(s.P["u1"][k + g, g + 6, g:g + 8], s.P["u1"][kk + g, g + 5, g:g + 8])
    # outflow in r, no inflow at the outer radius
    assert np.array_equal(s.P["rho"][:, :, g - 3], s.P["rho"][:, :, g])
    assert np.all(s.P["u1"][:, :, g + 8:] >= 0.0)


def test_uct_reduces_to_1d_hll():
    """Data varying along x^1 only: E_3 at x^3-edges must equal minus the 1-D
    HLL flux of B^2 through the x^1 faces built from the same face states."""
    g, d = box.entropy_wave_1d(16, axis=0, ntrans=4)
    s = Solver(g)
    rng = np.random.default_rng(2)
    x = (np.arange(16) + 0.5) / 16
    # transverse field and velocity varying along x
    d["B2f"] = np.broadcast_to(np.pad(0.2 + 0.1 * np.sin(2 * np.pi * x), 5, mode="wrap")[None, None, :], g.shape).copy()
    d["u2"] = np.broadcast_to((0.1 * np.cos(2 * np.pi * x))[None, None, :], d["u2"].shape).copy()
    s.set_face_fields(d)
    s.set_primitives(d)
    from oracle.boundary import fill_centred
    fill_centred(s.P, g)
    _, _, fdat, edges = s.rhs_parts()
    X = fdat[0]
    gg = g.ng
    sl = (slice(gg, gg + 4), slice(gg, gg + 4), slice(gg - 3, gg + 16 + 2))
    from oracle.mp5 import face_states
    from oracle.fd import take
    bl, br = face_states(s.U["Bf2"], 0, -3, 16 + 2, gg, take)
    b1 = s.U["Bf1"][sl]
    vxl, vxr = X["vdL"][sl], X["vdR"][sl]
    vyl, vyr = X["vcL"][sl], X["vcR"][sl]
    bl, br = bl[gg:gg + 4, gg:gg + 4], br[gg:gg + 4, gg:gg + 4]
    fl = vxl * bl - vyl * b1
    fr = vxr * br - vyr * b1
    ap, am = X["ap"][sl], X["am"][sl]
    hll = (ap * fl + am * fr - ap * am * (br - bl)) / (ap + am)
    e3 = edges[2][sl]
    assert np.allclose(e3, -hll, rtol=1e-12, atol=1e-15)
