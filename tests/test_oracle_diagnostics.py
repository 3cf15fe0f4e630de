"""Pins of the shell-flux diagnostic (oracle/diagnostics.py)."""
import numpy as np

from oracle.diagnostics import shell_fluxes


def _uniform_box(rho, v1, p, b1, n=8):
    from workloads.grid import box
    from oracle.scheme import Solver
    g = box(n)
    s = Solver(g)
    w = 1.0 / np.sqrt(1.0 - v1 * v1)
    sh = (n, n, n)
    data = {"rho": np.full(sh, rho), "u1": np.full(sh, w * v1), "u2": np.zeros(sh),
            "u3": np.zeros(sh), "p": np.full(sh, p)}
    gs = g.shape
    data.update({"B1f": np.full(gs, b1), "B2f": np.zeros(gs), "B3f": np.zeros(gs)})
    s.set_face_fields(data)
    s.set_primitives(data)
    return g, s, w


def test_uniform_state_closed_forms():
    """Uniform flow along x^1 with a uniform field along x^1 in a flat box:
    every shell carries D v^1, (S^1 - v^1 D) and |B^1| / 2 times its area."""
    rho, v1, p, b1, gam = 1.3, 0.4, 0.2, 0.7, 4.0 / 3.0
    g, s, w = _uniform_box(rho, v1, p, b1)
    out = shell_fluxes(s)
    area = 1.0
    h = 1.0 + gam / (gam - 1.0) * p / rho
    y = rho * h * w * w
    # B parallel to v: E = 0, (v.B) = v1 b1, S^1 = (y + B^2) v1 - (v1 b1) b1 = y v1
    s1 = y * v1
    for key, want in (("F_D", rho * w * v1 * area), ("F_tau", (s1 - v1 * rho * w) * area),
                      ("Phi", 0.5 * b1 * area), ("Phi_s", b1 * area)):
        assert np.allclose(out[key], want, rtol=1e-13, atol=0), (key, out[key], want)


def test_coordinate_static_gas_on_kerr_schild():
    """Gas at rest in Kerr-Schild coordinates (v = beta / alpha, no field)
    outside the ergosphere (inside it no observer can be at rest in these
    coordinates): no mass crosses any sphere (relative to the size of the two
    cancelling terms, sqrt(gamma) D |beta^1|), and the energy flux is the
    pressure term sqrt(gamma) beta^1 p alone."""
    from workloads.torus import torus
    from workloads.grid import GridSpec
    from workloads.metric import kerr_schild_tables
    from oracle.scheme import Solver
    g0, d, tab = torus(24, 12, 8)
    # the same grid starting outside the ergosphere (r <= 2 for a = 0.9), where
    # observers at rest in these coordinates exist
    g = GridSpec(n=g0.n, ng=g0.ng, coord=g0.coord, x0=(np.log(2.2), g0.x0[1], g0.x0[2]), dx=g0.dx,
                 bc=g0.bc, gamma_ad=g0.gamma_ad)
    s = Solver(g, kerr_schild_tables(g))
    m = s.centre_metric()
    sh = (g.n[2], g.n[1], g.n[0])      # the tables are axisymmetric: broadcast over x^3
    v1 = np.broadcast_to(m["beta1"] / m["alpha"], sh)
    vv = m["g11"] * v1 * v1
    assert vv.max() < 1.0
    w = 1.0 / np.sqrt(1.0 - vv)
    rng = np.random.default_rng(3)
    rho = 10.0 ** rng.uniform(-3, 0, sh)
    p = 10.0 ** rng.uniform(-4, -1, sh)
    data = {"rho": rho, "u1": w * v1, "u2": np.zeros(sh), "u3": np.zeros(sh), "p": p}
    gs = g.shape
    data.update({"B1f": np.zeros(gs), "B2f": np.zeros(gs), "B3f": np.zeros(gs)})
    s.set_face_fields(data)
    s.set_primitives(data)
    out = shell_fluxes(s)
    area = g.dx[1] * g.dx[2]
    terms = (m["sqrtg"] * rho * w * np.abs(m["beta1"])).sum(axis=(0, 1)) * area
    assert np.all(np.abs(out["F_D"]) <= 1e-13 * terms)
    want = (m["sqrtg"] * m["beta1"] * p).sum(axis=(0, 1)) * area
    assert np.allclose(out["F_tau"], want, rtol=1e-12, atol=0)
    assert np.all(out["Phi"] == 0.0)


def test_loop_field_has_no_net_flux():
    """The torus' loop field (curl of A_phi, zero near the axis): the signed
    flux through every sphere vanishes to round-off."""
    from workloads.torus import torus
    from oracle.scheme import Solver
    g, d, tab = torus(32, 16, 16)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    out = shell_fluxes(s)
    assert out["Phi"].max() > 0
    assert np.all(np.abs(out["Phi_s"]) <= 1e-13 * out["scale_B"] + 1e-300)
