"""Pins of the shell-flux diagnostic (oracle/diagnostics.py)."""
import numpy as np
import pytest

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


# ---------------------------------------------------------------- MRI resolution
def _ks_solver(n=(16, 12, 8), a=0.9, m=1.0, shift23=None):
    """Kerr-Schild tables; shift23 = (beta^2, beta^3) adds a tangential shift
    at the centres (still a valid 3+1 metric, e.g. a rotating frame), since
    Kerr-Schild itself has beta^2 = beta^3 = 0."""
    from workloads.grid import torus_grid
    from workloads.metric import kerr_schild_tables, comp_index
    from oracle.scheme import Solver
    g = torus_grid(*n)
    tab = kerr_schild_tables(g, a=a, m=m)
    if shift23 is not None:
        tab[comp_index("C", "beta2")] = shift23[0]
        tab[comp_index("C", "beta3")] = shift23[1]
    return g, Solver(g, tab)


def _set_prims(s, rho, u, p, b):
    for k, v in zip(("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3"), (rho, *u, p, *b)):
        s.set_interior(s.P[k], v)


@pytest.mark.parametrize("shift23", [None, (0.003, 0.01)])
def test_fluid_frame_four_vectors_on_kerr_schild(shift23):
    """On the a = 0.9 Kerr-Schild metric (and with an added tangential
    shift), for random states: u^mu u_mu = -1, u^mu b_mu = 0 and
    b^mu b_mu = b^2, with the full 4-metric built from alpha, beta and gamma;
    Omega = u^3 / u^t."""
    from oracle import physics
    from oracle.diagnostics import fluid_frame
    g, s = _ks_solver(shift23=shift23)
    m = s.centre_metric()
    sh = (g.n[2], g.n[1], g.n[0])
    rng = np.random.default_rng(21)
    u = tuple(rng.uniform(-0.5, 0.5, sh) for _ in range(3))
    b = tuple(rng.uniform(-1, 1, sh) for _ in range(3))
    rho, p = 10.0 ** rng.uniform(-2, 0, sh), 10.0 ** rng.uniform(-3, -1, sh)
    st = physics.state(rho, u, p, b, m, g.gamma_ad)
    ff = fluid_frame(st, m)
    al = m["alpha"]
    beta = (m["beta1"], m["beta2"], m["beta3"])
    beta_l = physics.lower(m, beta)
    g_tt = -al * al + sum(beta_l[i] * beta[i] for i in range(3))

    def dot(at, a, bt, bb):
        r = g_tt * at * bt
        for i in range(3):
            r = r + beta_l[i] * (at * bb[i] + bt * a[i])
            for j in range(3):
                r = r + physics.gl(m, i + 1, j + 1) * a[i] * bb[j]
        return r

    uu = dot(ff["ut"], ff["u"], ff["ut"], ff["u"])
    ub = dot(ff["ut"], ff["u"], ff["bt"], ff["b"])
    bb = dot(ff["bt"], ff["b"], ff["bt"], ff["b"])
    assert np.max(np.abs(uu + 1.0)) < 1e-12
    scale = np.sqrt(ff["b2"]) * np.abs(ff["ut"]) * 10
    assert np.max(np.abs(ub) / scale) < 1e-13
    assert np.max(np.abs(bb - ff["b2"]) / ff["b2"]) < 1e-11
    # relative to the two terms of Omega = alpha v^3 - beta^3, which can cancel
    terms = np.abs(al * st["v"][2]) + np.abs(beta[2])
    assert np.max(np.abs(ff["Omega"] - ff["u"][2] / ff["ut"]) / terms) < 1e-14


def test_mri_quality_newtonian_limit():
    """Flat spacetime in (ln r, theta, phi) (Kerr-Schild with m = 0): a cold,
    slowly rotating gas with a weak field has Q_2 equal to the Newtonian
    2 pi v_A / (Omega r dtheta), v_A = r |B^theta| / sqrt(rho) (the orthonormal
    field over the root of the density), to the size of the relativistic
    corrections (v^2, b^2 / rho, p / rho below 1e-6)."""
    from oracle.diagnostics import mri_quality
    g, s = _ks_solver(a=0.0, m=0.0)
    sh = (g.n[2], g.n[1], g.n[0])
    r = np.exp(g.x0[0] + (np.arange(g.n[0]) + 0.5) * g.dx[0])[None, None, :]
    th = (g.x0[1] + (np.arange(g.n[1]) + 0.5) * g.dx[1])[None, :, None]
    rng = np.random.default_rng(5)
    rho = np.broadcast_to(10.0 ** rng.uniform(-1, 0, (1, 1, g.n[0])), sh)
    omega = 1e-6 / np.broadcast_to(r, sh)
    u3 = omega                                   # W = 1 + O(1e-10)
    bth = np.broadcast_to(1e-5 / r, sh) * (1 + 0 * th)
    b = (np.full(sh, 1e-6) / np.broadcast_to(r, sh), bth, np.full(sh, 3e-7))
    _set_prims(s, rho, (np.zeros(sh), np.zeros(sh), u3), np.full(sh, 1e-9), b)
    out = mri_quality(s, rho_cut=0.0)
    va = np.broadcast_to(r, sh) * np.abs(bth) / np.sqrt(rho)
    newton = 2 * np.pi * va / (omega * np.broadcast_to(r, sh) * g.dx[1])
    assert np.max(np.abs(out["Q2"] / newton - 1)) < 1e-5
    # Q_3 uses the field and zone width along phi the same way
    va3 = np.broadcast_to(r * np.sin(th), sh) * 3e-7 / np.sqrt(rho)
    newton3 = 2 * np.pi * va3 / (omega * np.broadcast_to(r * np.sin(th), sh) * g.dx[2])
    assert np.max(np.abs(out["Q3"] / newton3 - 1)) < 1e-5


def test_mri_quality_gas_at_rest_in_a_rotating_frame():
    """Flat space seen from a frame rotating at rate w (shift beta^3 = w):
    gas at rest in the inertial frame is the Eulerian observer (v = 0) and
    turns at Omega = -w in these coordinates, so Q_2 = 2 pi |B^2| /
    (w dtheta sqrt(rho h + B^2))."""
    from oracle.diagnostics import mri_quality
    wr = 1e-3
    g, s = _ks_solver(a=0.0, m=0.0, shift23=(0.0, wr))
    sh = (g.n[2], g.n[1], g.n[0])
    z = np.zeros(sh)
    b2c = np.full(sh, 2e-3)
    _set_prims(s, np.ones(sh), (z, z, z), np.full(sh, 0.1), (z, b2c, z))
    out = mri_quality(s, rho_cut=0.0)
    r = np.exp(g.x0[0] + (np.arange(g.n[0]) + 0.5) * g.dx[0])[None, None, :]
    bsq = np.broadcast_to(r * r, sh) * b2c ** 2          # gamma_22 (B^2)^2, W = 1
    h = 1.0 + g.gamma_ad / (g.gamma_ad - 1.0) * 0.1
    want = 2 * np.pi * b2c / (wr * g.dx[1] * np.sqrt(h + bsq))
    assert np.allclose(out["Q2"], want, rtol=1e-13, atol=0)


def test_mri_quality_invariances_and_body_sums():
    """Q is unchanged when the field flips sign, zero without field; the shell
    sums run over the body zones (rho > rho_cut) with weight rho sqrt(gamma)."""
    from oracle.diagnostics import mri_quality
    g, s = _ks_solver()
    sh = (g.n[2], g.n[1], g.n[0])
    rng = np.random.default_rng(8)
    rho = 10.0 ** rng.uniform(-3, 0, sh)
    u = (rng.uniform(-0.1, 0.1, sh), rng.uniform(-0.05, 0.05, sh), rng.uniform(0.01, 0.05, sh))
    b = tuple(rng.uniform(-0.1, 0.1, sh) for _ in range(3))
    p = 10.0 ** rng.uniform(-4, -1, sh)
    _set_prims(s, rho, u, p, b)
    a = mri_quality(s, rho_cut=0.05)
    _set_prims(s, rho, u, p, tuple(-x for x in b))
    bneg = mri_quality(s, rho_cut=0.05)
    assert np.array_equal(a["Q2"], bneg["Q2"]) and np.array_equal(a["Q3"], bneg["Q3"])
    body = rho > 0.05
    sg = np.broadcast_to(s.centre_metric()["sqrtg"], sh)
    assert np.array_equal(a["n_body"], body.sum(axis=(0, 1)).astype(float))
    assert np.allclose(a["w"], np.where(body, rho * sg, 0).sum(axis=(0, 1)), rtol=1e-14, atol=0)
    assert np.allclose(a["wQ2"], np.where(body, rho * sg * a["Q2"], 0).sum(axis=(0, 1)), rtol=1e-14, atol=0)
    assert np.all(a["n_Q2_ok"] <= a["n_body"])
    _set_prims(s, rho, u, p, tuple(0 * x for x in b))
    z = mri_quality(s, rho_cut=0.05)
    assert np.all(z["Q2"] == 0) and np.all(z["n_Q2_ok"] == 0) and np.all(z["n_Q3_ok"] == 0)
