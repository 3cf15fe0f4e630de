"""Pins of the oracle's CFL step, floors / Lorentz-factor cap / atmosphere
reset, face-field ghost fill and the positivity bound of reconstructed rho
and p.  Each expected value is a closed form or an index rule written out
here from the scheme's definition, not a call of the function under test:

  * CFL step (SSP-RK3 stability bound with the summed form over
    directions): dt = C / max_cells sum_d max(|lambda+_d|, |lambda-_d|) / dx_d;
    for gas at rest lambda+-_d = +-alpha a sqrt(gamma^dd) - beta^d with the
    fast speed a^2 = c_s^2 + v_A^2 - c_s^2 v_A^2; for a flat state moving
    along one axis the speeds along it are the relativistic sums
    (v +- a)/(1 +- v a) and across it +-a sqrt((1 - v^2)/(1 - v^2 a^2));
  * floors: rho >= 1e-4 r^-3/2, p >= 1e-6 r^-5/2, W <= W_max with u rescaled
    by sqrt((W_max^2 - 1)/(W^2 - 1)); a zone whose inversion fails becomes
    atmosphere (floor rho and p, at rest) and every floored zone gets its
    conserved variables recomputed, which for gas at rest are
    D = sqrt(g) rho, S = 0, tau = sqrt(g) (p/(Gamma-1) + B^2/2);
  * face ghost fill on a torus grid: the rules of the outflow, polar-axis
    and periodic boundaries written as explicit index loops;
  * positivity bound: inactive on smooth data, and on a narrow density dip
    where MP5 undershoots it raises the left state to 0.1 rho_j and the
    right state to 0.1 rho_{j+1}, seen through the HLL mass flux of gas at
    rest, F = -a (rho_R - rho_L)/2.
"""
import math

import numpy as np
import pytest

from oracle import scheme
from oracle.scheme import Solver
from oracle.boundary import fill_faces, fill_centred
from oracle.mp5 import mp5
from workloads import metric as wmetric
from workloads.grid import GridSpec, torus_grid, box

GAM = 4.0 / 3.0


# ------------------------------------------------------------------ CFL step
def _fast_speed2(rho, p, b2):
    rhoh = rho + GAM / (GAM - 1.0) * p
    cs2 = GAM * p / rhoh
    va2 = b2 / (rhoh + b2)
    return cs2 + va2 - cs2 * va2


def test_cfl_dt_static_kerr_schild_closed_form():
    """Gas at rest with a random field on a log-spherical Kerr-Schild grid
    (three unequal spacings, beta^1 != 0 so |lambda-| != |lambda+|)."""
    gr = torus_grid(8, 6, 4)
    tab = wmetric.kerr_schild_tables(gr)
    s = Solver(gr, tab)
    rng = np.random.default_rng(11)
    shp = (4, 6, 8)
    rho = rng.uniform(0.5, 2.0, shp)
    p = rng.uniform(0.05, 0.2, shp)
    B = [rng.normal(scale=0.05, size=shp) for _ in range(3)]
    for k, v in (("rho", rho), ("p", p), ("u1", 0 * rho), ("u2", 0 * rho), ("u3", 0 * rho),
                 ("B1", B[0]), ("B2", B[1]), ("B3", B[2])):
        s.set_interior(s.P[k], v)
    g = gr.ng
    loc, _ = wmetric.unpack(tab)
    C = {nm: a[g:-g, g:-g][None] for nm, a in loc["C"].items()}
    gl = [["g11", "g12", "g13"], ["g12", "g22", "g23"], ["g13", "g23", "g33"]]
    b2 = sum(C[gl[a][b]] * B[a] * B[b] for a in range(3) for b in range(3))
    a_f = np.sqrt(_fast_speed2(rho, p, b2))
    tot = 0.0
    for d, gu in enumerate(("gu11", "gu22", "gu33")):
        lam = C["alpha"] * a_f * np.sqrt(C[gu])
        tot = tot + (lam + np.abs(C["beta%d" % (d + 1)])) / gr.dx[d]
    want = gr.cfl / np.max(tot)
    assert abs(s.cfl_dt() / want - 1.0) < 1e-14
    # the summed form is not the maximum over directions, and each direction
    # uses its own spacing
    assert len(set(gr.dx)) == 3


def test_cfl_dt_moving_flat_state_closed_form():
    """Minkowski box with unequal spacings, gas moving along x^2 with W v
    varying per zone, B = 0: relativistic velocity addition along x^2, the
    transverse form across it."""
    gr = GridSpec(n=(4, 5, 6), dx=(0.1, 0.2, 0.05))
    s = Solver(gr)
    rng = np.random.default_rng(12)
    shp = (6, 5, 4)
    rho = rng.uniform(0.5, 2.0, shp)
    p = rng.uniform(0.05, 0.2, shp)
    v = rng.uniform(-0.8, 0.8, shp)
    W = 1.0 / np.sqrt(1.0 - v * v)
    for k, val in (("rho", rho), ("p", p), ("u1", 0 * rho), ("u2", W * v), ("u3", 0 * rho),
                   ("B1", 0 * rho), ("B2", 0 * rho), ("B3", 0 * rho)):
        s.set_interior(s.P[k], val)
    a = np.sqrt(_fast_speed2(rho, p, 0.0))
    along = (np.abs(v) + a) / (1.0 + np.abs(v) * a)
    across = a * np.sqrt((1.0 - v * v) / (1.0 - v * v * a * a))
    tot = across / gr.dx[0] + along / gr.dx[1] + across / gr.dx[2]
    want = gr.cfl / np.max(tot)
    assert abs(s.cfl_dt() / want - 1.0) < 1e-13


# ------------------------------------------------------------------ floors
RHO_FL, P_FL, W_MAX = (1e-4, -1.5), (1e-6, -2.5), 10.0


def _floored_torus():
    gr = torus_grid(8, 6, 4, rho_fl_a=RHO_FL[0], rho_fl_n=RHO_FL[1], p_fl_a=P_FL[0],
                    p_fl_n=P_FL[1], w_max=W_MAX)
    tab = wmetric.kerr_schild_tables(gr)
    s = Solver(gr, tab)
    g = gr.ng
    # a small radial face field (B^1 face values times the face sqrt(gamma))
    loc, _ = wmetric.unpack(tab)
    bf1 = np.zeros(gr.shape)
    bf1[:, :, :] = 1e-3 * loc["F1"]["sqrtg"][None]
    s.U["Bf1"] = bf1
    s.U["Bf2"] = np.zeros(gr.shape)
    s.U["Bf3"] = np.zeros(gr.shape)
    fill_faces(s.U, gr)
    shp = (4, 6, 8)
    data = {"rho": np.ones(shp), "p": np.full(shp, 0.1), "u1": np.zeros(shp),
            "u2": np.zeros(shp), "u3": np.zeros(shp)}
    r = np.exp(gr.x0[0] + (np.arange(8) + 0.5) * gr.dx[0])
    return gr, tab, s, data, r


def _centre(tab, gr, name):
    g = gr.ng
    return wmetric.unpack(tab)[0]["C"][name][g:-g, g:-g]


def test_floors_wcap_and_atmosphere_reset():
    gr, tab, s, data, r = _floored_torus()
    g = gr.ng
    # zone A (k, j, i) = (0, 2, 3): density below its floor
    zA = (0, 2, 3)
    data["rho"][zA] = 0.5 * RHO_FL[0] * r[zA[2]] ** RHO_FL[1]
    # zone B: pressure below its floor
    zB = (1, 3, 5)
    data["p"][zB] = 0.5 * P_FL[0] * r[zB[2]] ** P_FL[1]
    # zone C: Lorentz factor 20 along x^2 (gamma_22 = Sigma, no cross terms)
    zC = (2, 2, 6)
    sig = _centre(tab, gr, "g22")[zC[1], zC[2]]
    u2c = math.sqrt((20.0 ** 2 - 1.0) / sig)
    data["u2"][zC] = u2c
    s.set_primitives(data)
    # zone D: negative total energy (U = tau + D < 0): the inversion fails
    zD = (3, 4, 2)
    gz = tuple(x + g for x in zD)
    s.U["tau"][gz] = -2.0 * s.U["D"][gz]
    # zone E: momentum beyond what any state with this energy can carry
    zE = (1, 1, 4)
    gz = tuple(x + g for x in zE)
    s.U["S1"][gz] = 10.0 * (s.U["tau"][gz] + s.U["D"][gz]) * math.sqrt(_centre(tab, gr, "g11")[zE[1], zE[2]])
    Bc = [s.interior(s.P["B%d" % (q + 1)]).copy() for q in range(3)]
    st = s.cons2prim()
    P = {k: s.interior(v) for k, v in s.P.items()}
    U = {k: s.interior(v) for k, v in s.U.items()}
    sg = _centre(tab, gr, "sqrtg")
    gl = {nm: _centre(tab, gr, nm) for nm in ("g11", "g12", "g13", "g22", "g23", "g33")}

    def b2_at(z):
        k, j, i = z
        b = [Bc[q][z] for q in range(3)]
        m = [[gl["g11"], gl["g12"], gl["g13"]], [gl["g12"], gl["g22"], gl["g23"]],
             [gl["g13"], gl["g23"], gl["g33"]]]
        return sum(m[a][c][j, i] * b[a] * b[c] for a in range(3) for c in range(3))

    def at_rest_cons(z, rho, p):
        k, j, i = z
        return (sg[j, i] * rho, 0.0, sg[j, i] * (p / (GAM - 1.0) + 0.5 * b2_at(z)))

    assert st["n_fail"] == 2
    assert st["n_floor_rho"] == 1 and st["n_floor_p"] == 1 and st["n_wcap"] == 1
    # A: rho raised to exactly its floor, p and rest frame kept; U recomputed
    rfl = RHO_FL[0] * r[zA[2]] ** RHO_FL[1]
    assert P["rho"][zA] == rfl
    assert abs(P["p"][zA] / 0.1 - 1.0) < 1e-10
    # (the inverted velocity of zones A and B is zero up to the inversion's
    # round-off, so their recomputed U meets the at-rest form to that level)
    D, S, tau = at_rest_cons(zA, rfl, P["p"][zA])
    assert abs(U["D"][zA] / D - 1) < 1e-12 and abs(U["tau"][zA] / tau - 1) < 1e-10
    # B: p raised to its floor, rho kept
    pfl = P_FL[0] * r[zB[2]] ** P_FL[1]
    assert P["p"][zB] == pfl and abs(P["rho"][zB] - 1.0) < 1e-10
    D, S, tau = at_rest_cons(zB, P["rho"][zB], pfl)
    assert abs(U["D"][zB] / D - 1) < 1e-12 and abs(U["tau"][zB] / tau - 1) < 1e-10
    # C: W capped at exactly W_max, direction kept
    w_new = math.sqrt(1.0 + gl["g22"][zC[1], zC[2]] * P["u2"][zC] ** 2)
    assert abs(w_new - W_MAX) < 1e-12
    assert abs(P["u2"][zC] / (u2c * math.sqrt((W_MAX ** 2 - 1) / (20.0 ** 2 - 1))) - 1) < 1e-10
    assert P["u1"][zC] == 0.0 or abs(P["u1"][zC]) < 1e-12
    # D, E: failed zones are atmosphere at rest with U recomputed
    for z in (zD, zE):
        rfl = RHO_FL[0] * r[z[2]] ** RHO_FL[1]
        pfl = P_FL[0] * r[z[2]] ** P_FL[1]
        assert P["rho"][z] == rfl and P["p"][z] == pfl
        assert P["u1"][z] == P["u2"][z] == P["u3"][z] == 0.0
        D, S, tau = at_rest_cons(z, rfl, pfl)
        assert abs(U["D"][z] / D - 1) < 1e-14 and abs(U["tau"][z] / tau - 1) < 1e-14
        assert U["S1"][z] == U["S2"][z] == U["S3"][z] == 0.0
    # the recomputed U of the capped zone inverts back to the capped state
    P_capped = {k: P[k][zC] for k in ("rho", "p", "u1", "u2", "u3")}
    st2 = s.cons2prim(guess="cold")
    # (W comes back equal to W_max up to round-off, so the cap may act again)
    assert st2["n_fail"] == 0
    P2 = {k: s.interior(v) for k, v in s.P.items()}
    for k, v in P_capped.items():
        assert abs(P2[k][zC] - v) <= 1e-10 * max(abs(v), 1.0), k


def test_failed_zone_keeps_primitives_without_floors():
    """Box (floors off): a failed zone keeps its previous primitives and its
    conserved variables are not rewritten."""
    gr = box(6)
    s = Solver(gr)
    shp = (6, 6, 6)
    rng = np.random.default_rng(3)
    data = {"rho": rng.uniform(0.5, 1.5, shp), "p": rng.uniform(0.05, 0.2, shp),
            "u1": rng.normal(scale=0.1, size=shp), "u2": np.zeros(shp), "u3": np.zeros(shp)}
    for f in ("Bf1", "Bf2", "Bf3"):
        s.U[f] = np.zeros(gr.shape)
    s.set_primitives(data)
    g = gr.ng
    z = (2, 3, 4)
    gz = tuple(x + g for x in z)
    before = {k: s.P[k][gz] for k in s.P}
    s.U["tau"][gz] = -3.0 * s.U["D"][gz]
    tau_bad = s.U["tau"][gz]
    st = s.cons2prim()
    assert st["n_fail"] == 1
    for k, v in before.items():
        assert s.P[k][gz] == v, k
    assert s.U["tau"][gz] == tau_bad


# ------------------------------------------------------------------ face ghost fill
@pytest.mark.parametrize("flo", [3, 2])
def test_face_ghost_fill_torus_rules(flo):
    """Faces normal to the outflow (x^1) and axis (x^2) boundaries: the
    ghost faces -flo .. -1 and n .. n + flo - 2 and the axis faces keep their
    (evolved) values; the rules fill only the faces beyond, and every face
    field's tangential ghosts."""
    n1, n2, n3 = 6, 6, 4
    gr = torus_grid(n1, n2, n3)
    g = gr.ng
    rng = np.random.default_rng(21)
    U = {f: rng.normal(size=gr.shape) for f in ("Bf1", "Bf2", "Bf3")}
    src = {f: v.copy() for f, v in U.items()}
    fill_faces(U, gr, flo)
    A = lambda f, i, j, k: U[f][k + g, j + g, i + g]
    S = lambda f, i, j, k: src[f][k + g, j + g, i + g]
    # interior elements are untouched (owned faces, the upper axis face too)
    for f in U:
        assert np.array_equal(U[f][g:-g, g:-g, g:-g], src[f][g:-g, g:-g, g:-g]), f
    for k in range(n3):
        kk = (k + n3 // 2) % n3
        for i in range(n1):
            # x^2-normal faces: the evolved ghosts (the lower axis face among
            # them) are untouched; beyond, ghost face -2-m is minus face m
            # half a turn away, ghost face n2+m minus face n2-2-m
            for j in list(range(-flo, 0)) + list(range(n2, n2 + flo - 1)):
                assert A("Bf2", i, j, k) == S("Bf2", i, j, k), (i, j, k)
            for m in range(flo - 1, g - 1):
                assert A("Bf2", i, -2 - m, k) == -S("Bf2", i, m, kk)
            for m in range(flo - 1, g):
                assert A("Bf2", i, n2 + m, k) == -S("Bf2", i, n2 - 2 - m, kk)
            # tangential faces across the axis: rows mirror, x^3 faces flip
            for m in range(g):
                assert A("Bf3", i, -1 - m, k) == -S("Bf3", i, m, kk)
                assert A("Bf3", i, n2 + m, k) == -S("Bf3", i, n2 - 1 - m, kk)
                assert A("Bf1", i, -1 - m, k) == S("Bf1", i, m, kk)
                assert A("Bf1", i, n2 + m, k) == S("Bf1", i, n2 - 1 - m, kk)
        for j in range(n2):
            # outflow in x^1: the x^1-normal field keeps its evolved ghosts
            # and copies the outermost of them beyond; the others copy their
            # nearest owned x^1 index
            for m in range(1, g + 1):
                lo, hi = -m, n1 - 1 + m
                want_lo = S("Bf1", lo, j, k) if m <= flo else S("Bf1", -flo, j, k)
                want_hi = S("Bf1", hi, j, k) if hi <= n1 + flo - 2 else S("Bf1", n1 + flo - 2, j, k)
                assert A("Bf1", lo, j, k) == want_lo, (m, j, k)
                assert A("Bf1", hi, j, k) == want_hi, (m, j, k)
                for f in ("Bf2", "Bf3"):
                    assert A(f, lo, j, k) == S(f, 0, j, k), (f, m, j, k)
                    assert A(f, hi, j, k) == S(f, n1 - 1, j, k), (f, m, j, k)
    # periodic x^3: every ghost plane is the interior plane k mod n3
    for f in U:
        for kg in list(range(-g, 0)) + list(range(n3, n3 + g)):
            assert np.array_equal(U[f][kg + g], U[f][kg % n3 + g])


def test_centred_outflow_no_inflow_and_axis():
    """Centred fields: outflow copies the nearest interior cell, u^1 at the
    outer radius is clipped to >= 0, the axis mirrors rows with u^2, u^3,
    B^2, B^3 negated half a turn away."""
    n1, n2, n3 = 6, 6, 4
    gr = torus_grid(n1, n2, n3)
    g = gr.ng
    rng = np.random.default_rng(22)
    P = {k: rng.normal(size=gr.shape) for k in scheme.PRIM}
    src = {k: v.copy() for k, v in P.items()}
    fill_centred(P, gr)
    for k in range(n3):
        kk = (k + n3 // 2) % n3
        for j in range(n2):
            for m in range(1, g + 1):
                assert P["rho"][k + g, j + g, g - m] == src["rho"][k + g, j + g, g]
                assert P["u1"][k + g, j + g, g + n1 - 1 + m] == max(src["u1"][k + g, j + g, g + n1 - 1], 0.0)
                assert P["u1"][k + g, j + g, g - m] == src["u1"][k + g, j + g, g]
        for i in range(n1):
            for m in range(g):
                for name in scheme.PRIM:
                    sgn = -1.0 if name in ("u2", "u3", "B2", "B3") else 1.0
                    assert P[name][k + g, -1 - m + g, i + g] == sgn * src[name][kk + g, m + g, i + g]
                    assert P[name][k + g, n2 + m + g, i + g] == sgn * src[name][kk + g, n2 - 1 - m + g, i + g]


# ------------------------------------------------------------------ positivity bound
def _static_x1_box(rho_row, p=0.1):
    n1 = len(rho_row)
    gr = GridSpec(n=(n1, 4, 4), dx=(1.0 / n1, 0.25, 0.25))
    s = Solver(gr)
    shp = (4, 4, n1)
    rho = np.broadcast_to(np.asarray(rho_row, dtype=np.float64)[None, None, :], shp).copy()
    for k, v in (("rho", rho), ("p", np.full(shp, p)), ("u1", 0 * rho), ("u2", 0 * rho),
                 ("u3", 0 * rho), ("B1", 0 * rho), ("B2", 0 * rho), ("B3", 0 * rho)):
        s.set_interior(s.P[k], v)
    for f in ("Bf1", "Bf2", "Bf3"):
        s.U[f] = np.zeros(gr.shape)
    fill_centred(s.P, gr)
    return gr, s


def test_positivity_bound_on_a_density_dip():
    # a two-cell dip: MP5 undershoots on both sides of the face between the
    # two low cells
    row = [1.0, 1.0, 2.0, 0.001, 0.002, 2.0, 1.0, 1.0]
    q = np.array(row)
    n = len(q)
    c = lambda j: q[j % n]
    j = 3                                     # face 3 + 1/2, between cells 3 and 4
    l_mp5 = float(mp5(c(j - 2), c(j - 1), c(j), c(j + 1), c(j + 2)))
    r_mp5 = float(mp5(c(j + 3), c(j + 2), c(j + 1), c(j), c(j - 1)))
    assert l_mp5 < 0.1 * c(j) and r_mp5 < 0.1 * c(j + 1)   # both undershoot
    rho_l, rho_r = 0.1 * c(j), 0.1 * c(j + 1)
    p = 0.1

    def cs(rho):
        return math.sqrt(GAM * p / (rho + GAM / (GAM - 1.0) * p))
    a = max(cs(rho_l), cs(rho_r))
    want = -0.5 * a * (rho_r - rho_l)
    gr, s = _static_x1_box(row, p)
    out = s.sweep(0)
    g = gr.ng
    got = out["F_D"][g + 1, g + 2, g + j]
    assert abs(got - want) <= 1e-15 * abs(want) + 1e-18, (got, want)
    # the momentum flux of gas at rest is the pressure, untouched by the bound
    assert abs(out["F_S1"][g + 1, g + 2, g + j] - p) < 1e-15


def test_positivity_bound_inactive_on_smooth_data(monkeypatch):
    """On the turbulent box the bound changes nothing: every face output of
    the three sweeps is the same with the bound switched off."""
    from workloads import box as wbox
    gr, d = wbox.turbulent_box(12)
    s = Solver(gr)
    s.curl_potential(d)
    s.set_primitives(d)
    fill_centred(s.P, gr)
    with_bound = [s.sweep(dd) for dd in range(3)]
    monkeypatch.setattr(scheme, "POS_FRAC", 0.0)
    without = [s.sweep(dd) for dd in range(3)]
    for a, b in zip(with_bound, without):
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
