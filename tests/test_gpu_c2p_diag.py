"""GPU parity of the inversion's failure paths and of the diagnostics, through
the C ABI, against the FP64 oracle on identical inputs: the oracle's state is
copied into the GPU grid (primitives with ghosts, interior hydro conserved
variables, face fields with ghosts), both invert or reduce it, and every
zone, counter and diagnostic is compared.

Injected failures (the inversion fails for a zone with U = tau + D <= 0, or
with a momentum no state of that energy can carry, S^2 > (tau + D)^2):
  * box (floors off): a failed zone keeps its previous primitives and its
    conserved variables; strict mode returns ENOCONV;
  * torus (floors on): a failed zone becomes atmosphere at rest and its
    conserved variables are recomputed; density and pressure floors and the
    Lorentz-factor cap W <= 10 act on planted zones.
Iteration counts: the inversion stops when its residual is at the round-off
level of its own evaluation, which the two sides evaluate in different
orders, so a zone's count may differ by one where the residual sits at that
threshold; per-zone counts are compared through the batched point inversion
(same Newton) and the grid totals within the number of such zones."""
import math

import numpy as np
import pytest

from helpers import max_rel, interior

gpu = pytest.mark.gpu

PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")
HYDRO = ("D", "S1", "S2", "S3", "tau")


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _load_oracle_state(s, G):
    """Oracle state -> GPU grid: primitives (ghosted), interior hydro
    conserved variables, face fields (ghosted)."""
    import torch
    gg = s.g
    for f, k in enumerate(PRIM):
        G.field_view(G.prim, f).copy_(torch.from_numpy(np.ascontiguousarray(s.P[k])))
    for f, k in enumerate(CONS):
        v = G.field_view(G.cons, f)
        if k in HYDRO:
            v[gg:-gg, gg:-gg, gg:-gg].copy_(torch.from_numpy(np.ascontiguousarray(interior(s.U[k], gg))))
        else:
            v.copy_(torch.from_numpy(np.ascontiguousarray(s.U[k])))
    G.synchronize()


def _box(n=16, guess=None):
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g, d = box.turbulent_box(n)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, guess=L.GUESS_WARM if guess is None else guess)
    return g, s, G


def _perturb(s, seed=5):
    rng = np.random.default_rng(seed)
    gg = s.g
    for k in HYDRO:
        sl = s.U[k][gg:-gg, gg:-gg, gg:-gg]
        sl *= 1.0 + 1e-3 * rng.uniform(-1, 1, size=sl.shape)


def _zones_equal(a, b, names, tol):
    e = max_rel(a, b, names)
    assert max(e.values()) < tol, e


def _gidx(z, gg):
    return tuple(x + gg for x in z)


@gpu
def test_box_failure_injection_keeps_primitives_and_strict_mode():
    _torch()
    from paper_1810_04597_amd import _lib as L
    g, s, G = _box(16)
    _perturb(s)
    gg = s.g
    zD, zE = (3, 4, 5), (10, 2, 7)
    # zone D: negative total energy U = tau + D; zone E: |S| = 2 (tau + D)
    s.U["tau"][_gidx(zD, gg)] = -2.0 * s.U["D"][_gidx(zD, gg)]
    gE = _gidx(zE, gg)
    s.U["S1"][gE] = 2.0 * (s.U["tau"][gE] + s.U["D"][gE])
    _load_oracle_state(s, G)
    P0 = {k: interior(v, gg).copy() for k, v in s.P.items()}
    U0 = {k: interior(s.U[k], gg).copy() for k in HYDRO}
    G.reset_run_counters()
    st = s.cons2prim()
    nf = G.cons2prim()
    assert st["n_fail"] == 2 and nf == 2
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    P = {k: interior(v, gg) for k, v in s.P.items()}
    _zones_equal(gp, P, PRIM, 1e-12)
    for z in (zD, zE):
        # (the centred field is recomputed from the face fields in every zone)
        for k in ("rho", "u1", "u2", "u3", "p"):
            assert gp[k][z] == P0[k][z] == P[k][z], (z, k)
        for k in HYDRO:
            assert gc[k][z] == U0[k][z], (z, k)
    # every other zone's conserved variables are untouched without floors
    for k in HYDRO:
        assert np.array_equal(gc[k], U0[k]), k
    dg = G.diagnostics()
    assert dg["n_c2p_fail"] == 2 and dg["n_floor_rho"] == dg["n_floor_p"] == dg["n_wcap"] == 0
    assert dg["run_c2p_fail"] == 2
    # strict mode: the same failures are an error return
    with pytest.raises(L.GrmhdError) as ei:
        G.cons2prim(strict=True)
    assert ei.value.code == L.ENOCONV
    dg = G.diagnostics()
    assert dg["run_c2p_fail"] == 4 and dg["n_c2p_fail"] == 2
    G.reset_run_counters()
    assert G.diagnostics()["run_c2p_fail"] == 0
    G.close()


def _torus_pair(n1=32, n2=16, n3=16):
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(n1, n2, n3)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab)
    return g, tab, s, G


def _floors(g, s):
    r = s.r_int
    return g.rho_fl_a * r ** g.rho_fl_n, g.p_fl_a * r ** g.p_fl_n


@gpu
def test_torus_failure_floors_and_lorentz_cap_match_oracle():
    """32 x 16 x 16 torus: the atmosphere is lifted to 1.5 times the floors
    (so no zone meets a floor by round-off), then planted zones go below the
    density floor (A) and the pressure floor (B), one moves at W = 20 (C),
    and two fail (D: U < 0; E: |S| = 10 (tau + D))."""
    _torch()
    g, tab, s, G = _torus_pair()
    gg = s.g
    rfl, pfl = _floors(g, s)
    P = {k: interior(v, gg) for k, v in s.P.items()}
    rho = np.maximum(P["rho"], 1.5 * rfl)
    p = np.maximum(P["p"], 1.5 * pfl)
    zA, zB, zC, zD, zE = (2, 5, 9), (9, 7, 12), (4, 8, 11), (12, 6, 7), (6, 9, 14)
    rho[zA] = 0.5 * rfl[0, 0, zA[2]]
    p[zB] = 0.5 * pfl[0, 0, zB[2]]
    # W = 20 along x^3 (u^3 only: W^2 = 1 + gamma_33 (u^3)^2)
    from oracle.scheme import Metric
    g33 = Metric.interior(s.met.loc["C"], gg)["g33"][0, zC[1], zC[2]]
    u3 = P["u3"].copy()
    u1, u2 = P["u1"].copy(), P["u2"].copy()
    u1[zC] = u2[zC] = 0.0
    u3[zC] = math.sqrt((20.0 ** 2 - 1.0) / g33)
    for k, v in (("rho", rho), ("p", p), ("u1", u1), ("u2", u2), ("u3", u3)):
        s.set_interior(s.P[k], v)
    s.prim2cons()
    s.U["tau"][_gidx(zD, gg)] = -2.0 * s.U["D"][_gidx(zD, gg)]
    gE = _gidx(zE, gg)
    g11 = Metric.interior(s.met.loc["C"], gg)["g11"][0, zE[1], zE[2]]
    s.U["S1"][gE] = 10.0 * (s.U["tau"][gE] + s.U["D"][gE]) * math.sqrt(g11)
    _load_oracle_state(s, G)
    G.reset_run_counters()
    st = s.cons2prim()
    nf = G.cons2prim()
    assert st["n_fail"] == 2 and nf == 2, (st, nf)
    assert st["n_floor_rho"] >= 1 and st["n_floor_p"] >= 1 and st["n_wcap"] == 1, st
    dg = G.diagnostics()
    for key, okey in (("n_c2p_fail", "n_fail"), ("n_floor_rho", "n_floor_rho"),
                      ("n_floor_p", "n_floor_p"), ("n_wcap", "n_wcap")):
        assert dg[key] == st[okey], (key, dg[key], st[okey])
    assert (dg["run_c2p_fail"], dg["run_floor_rho"], dg["run_floor_p"], dg["run_wcap"]) == (
        st["n_fail"], st["n_floor_rho"], st["n_floor_p"], st["n_wcap"])
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    Po = {k: interior(v, gg) for k, v in s.P.items()}
    Uo = {k: interior(s.U[k], gg) for k in HYDRO}
    # velocities against the largest |u| (u^2 vanishes in the torus up to
    # round-off); p to 1e-11: in the capped zone (W = 20, cold) the pressure
    # is a difference of nearly equal terms, the inversion's own conditioning
    umax = max(float(np.max(np.abs(Po[k]))) for k in ("u1", "u2", "u3"))
    for k in ("u1", "u2", "u3"):
        assert np.max(np.abs(gp[k] - Po[k])) < 1e-12 * umax, k
    _zones_equal(gp, Po, ("rho", "B1", "B2", "B3"), 1e-12)
    _zones_equal(gp, Po, ("p",), 1e-11)
    _zones_equal({k: gc[k] for k in HYDRO}, Uo, HYDRO, 1e-12)
    # failed zones: atmosphere at rest; capped zone: W = 10
    for z in (zD, zE):
        assert abs(gp["rho"][z] / rfl[0, 0, z[2]] - 1) < 1e-14
        assert abs(gp["p"][z] / pfl[0, 0, z[2]] - 1) < 1e-14
        assert gp["u1"][z] == gp["u2"][z] == gp["u3"][z] == 0.0
        assert gc["S1"][z] == gc["S2"][z] == gc["S3"][z] == 0.0
    assert abs(gp["rho"][zA] / rfl[0, 0, zA[2]] - 1) < 1e-14
    assert abs(gp["p"][zB] / pfl[0, 0, zB[2]] - 1) < 1e-14
    w = math.sqrt(1.0 + g33 * gp["u3"][zC] ** 2 + 0.0)
    assert abs(w - 10.0) < 1e-9, w
    G.close()


@gpu
def test_cold_guess_grid_matches_oracle():
    """A grid built with the cold guess (y0 = Gamma U) against the oracle's
    cold-guess inversion of the same perturbed 16^3 state."""
    _torch()
    from paper_1810_04597_amd import _lib as L
    g, s, G = _box(16, guess=L.GUESS_COLD)
    _perturb(s, seed=7)
    _load_oracle_state(s, G)
    st = s.cons2prim(guess="cold")
    nf = G.cons2prim()
    assert nf == st["n_fail"] == 0
    gg = s.g
    _zones_equal(G.to_numpy("prim", interior=True), {k: interior(v, gg) for k, v in s.P.items()},
                 PRIM, 1e-12)
    dg = G.diagnostics()
    n = 16 ** 3
    # the cold start needs several more iterations than the warm one
    assert dg["newton_iters_sum"] > 2 * n
    assert abs(dg["newton_iters_sum"] - st["iters_sum"]) <= 0.02 * n, (dg["newton_iters_sum"], st["iters_sum"])
    assert abs(dg["newton_iters_max"] - st["iters_max"]) <= 1
    G.close()


@gpu
@pytest.mark.parametrize("guess", ["warm", "cold"])
def test_newton_iterations_per_zone(guess):
    """Per-zone Newton iteration counts of the perturbed 16^3 state: the
    batched point inversion (the grid inversion's Newton, flat frame) against
    the oracle's Newton from the same guesses; the grid's totals against the
    oracle's."""
    torch = _torch()
    from oracle.c2p import newton, warm_guess
    from oracle.scheme import Metric
    g, s, G = _box(16)
    _perturb(s, seed=9)
    _load_oracle_state(s, G)
    gg = s.g
    m = Metric.interior(s.met.loc["C"], gg)
    P = {k: interior(v, gg) for k, v in s.P.items()}
    U = {k: interior(s.U[k], gg) for k in HYDRO}
    b = s.centred_b()
    if guess == "warm":
        y0 = warm_guess(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"], m, s.gam)
    else:
        y0 = s.gam * (U["tau"] + U["D"])
    res = newton(U["D"], (U["S1"], U["S2"], U["S3"]), U["tau"], b, m, s.gam, y0)
    rows = np.stack([U["D"], U["S1"], U["S2"], U["S3"], U["tau"], b[0], b[1], b[2]], axis=-1).reshape(-1, 8)
    cons = torch.from_numpy(np.ascontiguousarray(rows)).to(G.device)
    y0t = torch.from_numpy(np.array(np.broadcast_to(y0, U["D"].shape).reshape(-1))).to(G.device)
    prim, it = G.cons2prim_points(cons, y0t)
    it = it.cpu().numpy()
    ito = res["iters"].reshape(-1)
    assert np.all(it > 0) and np.all(res["ok"])
    diff = np.abs(it - ito)
    assert diff.max() <= 1, diff.max()
    frac = float((diff == 0).mean())
    print("Newton iterations (%s): equal in %.4f of %d zones; sums %d vs %d" % (
        guess, frac, it.size, int(it.sum()), int(ito.sum())))
    assert frac >= 0.95
    pr = prim.cpu().numpy()
    for q, k in enumerate(("rho", "u1", "u2", "u3", "p")):
        ref = res[k].reshape(-1) if k in ("rho", "p") else res["u"][q - 1].reshape(-1)
        scale = np.abs(ref) if k in ("rho", "p") else np.max(np.abs(ref))
        assert np.max(np.abs(pr[:, q] - ref) / scale) < 1e-12, k
    if guess == "warm":
        # the grid inversion from the same warm start: totals within the
        # zones whose counts may differ
        st = s.cons2prim()
        G.cons2prim()
        dg = G.diagnostics()
        nd = int((diff != 0).sum())
        assert abs(dg["newton_iters_sum"] - st["iters_sum"]) <= max(nd, 0.02 * it.size)
        assert abs(dg["newton_iters_max"] - st["iters_max"]) <= 1
    G.close()


def _diag_close(dg, do, U_abs_sums, exact_extrema=True):
    names = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")
    for q, k in enumerate(names):
        assert abs(dg["sum_cons"][q] - do["sum_" + k]) <= 1e-13 * U_abs_sums[k], (k, dg["sum_cons"][q], do["sum_" + k])
    for k in ("rho_min", "rho_max", "p_min", "p_max"):
        if exact_extrema:
            assert dg[k] == do[k], (k, dg[k], do[k])
        else:
            assert abs(dg[k] - do[k]) <= 1e-10 * abs(do[k]), (k, dg[k], do[k])
    assert abs(dg["w_max"] - do["w_max"]) <= 1e-14 * do["w_max"]
    assert dg["n_nonfinite"] == do["n_nonfinite"]


def _abs_sums(s):
    return {k: float(np.sum(np.abs(interior(s.U[k], s.g)))) for k in CONS}


@gpu
def test_diagnostics_match_oracle_box():
    """16^3 box: the same state on both sides after init and after three RK3
    steps of the oracle (sums to 1e-13 of sum |U|, extrema exactly, the
    Lorentz factor to rounding); the GPU's own three steps within the step
    parity bar; a planted divergence (random face fields) to 1e-12."""
    _torch()
    g, s, G = _box(16)
    _load_oracle_state(s, G)
    _diag_close(G.diagnostics(), s.diagnostics(), _abs_sums(s))
    for _ in range(3):
        dt = s.cfl_dt()
        s.rk_step(dt)
        G.rk_step(dt)
    # GPU evolved independently: within the parity bar of the steps
    dgo = s.diagnostics()
    _diag_close(G.diagnostics(), dgo, _abs_sums(s), exact_extrema=False)
    assert G.diagnostics()["max_divb"] <= 1e-12 and dgo["max_divb"] <= 1e-12
    # the oracle's stepped state loaded into the GPU: the same numbers
    _load_oracle_state(s, G)
    dg = G.diagnostics()
    _diag_close(dg, dgo, _abs_sums(s))
    # planted divergence: random face fields (seeded), same on both sides
    rng = np.random.default_rng(31)
    from oracle.boundary import fill_faces
    for k in ("Bf1", "Bf2", "Bf3"):
        s.U[k] = rng.normal(scale=0.1, size=s.U[k].shape)
    fill_faces(s.U, g)
    s.prim2cons()
    _load_oracle_state(s, G)
    dg, do = G.diagnostics(), s.diagnostics()
    assert do["max_divb"] > 1.0
    assert abs(dg["max_divb"] / do["max_divb"] - 1) < 1e-12, (dg["max_divb"], do["max_divb"])
    assert abs(dg["max_divb_norm"] / do["max_divb_norm"] - 1) < 1e-12
    _diag_close(dg, do, _abs_sums(s))
    # non-finite primitives: counted (two planted)
    import torch
    gg = s.g
    s.P["rho"][gg + 2, gg + 3, gg + 4] = np.nan
    s.P["u2"][gg + 5, gg + 1, gg + 0] = np.inf
    G.field_view(G.prim, 0)[gg + 2, gg + 3, gg + 4] = float("nan")
    G.field_view(G.prim, 2)[gg + 5, gg + 1, gg + 0] = float("inf")
    G.synchronize()
    dg, do = G.diagnostics(), s.diagnostics()
    assert dg["n_nonfinite"] == do["n_nonfinite"] == 2
    assert dg["rho_min"] == do["rho_min"] and dg["rho_max"] == do["rho_max"]
    G.close()


@gpu
def test_diagnostics_match_oracle_torus():
    """32 x 16 x 16 Kerr-Schild torus: initial state and after two RK3 steps
    of the oracle, loaded into the GPU grid; the Lorentz factor with the
    metric, sums, extrema, div B.  The accumulated counters of the GPU's own
    two steps against the sums of the oracle's per-stage counts: on this
    coarse grid at the CFL step a few hundred atmosphere zones near the inner
    boundary fail per step and are reset, and hundreds more meet a floor or
    the W cap; which zones do is decided at round-off (the state there is
    ill-conditioned), so the totals agree to a few percent, not exactly."""
    _torch()
    g, tab, s, G = _torus_pair()
    _load_oracle_state(s, G)
    _diag_close(G.diagnostics(), s.diagnostics(), _abs_sums(s))
    G.reset_run_counters()
    tot = {"n_fail": 0, "n_floor_rho": 0, "n_floor_p": 0, "n_wcap": 0}
    for _ in range(2):
        dt = s.cfl_dt()
        s.rk_step(dt)
        G.rk_step(dt)
        for stt in s.last_stage_stats:
            for k in tot:
                tot[k] += stt[k]
    dg = G.diagnostics()
    run = {"n_fail": dg["run_c2p_fail"], "n_floor_rho": dg["run_floor_rho"],
           "n_floor_p": dg["run_floor_p"], "n_wcap": dg["run_wcap"]}
    print("torus 32x16x16, 2 steps: accumulated counters gpu %s oracle %s" % (run, tot))
    for k in tot:
        assert abs(run[k] - tot[k]) <= max(5, 0.03 * tot[k]), (k, run[k], tot[k])
    assert tot["n_floor_rho"] > 0 and tot["n_floor_p"] > 0 and tot["n_fail"] > 0
    _load_oracle_state(s, G)
    dg, do = G.diagnostics(), s.diagnostics()
    _diag_close(dg, do, _abs_sums(s))
    # a field kept divergence-free by the update, next to the boundaries too
    # (round-off against the face fields' differences), and the same value on
    # both sides up to the round-off of the divergence sum itself
    bscale = max(float(np.max(np.abs(interior(s.U[k], s.g)))) / s.grid.dx[a]
                 for a, k in enumerate(("Bf1", "Bf2", "Bf3")))
    assert do["max_divb"] <= 1e-13 * bscale, (do["max_divb"], bscale)
    assert abs(dg["max_divb"] - do["max_divb"]) <= 1e-6 * do["max_divb"] + 1e-14 * bscale, \
        (dg["max_divb"], do["max_divb"], bscale)
    G.close()
