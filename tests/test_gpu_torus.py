"""GPU parity in curved spacetime (Kerr-Schild a = 0.9 torus) and the
reduction of the table-driven path to the flat path."""
import numpy as np
import pytest

from helpers import max_rel, interior

gpu = pytest.mark.gpu
PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _pair_torus(n1, n2, n3):
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(n1, n2, n3)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab)
    G.curl_potential(d)
    G.set_primitives(d)
    return g, d, tab, s, G


@gpu
def test_table_path_with_flat_tables_equals_flat_path():
    _torch()
    from workloads import box
    from workloads.metric import minkowski_tables
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(16)
    A = Grid(g)
    B = Grid(g, tables=minkowski_tables(g))
    for G in (A, B):
        G.curl_potential(d)
        G.set_primitives(d)
        for _ in range(3):
            G.rk_step(2e-3)
    a = A.to_numpy("cons", interior=True)
    b = B.to_numpy("cons", interior=True)
    e = max_rel(a, b, CONS)
    assert max(e.values()) < 1e-13, e


@gpu
def test_torus_init_and_rhs_match_oracle():
    _torch()
    g, d, tab, s, G = _pair_torus(32, 16, 16)
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-12, e
    L_o = s.rhs()
    L_g = G.read_group(G.rhs(), CONS, interior=True)
    errs = {k: float(np.max(np.abs(L_g[k] - L_o[k])) / np.max(np.abs(L_o[k]))) for k in CONS}
    assert max(errs.values()) < 1e-11, errs


@gpu
def test_torus_one_step_parity_all_zones():
    """Torus 48x24x24, one RK3 step with the oracle's CFL step: every zone
    and field within 1e-10 relative."""
    _torch()
    g, d, tab, s, G = _pair_torus(48, 24, 24)
    dt = s.cfl_dt()
    assert abs(G.compute_dt() / dt - 1) < 1e-12
    s.rk_step(dt)
    G.rk_step(dt)
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e


@gpu
@pytest.mark.parametrize("n,fixed_dt", [((48, 24, 24), 0.02), ((64, 32, 32), None)])
def test_torus_ten_steps_within_oracle_envelope(n, fixed_dt):
    """10 RK3 steps of the torus (48 x 24 x 24 at dt = 0.02; 64 x 32 x 32 at
    the oracle's CFL step of each step).  The magnetised, floored atmosphere
    makes this run ill-conditioned: the oracle itself moves by up to O(1) in
    near-floor zones (and ~1e-3 in the torus body) when its initial density
    is perturbed by 1e-14.  The GPU result must be as close to the oracle as
    the oracle is to itself: per field, the 99th percentile of
    |GPU - oracle| is at most 10 times the 99th percentile of
    |oracle(1e-14) - oracle| (plus 1e-10 of the field scale), and the torus
    body (rho > 0.05) agrees within 1e-2 of the field scale."""
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    g, d, tab, s, G = _pair_torus(*n)
    dp = dict(d)
    dp["rho"] = d["rho"] * (1.0 + 1e-14)
    s2 = Solver(g, tab)
    s2.curl_potential(dp)
    s2.set_primitives(dp)
    for _ in range(10):
        dt = fixed_dt if fixed_dt else s.cfl_dt()
        s.rk_step(dt)
        s2.rk_step(dt)
        G.rk_step(dt)
    gp = G.to_numpy("prim", interior=True)
    body = interior(s.P["rho"]) > 0.05
    report = {}
    for k in PRIM:
        ref = interior(s.P[k])
        scale = np.max(np.abs(ref))
        env = np.percentile(np.abs(interior(s2.P[k]) - ref), 99)
        diff = np.abs(gp[k] - ref)
        q = np.percentile(diff, 99)
        report[k] = (q / scale, env / scale, float(np.max(diff[body]) / scale))
        assert q <= 10.0 * env + 1e-10 * scale, (k, report[k])
        assert np.max(diff[body]) < 1e-2 * scale, (k, report[k])
        if fixed_dt is None:
            # at the CFL step this grid stays well conditioned: the FP64 bar
            # holds at every zone
            assert np.max(diff) < 1e-10 * scale, (k, float(np.max(diff) / scale))
    print("torus envelope report (gpu q99, oracle q99, body max):", report)
    assert G.diagnostics()["n_nonfinite"] == 0


def _shell_close(gs, os_):
    for a, scale in (("F_D", "scale_D"), ("F_tau", "scale_tau"), ("Phi", "scale_B"), ("Phi_s", "scale_B")):
        err = np.abs(gs[a] - os_[a]) / np.maximum(os_[scale], 1e-300)
        assert err.max() < 1e-12, (a, err.max())


@gpu
def test_shell_fluxes_match_oracle():
    """Fluxes through the x^1 = const shells (accretion rate, energy and
    magnetic flux) on the 32 x 16 x 16 torus, initially and after one step:
    every shell within 1e-12 of the sum of |terms|."""
    _torch()
    from oracle.diagnostics import shell_fluxes
    g, d, tab, s, G = _pair_torus(32, 16, 16)
    _shell_close(G.shell_fluxes(), shell_fluxes(s))
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    _shell_close(G.shell_fluxes(), shell_fluxes(s))


@gpu
def test_shell_fluxes_full_size_torus():
    """The same diagnostic on the full 256 x 128 x 128 torus (initial state;
    the oracle evaluates the pointwise fluxes of the whole grid)."""
    _torch()
    from oracle.diagnostics import shell_fluxes
    g, d, tab, s, G = _pair_torus(256, 128, 128)
    _shell_close(G.shell_fluxes(), shell_fluxes(s))
    G.close()


def _mri_close(gm, om, q_min):
    """Shell sums within 1e-12 of their size; threshold counts equal except
    for zones whose Q lies within rounding of q_min."""
    for a in ("wQ2", "wQ3", "w"):
        err = np.abs(gm[a] - om[a]) / np.maximum(np.abs(om[a]), 1e-300)
        assert err.max() < 1e-12, (a, err.max())
    assert np.array_equal(gm["n_body"], om["n_body"])
    for a, q in (("n_Q2_ok", "Q2"), ("n_Q3_ok", "Q3")):
        near = (np.abs(om[q] - q_min) <= 1e-10 * q_min).sum(axis=(0, 1))
        assert np.all(np.abs(gm[a] - om[a]) <= near), a


@gpu
@pytest.mark.parametrize("steps", [0, 1])
def test_mri_quality_matches_oracle(steps):
    """MRI resolution sums of the 48x24x24 torus (body rho > 1e-2), at the
    initial state and after one RK3 step."""
    _torch()
    from oracle.diagnostics import mri_quality
    g, d, tab, s, G = _pair_torus(48, 24, 24)
    if steps:
        dt = s.cfl_dt()
        s.rk_step(dt)
        G.rk_step(dt)
    om = mri_quality(s, 1e-2, 8.0)
    gm = G.mri_quality(1e-2, 8.0)
    _mri_close(gm, om, 8.0)
    assert gm["n_body"].sum() > 0 and gm["wQ3"].sum() > 0


@gpu
def test_mri_quality_full_size_torus():
    """The 256 x 128 x 128 torus (the benchmark's size): shell sums against
    the oracle on the whole initial grid."""
    _torch()
    from oracle.diagnostics import mri_quality
    g, d, tab, s, G = _pair_torus(256, 128, 128)
    om = mri_quality(s, 1e-2, 8.0)
    gm = G.mri_quality(1e-2, 8.0)
    _mri_close(gm, om, 8.0)
    print("torus 256x128x128 MRI: <Q2> %.2f <Q3> %.2f, Q2 >= 8 in %.3f, Q3 >= 8 in %.3f of %d body zones"
          % (gm["Q2_mean"], gm["Q3_mean"], gm["frac_Q2_ok"], gm["frac_Q3_ok"], int(gm["n_body"].sum())))
    G.close()


def _load_state(s, G):
    """Oracle state -> GPU grid: primitives (ghosted), interior hydro
    conserved variables, face fields (ghosted)."""
    import torch
    gg = s.g
    for f, k in enumerate(PRIM):
        G.field_view(G.prim, f).copy_(torch.from_numpy(np.ascontiguousarray(s.P[k])))
    for f, k in enumerate(CONS):
        v = G.field_view(G.cons, f)
        if f < 5:
            v[gg:-gg, gg:-gg, gg:-gg].copy_(torch.from_numpy(np.ascontiguousarray(interior(s.U[k], gg))))
        else:
            v.copy_(torch.from_numpy(np.ascontiguousarray(s.U[k])))
    G.synchronize()


@gpu
@pytest.mark.parametrize("order", [6, 4])
def test_planted_divergence_keeps_its_value_next_to_every_boundary(order):
    """A seeded divergence planted in the torus face fields (owned faces and
    the evolved ghost faces normal to the radial and polar-axis boundaries):
    over a step the GPU carries it unchanged in every interior cell, the
    cells beside the boundaries included (ghost faces evolved with the
    induction equation, zero edge field on the axis), and matches the
    oracle's state within 1e-10."""
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver, FACE
    from oracle.boundary import fill_faces
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24)
    s = Solver(g, tab, deriv_order=order)
    s.curl_potential(d)
    s.set_primitives(d)
    rng = np.random.default_rng(41)
    scale = max(float(np.nanmax(np.abs(s.U[k]))) for k in FACE)
    for nd, k in enumerate(FACE):
        reg = s.face_region(nd)
        s.U[k][reg] += 1e-6 * scale * rng.normal(size=s.U[k][reg].shape)
    fill_faces(s.U, g, s.flo)
    s.prim2cons()
    d0 = s.div_b().copy()
    G = Grid(g, tables=tab, deriv_order=order)
    G.curl_potential(d)
    G.set_primitives(d)
    _load_state(s, G)
    s.rk_step(2e-3)
    G.rk_step(2e-3)
    probe = Solver(g, tab, deriv_order=order)
    cg = G.to_numpy("cons")
    for k in FACE:
        probe.U[k] = cg[k]
    d1 = probe.div_b()
    err = np.abs(d1 - d0)
    edge = np.zeros(d0.shape, dtype=bool)
    edge[:, :3, :] = edge[:, -3:, :] = True
    edge[:, :, :3] = edge[:, :, -3:] = True
    print("planted div B %.3e; change over a step: all %.3e, beside the boundaries %.3e"
          % (np.max(np.abs(d0)), err.max(), err[edge].max()))
    assert err.max() < 1e-9 * np.max(np.abs(d0))
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e
    G.close()


@gpu
def test_planted_divergence_on_an_outflow_box():
    """The same on a box with outflow in all three directions (x^3 boundary
    faces included): the GPU carries the planted divergence unchanged over a
    step and matches the oracle within 1e-10."""
    _torch()
    from dataclasses import replace
    from workloads import box
    from oracle.scheme import Solver, FACE
    from oracle.boundary import fill_faces
    from paper_1810_04597_amd.grid import Grid
    g0, d = box.turbulent_box(20)
    g = replace(g0, bc=(1,) * 6)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    rng = np.random.default_rng(43)
    for nd, k in enumerate(FACE):
        reg = s.face_region(nd)
        s.U[k][reg] += 1e-6 * rng.normal(size=s.U[k][reg].shape)
    fill_faces(s.U, g, s.flo)
    s.prim2cons()
    d0 = s.div_b().copy()
    G = Grid(g)
    G.curl_potential(d)
    G.set_primitives(d)
    _load_state(s, G)
    s.rk_step(2e-3)
    G.rk_step(2e-3)
    probe = Solver(g)
    cg = G.to_numpy("cons")
    for k in FACE:
        probe.U[k] = cg[k]
    err = np.max(np.abs(probe.div_b() - d0))
    assert err < 1e-9 * np.max(np.abs(d0)), (err, np.max(np.abs(d0)))
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e
    G.close()
