"""Split inversion (Newton load balance): a first pass of at most K
iterations per zone, the zones not converged by then finished in a second,
compact pass from the iterate they stopped at.  The roots are those of the
one-pass inversion, so the results match the oracle and the one-pass GPU
inversion to the FP64 bars; counters and the device CFL step stay right when
the split is switched on and off."""
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


def _box_pair(n, split):
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(n)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g)
    G.set_newton_split(split)
    G.curl_potential(d)
    G.set_primitives(d)
    return g, d, s, G


@gpu
@pytest.mark.parametrize("split", [1, 2])
def test_box_ten_steps_split_matches_oracle(split):
    """32^3 box, ten steps with the device CFL step: with K = 1 nearly every
    zone goes through the second pass; every zone and field within 1e-10 of
    the oracle, the device dt within 1e-11, no failed inversion."""
    _torch()
    g, d, s, G = _box_pair(32, split)
    G.set_profiling(True)
    for _ in range(10):
        dt_o = s.cfl_dt()
        dt_g = G.rk_step(0.0, want_dt=True)
        assert abs(dt_g / dt_o - 1) < 1e-11
        s.rk_step(dt_o)
    prof = G.profile()
    assert prof["newton_split"][1] == 30   # one second pass per stage
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e
    dg = G.diagnostics()
    assert dg["n_c2p_fail"] == 0 and dg["max_divb"] <= 1e-12
    G.close()


@gpu
def test_split_equals_one_pass_inversion():
    """Torus grid with a poor warm start (stored primitives replaced by a
    uniform state, so many zones need many iterations), inverted one-pass and
    split (K = 1, 2, 3): the same roots to 1e-12, the same failure count and
    floors."""
    _torch()
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24)
    res = {}
    for k in (0, 1, 2, 3):
        G = Grid(g, tables=tab)
        G.set_newton_split(k)
        G.curl_potential(d)
        G.set_primitives(d)
        # a poor warm start: stored primitives replaced by a uniform state
        for f, val in ((0, 1.0), (1, 0.0), (2, 0.0), (3, 0.0), (4, 1.0)):
            G._interior(G.field_view(G.prim, f)).fill_(val)
        nf = G.cons2prim()
        res[k] = (G.to_numpy("prim", interior=True), G.diagnostics(), nf)
        G.close()
    p0, d0, nf0 = res[0]
    for k in (1, 2, 3):
        pk, dk, nfk = res[k]
        assert nfk == nf0
        e = max_rel(pk, p0, ("rho", "p", "u1", "u3"))
        e["u2"] = float(np.max(np.abs(pk["u2"] - p0["u2"])))
        assert max(e.values()) < 1e-12, (k, e)
        assert dk["n_floor_rho"] == d0["n_floor_rho"] and dk["n_floor_p"] == d0["n_floor_p"]
        print("split K=%d: iterations %d (one pass %d), max %d (one pass %d)" % (
            k, dk["newton_iters_sum"], d0["newton_iters_sum"], dk["newton_iters_max"],
            d0["newton_iters_max"]))


@gpu
def test_torus_one_step_split_matches_oracle():
    """Torus 48x24x24 with floors, one RK3 step with the oracle's CFL step and
    K = 2: every zone and field within 1e-10."""
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab)
    G.set_newton_split(2)
    G.curl_potential(d)
    G.set_primitives(d)
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    P = {k: interior(v) for k, v in s.P.items()}
    U = {k: interior(v) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e
    G.close()


@gpu
def test_split_switched_on_and_off():
    """Counters after switching the split off match those of a grid that
    never used it (the second pass's counter slots are cleared: stale slots
    would add a whole pass's iterations), and the device CFL step follows
    the state.  The two states differ by rounding after the first step, so
    iteration counts may differ by a few."""
    _torch()
    g, d, s, G = _box_pair(16, 1)
    G.rk_step()
    G.set_newton_split(0)
    G.rk_step()
    da = G.diagnostics()
    _, _, _, H = _box_pair(16, 0)
    H.rk_step()
    H.rk_step()
    db = H.diagnostics()
    for k in ("n_c2p_fail", "n_floor_rho", "n_floor_p"):
        assert da[k] == db[k], k
    assert abs(da["newton_iters_max"] - db["newton_iters_max"]) <= 1
    assert abs(da["newton_iters_sum"] - db["newton_iters_sum"]) <= 1e-3 * db["newton_iters_sum"]
    assert abs(da["t"] / db["t"] - 1) < 1e-12
    G.close()
    H.close()


@gpu
def test_split_argument_checks():
    _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g, _ = box.turbulent_box(8)
    G = Grid(g)
    for bad in (-1, g.newton_maxit, 1000):
        with pytest.raises(L.GrmhdError):
            G.set_newton_split(bad)
    G.set_newton_split(g.newton_maxit - 1)
    G.set_newton_split(0)
    G.close()
    H = Grid(g, guess=L.GUESS_MLP)
    with pytest.raises(L.GrmhdError):
        H.set_newton_split(2)
    H.set_newton_split(0)
    H.close()
