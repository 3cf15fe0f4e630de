"""GPU parity of the lower-order fallback (grmhd_grid_desc.fallback = 1)
with the oracle's Solver(fallback=True), through the C ABI.

  * the Kerr-Schild torus (48 x 24 x 24) at its CFL step, where the
    high-order update leaves unphysical states in the first stage: the same
    troubled zones on both sides, every zone and field within 1e-10 of the
    oracle, no failed inversion (WENO5, MP5, MP7 on six ghost layers, PLM;
    sixth- and fourth-order derivatives, the latter also on four layers);
  * the blast (pressure jump 3e4, unmagnetised) on a flat periodic box
    (the x^3-marching update with its flags; 16^3 writes the ghost images in
    the update, 16 x 16 x 8 fills ghosts separately): the same troubled
    zones, no failed inversion, every zone and field within 1e-10.  (With a
    field, b0 = 0.1, failed inversions remain after the fallback: states
    whose hydro part is admissible but which no primitives give with that
    field, which the criterion does not test; their failure decisions sit at
    round-off, so that case is no parity case.)
  * the same blast centred on the box corner, so that troubled zones sit on
    both sides of every periodic boundary (faces written at their periodic
    images): parity with the oracle, and the centred run rolled by half the
    box bit for bit;
  * where nothing is troubled (the turbulent box) the option changes no bit
    of the state, eager and graph-replayed, FP64 and FP32 forms;
  * with troubled zones in every step (the blast, the torus), steps replayed
    from a captured graph equal eager steps bit for bit.
"""
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


def _compare(s, G, tol):
    P = {k: interior(v, s.g) for k, v in s.P.items()}
    U = {k: interior(v, s.g) for k, v in s.U.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < tol, e


@gpu
@pytest.mark.parametrize("recon,order,ng", [("weno5", 6, 5), ("mp5", 6, 5), ("weno5", 4, 5), ("mp7", 6, 6),
                                            ("plm", 6, 5), ("mp5", 4, 4)])
def test_torus_cfl_step_matches_oracle(recon, order, ng):
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24, ng=ng)
    s = Solver(g, tab, recon=recon, deriv_order=order, fallback=True)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab, recon=recon, deriv_order=order, fallback=True)
    G.curl_potential(d)
    G.set_primitives(d)
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    dg = G.diagnostics()
    print("%s D%d: troubled oracle %d gpu %d; failed inversions oracle %s gpu %d"
          % (recon, order, s.n_troubled, dg["run_troubled"],
             [x["n_fail"] for x in s.last_stage_stats], dg["run_c2p_fail"]))
    assert s.n_troubled > 0
    assert dg["run_troubled"] == s.n_troubled
    assert sum(x["n_fail"] for x in s.last_stage_stats) == 0
    assert dg["run_c2p_fail"] == 0
    _compare(s, G, 1e-10)


@gpu
def test_torus_fp32_form_with_fallback():
    """FP32 form (fluxes from float32 face physics): against the oracle's
    float32 form with the fallback, the same troubled zones up to decisions
    at float32 rounding, no failed inversion, and the float32 difference
    level (the oracle's own FP32-vs-FP64 difference here: rho 3e-6, u 5e-6,
    p 4e-4 in the cold atmosphere)."""
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24)
    s = Solver(g, tab, recon="weno5", precision="fp32", fallback=True)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab, recon="weno5", precision=1, fallback=True)
    G.curl_potential(d)
    G.set_primitives(d)
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    dg = G.diagnostics()
    print("fp32 form: troubled oracle %d gpu %d, failed gpu %d" % (s.n_troubled, dg["run_troubled"],
                                                                 dg["run_c2p_fail"]))
    assert dg["run_c2p_fail"] == 0
    assert abs(dg["run_troubled"] - s.n_troubled) <= 0.01 * s.n_troubled
    P = {k: interior(v, s.g) for k, v in s.P.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    print("fp32 form vs oracle fp32 form:", e)
    assert max(e[k] for k in PRIM if k != "p") < 1e-4, e
    assert e["p"] < 5e-3, e


@gpu
def test_torus_without_fallback_fails_where_it_does_not():
    """The same step without the option: the GPU leaves failed inversions."""
    _torch()
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    g, d, tab = torus(48, 24, 24)
    out = {}
    for fb in (False, True):
        G = Grid(g, tables=tab, recon="weno5", fallback=fb)
        G.curl_potential(d)
        G.set_primitives(d)
        G.rk_step(G.compute_dt())
        dg = G.diagnostics()
        out[fb] = (dg["run_c2p_fail"], dg["run_troubled"])
    assert out[False][0] > 0 and out[False][1] == 0
    assert out[True][0] == 0 and out[True][1] > 0, out


@gpu
@pytest.mark.parametrize("n", [16, (16, 16, 8)])
@pytest.mark.parametrize("recon", ["mp5", "weno5"])
def test_blast_box_matches_oracle(n, recon):
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d = box.blast_box(n, b0=0.0)
    s = Solver(g, recon=recon, fallback=True)
    s.set_face_fields(d)
    s.set_primitives(d)
    G = Grid(g, recon=recon, fallback=True)
    G.set_face_fields(d)
    G.set_primitives(d)
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    dg = G.diagnostics()
    print("blast %s %s: troubled oracle %d gpu %d; failed oracle %s gpu %d"
          % (n, recon, s.n_troubled, dg["run_troubled"],
             [x["n_fail"] for x in s.last_stage_stats], dg["run_c2p_fail"]))
    assert s.n_troubled > 0
    assert dg["run_troubled"] == s.n_troubled
    assert sum(x["n_fail"] for x in s.last_stage_stats) == 0
    assert dg["run_c2p_fail"] == 0
    _compare(s, G, 1e-10)


@gpu
@pytest.mark.parametrize("n", [16, (16, 16, 8)])
def test_blast_on_the_corner(n):
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    got = {}
    for name, c in (("centre", (0.5, 0.5, 0.5)), ("corner", (0.0, 0.0, 0.0))):
        g, d = box.blast_box(n, b0=0.0, centre=c)
        G = Grid(g, recon="mp5", fallback=True)
        G.set_face_fields(d)
        G.set_primitives(d)
        G.rk_step(2.0e-3)
        got[name] = (G.to_numpy("cons", interior=True), G.diagnostics()["run_troubled"])
        if name == "corner":
            s = Solver(g, recon="mp5", fallback=True)
            s.set_face_fields(d)
            s.set_primitives(d)
            s.rk_step(2.0e-3)
            assert got[name][1] == s.n_troubled > 0
            _compare(s, G, 1e-10)
        G.close()
    nn = (n, n, n) if np.isscalar(n) else n
    shift = (nn[2] // 2, nn[1] // 2, nn[0] // 2)
    for k in CONS:
        rolled = np.roll(got["centre"][0][k], shift, axis=(0, 1, 2))
        assert np.array_equal(got["corner"][0][k], rolled), k


@gpu
@pytest.mark.parametrize("precision,order", [(0, 6), (1, 6), (0, 4)])
def test_option_changes_nothing_without_troubled_zones(precision, order):
    torch = _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(24)
    out = {}
    for fb in (False, True):
        G = Grid(g, precision=precision, deriv_order=order, fallback=fb, stream=torch.cuda.Stream())
        G.curl_potential(d)
        G.set_primitives(d)
        for _ in range(2):
            G.rk_step()
        G.rk_steps_graph(3)
        out[fb] = (G.to_numpy("cons"), G.to_numpy("prim"), G.diagnostics())
    assert out[True][2]["run_troubled"] == 0
    for a in range(2):
        for k in out[False][a]:
            assert np.array_equal(out[False][a][k], out[True][a][k]), k


@gpu
@pytest.mark.parametrize("case", ["blast", "torus"])
def test_fallback_in_graph_replays_equals_eager(case):
    """With troubled zones in every step: device-dt steps replayed from a
    captured graph equal eager steps bit for bit (the troubled-zone list is
    filled in whatever order the atomics give, but each face value is formed
    once and each zone gathers its own), every replay checked, with eager
    work and synchronisations between the replays; the counters agree."""
    torch = _torch()
    from paper_1810_04597_amd.grid import Grid
    if case == "blast":
        from workloads import box
        g, d = box.blast_box(16, b0=0.0)
        kw = dict(recon="mp5")
    else:
        from workloads.torus import torus
        g, d, tab = torus(48, 24, 24)
        kw = dict(tables=tab, recon="weno5")
    grids = []
    for _ in range(2):
        G = Grid(g, fallback=True, stream=torch.cuda.Stream(), **kw)
        if case == "blast":
            G.set_face_fields(d)
        else:
            G.curl_potential(d)
        G.set_primitives(d)
        grids.append(G)
    Ge, Gg = grids
    troubled = []
    for rep in range(4):        # the first graph call steps eagerly, then capture and replays
        Ge.rk_step(0.0)
        Gg.rk_steps_graph(1)
        Gg.synchronize()
        de, dg = Ge.diagnostics(), Gg.diagnostics()
        troubled.append(de["run_troubled"])
        assert de["run_troubled"] == dg["run_troubled"], rep
        ce, cg = Ge.to_numpy("cons"), Gg.to_numpy("cons")
        for k in ce:
            assert np.array_equal(ce[k], cg[k], equal_nan=True), (rep, k)
    print("%s: accumulated troubled zones per step" % case, troubled)
    assert troubled[0] > 0 and troubled[3] > troubled[0], troubled   # also during the replays
    for G in grids:
        G.close()
