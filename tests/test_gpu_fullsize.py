"""Parity at the full workload sizes, in the launch shapes the benchmark uses.

The oracle cannot step these grids whole.  One SSP-RK3 step moves
information a bounded distance (tests/windows.py), so the oracle steps a
sub-box cut out of the same seeded initial data, with a margin of
windows.MARGIN zones, and the GPU's full-grid step is compared with the
oracle at the window's centre, zone by zone and field by field.  The
oracle can still set up the whole grid and reduce its CFL step (seconds), so
the GPU steps with its device CFL step, as benchmarked, and that step is
compared with the oracle's; the windows step with the oracle's value.
Properties that hold at any size (conservation on the periodic box, div B,
determinism) are checked on the whole grid.
"""
import numpy as np
import pytest

from windows import MARGIN, window_spec, window_data

gpu = pytest.mark.gpu
PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")
W = 4   # compared zones per axis at each window centre


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _gpu_block(G, which, idx):
    """Interior values of G at the outer product of index arrays (x1, x2, x3)."""
    import torch
    flat = G.prim if which == "prim" else G.cons
    names = PRIM if which == "prim" else CONS
    ti = [torch.as_tensor(np.asarray(a), dtype=torch.long, device=G.device) for a in idx]
    out = {}
    for f, name in enumerate(names):
        v = G._interior(G.field_view(flat, f))
        v = v.index_select(0, ti[2]).index_select(1, ti[1]).index_select(2, ti[0])
        out[name] = v.cpu().numpy().copy()
    return out


def _oracle_window(g, d, origin, size, bc, wrap, tables_fn=None, precision="fp64"):
    from oracle.scheme import Solver
    gw = window_spec(g, origin, size, bc)
    dw = window_data(g, d, origin, size, wrap)
    s = Solver(gw, tables_fn(gw) if tables_fn else None, precision=precision)
    s.curl_potential(dw)
    s.set_primitives(dw)
    return s


def _oracle_full_dt(g, d, tab=None):
    """The oracle's CFL step of the whole initial grid."""
    from oracle.scheme import Solver
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    return s.cfl_dt()


def _compare(G, s, g, origin, wrap, tol):
    """GPU interior at the window centre vs the oracle window's centre.
    Positive fields: per-zone relative error; signed fields: error over the
    field's maximum in the whole window."""
    idx = []
    for a in range(3):
        r = np.arange(origin[a] + MARGIN, origin[a] + MARGIN + W)
        idx.append(r % g.n[a] if wrap[a] else r)
    c = slice(s.grid.ng + MARGIN, s.grid.ng + MARGIN + W)
    errs = {}
    for which, names, grp in (("prim", PRIM, s.P), ("cons", CONS, s.U)):
        gv = _gpu_block(G, which, idx)
        for k in names:
            ref_all = s.interior(grp[k])
            ref = grp[k][c, c, c]
            if k in ("rho", "p", "D", "tau"):
                e = np.max(np.abs(gv[k] - ref) / np.abs(ref))
            else:
                e = np.max(np.abs(gv[k] - ref)) / np.max(np.abs(ref_all))
            errs[k] = float(e)
    assert max(errs.values()) < tol, (origin, errs)
    return errs


BOX_WINDOWS = [(100, 120, 140), (256 - 30, 250, 2), (7, 200, 255 - 40)]


@gpu
def test_box256_one_step_windows():
    """Turbulent SRMHD box 256^3 (FP64, device layout, kernels and device
    CFL step of the benchmark): the device dt equals the oracle's global CFL
    step to 1e-13; after one RK3 step, at three windows (two wrapping across
    the periodic boundaries) every compared zone and field within 1e-11."""
    _torch()
    from workloads import box
    from workloads.grid import BC_OUTFLOW
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(256)
    dt = _oracle_full_dt(g, d)
    G = Grid(g)
    G.curl_potential(d)
    G.set_primitives(d)
    dt_gpu = G.rk_step(0.0, want_dt=True)
    assert abs(dt_gpu / dt - 1) < 1e-13, (dt_gpu, dt)
    m = W + 2 * MARGIN
    for o in BOX_WINDOWS:
        s = _oracle_window(g, d, o, (m, m, m), (BC_OUTFLOW,) * 6, (True, True, True))
        s.rk_step(dt)
        _compare(G, s, g, o, (True, True, True), 1e-11)
    G.close()


@gpu
def test_box256_invariants_device_dt():
    """256^3, three steps with the device CFL step as benchmarked: total D,
    S, tau and face-field sums conserved to round-off, div B at round-off,
    no failed inversions, and two runs bitwise identical."""
    torch = _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(256)
    runs = []
    for rep in range(2):
        G = Grid(g)
        G.curl_potential(d)
        G.set_primitives(d)
        d0 = G.diagnostics()
        for _ in range(3):
            G.rk_step()
        d1 = G.diagnostics()
        if rep == 0:
            for q in range(8):
                v = G._interior(G.field_view(G.cons, q))
                scale = float(torch.sum(torch.abs(v)))
                assert abs(d1["sum_cons"][q] - d0["sum_cons"][q]) <= 1e-12 * scale, CONS[q]
            assert d1["max_divb"] <= 1e-12
            assert d1["n_c2p_fail"] == 0 and d1["n_nonfinite"] == 0
            assert d1["dt"] > 0 and d1["t"] > 0
        G.synchronize()
        runs.append(G.cons.clone())
        G.close()
        del G
    assert torch.equal(runs[0], runs[1])


@gpu
def test_box256_graph_replay_equals_eager():
    """The benchmark's launch configuration at 256^3: a grid on its own
    stream replaying the captured device-dt step equals a grid stepped
    launch by launch, bit for bit (state, primitives including ghosts, time
    and dt), over two steps; the eager path is the one checked against the
    oracle above."""
    torch = _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(256)
    E = Grid(g)
    R = Grid(g, stream=torch.cuda.Stream())
    for G in (E, R):
        G.curl_potential(d)
        G.set_primitives(d)
    for _ in range(2):
        E.rk_step()
    R.rk_steps_graph(2)
    E.synchronize()
    R.synchronize()
    assert torch.equal(E.cons, R.cons)
    assert torch.equal(E.prim, R.prim)
    de, dr = E.diagnostics(), R.diagnostics()
    assert de["t"] == dr["t"] and de["dt"] == dr["dt"] and de["step"] == dr["step"] == 2
    E.close()
    R.close()


def _torus_window_case(n, origins, guess_trained=False):
    from workloads.torus import torus
    from workloads.metric import kerr_schild_tables
    from workloads.grid import BC_OUTFLOW
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g, d, tab = torus(*n)
    m = W + 2 * MARGIN
    wrap = (False, False, True)
    dt = _oracle_full_dt(g, d, tab)
    if guess_trained:
        G = Grid(g, tables=tab, guess=L.GUESS_MLP)
        flat, norm = _quick_weights()
        G.mlp_set_weights(flat, norm)
    else:
        G = Grid(g, tables=tab)
    G.curl_potential(d)
    G.set_primitives(d)
    dt_gpu = G.rk_step(0.0, want_dt=True)
    assert abs(dt_gpu / dt - 1) < 1e-13, (dt_gpu, dt)
    for o in origins:
        s = _oracle_window(g, d, o, (m, m, m), (BC_OUTFLOW,) * 6, wrap,
                           tables_fn=kerr_schild_tables)
        s.rk_step(dt)
        _compare(G, s, g, o, wrap, 1e-10)
    dg = G.diagnostics()
    G.close()
    return dg


def _quick_weights():
    """A network trained briefly on the GPU (2^18 seeded samples, 3 epochs)."""
    from workloads import box
    from workloads.mlp_data import sample_prims, init_weights
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g, _ = box.turbulent_box(8)
    G = Grid(g)
    G.mlp_set_weights(L.mlp_pack(init_weights()), np.ones(32, np.float32))
    feat, targ = G.mlp_datagen(sample_prims(1 << 18, seed=1810), set_norm=True)
    for _ in range(3):
        for s0 in range(0, feat.shape[0], 4096):
            G.mlp_train_step(feat[s0:s0 + 4096], targ[s0:s0 + 4096], 1e-3)
    out = G.mlp_get_weights()
    G.close()
    return out


@gpu
def test_torus_256x128x128_one_step_window():
    """Kerr-Schild a = 0.9 torus at 256 x 128 x 128 (floors on): one RK3
    step; two equatorial windows (theta about 0.30 .. 0.73 pi), centred on
    the density maximum (r about 9.9) and on the inner edge of the torus
    (r about 6.4, torus against floored atmosphere), one wrapping in phi;
    every compared zone and field within 1e-10."""
    _torch()
    _torus_window_case((256, 128, 128), [(116, 38, 128 - 20), (86, 38, 5)])


@gpu
def test_torus_384x192x192_learned_guess_window():
    """The learned-guess configuration at its full size (384 x 192 x 192,
    Newton started from the network's guess, warm-guess fallback): the step
    reaches the same state as the oracle's plain Newton, within 1e-10, at
    an equatorial window."""
    _torch()
    dg = _torus_window_case((384, 192, 192), [(189, 68, 150)], guess_trained=True)
    assert dg["n_c2p_fail"] == 0


@gpu
def test_precision_form_512_one_step_window():
    """FP32-flux form at 512^3 (the precision workload): one RK3 step
    against the oracle's float32 form at a window; the two differ only by
    float32 rounding order, so the bound is float32-level (2e-6 of the
    field scale after one step)."""
    _torch()
    from workloads import box
    from workloads.grid import BC_OUTFLOW
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(512)
    m = W + 2 * MARGIN
    o = (512 - 25, 300, 17)
    s = _oracle_window(g, d, o, (m, m, m), (BC_OUTFLOW,) * 6, (True, True, True),
                       precision="fp32")
    dt = 0.9 * s.cfl_dt()
    G = Grid(g, precision=1)
    G.curl_potential(d)
    G.set_primitives(d)
    del d
    G.rk_step(dt)
    s.rk_step(dt)
    _compare(G, s, g, o, (True, True, True), 2e-6)
    G.close()
