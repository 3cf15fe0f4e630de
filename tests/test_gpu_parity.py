"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  FP64 tolerance for one application of an operator:
1e-12 relative (round-off of a few hundred operations with different FMA
contraction and reciprocal order); after 10 RK3 steps: 1e-10 relative per
zone and field."""
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


def _pair_box(n, precision=0):
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(n)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, precision=precision)
    G.curl_potential(d)
    G.set_primitives(d)
    return g, d, s, G


def _oracle_fields(s):
    return ({k: interior(v) for k, v in s.P.items()}, {k: interior(v) for k, v in s.U.items()})


@gpu
def test_library_path_is_native():
    _torch()
    from paper_1810_04597_amd import _lib
    L = _lib.lib()
    assert L._name.endswith("libgrmhd.so")


@gpu
@pytest.mark.parametrize("n", [16, 19])
def test_init_prim2cons_matches_oracle(n):
    _torch()
    g, d, s, G = _pair_box(n)
    P, U = _oracle_fields(s)
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    e = max_rel(gc, U, CONS)
    e.update(max_rel(gp, P, PRIM))
    assert max(e.values()) < 1e-12, e


@gpu
@pytest.mark.parametrize("n", [16, 21])
def test_rhs_matches_oracle(n):
    _torch()
    g, d, s, G = _pair_box(n)
    L_o = s.rhs()
    out = G.rhs()
    L_g = G.read_group(out, CONS, interior=True)
    errs = {}
    for k in CONS:
        ref = L_o[k]
        scale = np.max(np.abs(ref))
        errs[k] = float(np.max(np.abs(L_g[k] - ref)) / scale)
    assert max(errs.values()) < 1e-11, errs


@gpu
def test_cons2prim_matches_oracle_perturbed():
    _torch()
    import torch
    g, d, s, G = _pair_box(16)
    # perturb the conserved hydro state identically on both sides, then invert
    rng = np.random.default_rng(5)
    gg = g.ng
    for f, k in enumerate(("D", "S1", "S2", "S3", "tau")):
        fac = 1.0 + 1e-3 * rng.uniform(-1, 1, size=(16, 16, 16))
        s.U[k][gg:-gg, gg:-gg, gg:-gg] *= fac
        v = G.field_view(G.cons, f)[gg:-gg, gg:-gg, gg:-gg]
        v.mul_(torch.from_numpy(fac).to(v.device))
    st = s.cons2prim()
    nf = G.cons2prim()
    assert nf == st["n_fail"] == 0
    P, _ = _oracle_fields(s)
    gp = G.to_numpy("prim", interior=True)
    e = max_rel(gp, P, PRIM)
    assert max(e.values()) < 1e-12, e


@gpu
def test_cfl_dt_matches_oracle():
    _torch()
    g, d, s, G = _pair_box(16)
    assert abs(G.compute_dt() / s.cfl_dt() - 1) < 1e-13


@gpu
def test_dt_reduction_over_a_ragged_block_count():
    """136^3 box: 9826 per-block CFL partials, more than one round of the
    final reduction's eight loads per thread over 1024 threads, plus a
    remainder.  The device CFL step of the initial state equals the oracle's;
    the step the last inversion of a step reduces for the next step equals a
    fresh reduction of the same state by the CFL kernel (a second grid from
    the same data, stepped the same way)."""
    _torch()
    from paper_1810_04597_amd.grid import Grid
    n = 136
    nblk = -(-n ** 3 // 256)
    assert nblk > 8 * 1024 and nblk % (8 * 1024) != 0
    g, d, s, G = _pair_box(n)
    assert abs(G.compute_dt() / s.cfl_dt() - 1) < 1e-13
    G2 = Grid(g)
    G2.curl_potential(d)
    G2.set_primitives(d)
    G.rk_step(0.0)
    G2.rk_step(0.0)
    dt_fresh = G2.compute_dt()
    dt_inv = G.rk_step(0.0, want_dt=True)
    assert abs(dt_inv / dt_fresh - 1) < 1e-14, (dt_inv, dt_fresh)


@gpu
def test_ten_steps_config0_parity():
    """Turbulent SRMHD box 32^3, 10 SSP-RK3 steps with the device CFL step:
    every zone and field within 1e-10 relative of the oracle."""
    _torch()
    g, d, s, G = _pair_box(32)
    for _ in range(10):
        dt_o = s.cfl_dt()
        dt_g = G.rk_step(0.0, want_dt=True)
        assert abs(dt_g / dt_o - 1) < 1e-11
        s.rk_step(dt_o)
    P, U = _oracle_fields(s)
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    e = max_rel(gp, P, PRIM)
    e.update(max_rel(gc, U, CONS))
    assert max(e.values()) < 1e-10, e


@gpu
def test_ten_steps_64_parity():
    """The 256^3 benchmark's generator at 64^3 (several tiles of every kernel
    in every direction, four x^3 segments of the update), 10 SSP-RK3 steps with
    the device CFL step: every zone and field within 1e-10 relative of the
    oracle, div B at round-off, no failed inversion."""
    _torch()
    g, d, s, G = _pair_box(64)
    for _ in range(10):
        dt_o = s.cfl_dt()
        dt_g = G.rk_step(0.0, want_dt=True)
        assert abs(dt_g / dt_o - 1) < 1e-11
        s.rk_step(dt_o)
    P, U = _oracle_fields(s)
    e = max_rel(G.to_numpy("prim", interior=True), P, PRIM)
    e.update(max_rel(G.to_numpy("cons", interior=True), U, CONS))
    assert max(e.values()) < 1e-10, e
    dg = G.diagnostics()
    assert dg["max_divb"] <= 1e-12 and dg["n_c2p_fail"] == 0
    G.close()


@gpu
@pytest.mark.parametrize("shape", [(37, 21, 27), (70, 10, 18)])
def test_ten_steps_ragged_box_parity(shape):
    """Non-cubic periodic boxes whose sizes are not multiples of the kernels'
    tiles: 37 x 21 x 27 (a partial 64-wide x^1 row in the x^2/x^3 stencil
    tiles, ragged 4-face tiles, a 16-zone x^3 segment plus an 11-zone tail in
    the update) and 70 x 10 x 18 (two x^1 rows of 64 with a 6-wide tail, a
    2-zone x^3 tail).  Ten SSP-RK3 steps with the device CFL step: every zone
    and field within 1e-10 relative of the oracle."""
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box_shape(*shape)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g)
    G.curl_potential(d)
    G.set_primitives(d)
    for _ in range(10):
        dt_o = s.cfl_dt()
        dt_g = G.rk_step(0.0, want_dt=True)
        assert abs(dt_g / dt_o - 1) < 1e-11
        s.rk_step(dt_o)
    P, U = _oracle_fields(s)
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    e = max_rel(gp, P, PRIM)
    e.update(max_rel(gc, U, CONS))
    assert max(e.values()) < 1e-10, e
    dg = G.diagnostics()
    assert dg["max_divb"] <= 1e-12 and dg["n_c2p_fail"] == 0
    G.close()


@gpu
@pytest.mark.parametrize("shape", [(24, 1, 1), (16, 12, 1), (1, 10, 14), (9, 2, 7)])
def test_thin_grids_parity(shape):
    """Degenerate boxes: one zone (or two) along some directions, so the
    periodic ghost fill wraps several times and the staged tiles, the x^3
    segments and the face ranges hold a single interior row; the ghost
    images are filled by the separate fill kernels (n < 2 ng).  Five steps
    with the device CFL step: every zone and field within 1e-10 relative of
    the oracle, div B at round-off."""
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box_shape(*shape)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g)
    G.curl_potential(d)
    G.set_primitives(d)
    for _ in range(5):
        dt_o = s.cfl_dt()
        dt_g = G.rk_step(0.0, want_dt=True)
        assert abs(dt_g / dt_o - 1) < 1e-11
        s.rk_step(dt_o)
    P, U = _oracle_fields(s)
    gp = G.to_numpy("prim", interior=True)
    gc = G.to_numpy("cons", interior=True)
    e = max_rel(gp, P, PRIM)
    e.update(max_rel(gc, U, CONS))
    assert max(e.values()) < 1e-10, e
    dg = G.diagnostics()
    assert dg["max_divb"] <= 1e-12 and dg["n_c2p_fail"] == 0
    G.close()


@gpu
def test_conservation_and_divb_on_gpu():
    _torch()
    g, d, s, G = _pair_box(24)
    d0 = G.diagnostics()
    for _ in range(5):
        G.rk_step()
    d1 = G.diagnostics()
    c = G.to_numpy("cons", interior=True)
    for q, k in enumerate(CONS):
        scale = np.sum(np.abs(c[k]))
        assert abs(d1["sum_cons"][q] - d0["sum_cons"][q]) <= 1e-13 * scale, k
    assert d1["max_divb"] <= 1e-12
    assert d1["n_c2p_fail"] == 0 and d1["n_nonfinite"] == 0


@gpu
def test_determinism_bitwise():
    _torch()
    outs = []
    for _ in range(2):
        g, d, s, G = _pair_box(16)
        for _ in range(3):
            G.rk_step()
        outs.append(G.to_numpy("cons"))
    for k in CONS:
        assert np.array_equal(outs[0][k], outs[1][k], equal_nan=True), k


@gpu
def test_device_dt_follows_state_changes():
    """A device-dt step stores the CFL step of the state it leaves; a new
    state (curl_potential / set_primitives) drops it, and the next
    device-dt step takes the CFL step of the new state."""
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    g, d, s, G = _pair_box(16)
    G.rk_step(0.0)
    g2, d2 = box.turbulent_box(16, seed=7)
    s2 = Solver(g2)
    s2.curl_potential(d2)
    s2.set_primitives(d2)
    G.curl_potential(d2)
    G.set_primitives(d2)
    dt_g = G.rk_step(0.0, want_dt=True)
    assert abs(dt_g / s2.cfl_dt() - 1) < 1e-13
    # the stored value of the state just left is the CFL step of that state
    dt_next = G.rk_step(0.0, want_dt=True)
    s2.rk_step(s2.cfl_dt())
    assert abs(dt_next / s2.cfl_dt() - 1) < 1e-11


@gpu
def test_periodic_ghost_images_after_step():
    """On a periodic box the update and the inversion write the ghost images
    of what they produce (the step runs no separate ghost fill): after a step
    and after a standalone inversion, every ghost element of the primitives
    and of the face fields equals its periodic source, bit for bit."""
    _torch()
    g, d, s, G = _pair_box(12)
    n, ng = 12, 5
    idx = (np.arange(-ng, n + ng) % n) + ng
    for action in ("step", "cons2prim"):
        if action == "step":
            G.rk_step()
        else:
            G.cons2prim()
        P = G.to_numpy("prim")
        U = G.to_numpy("cons")
        for name, a in list(P.items()) + [(k, U[k]) for k in ("Bf1", "Bf2", "Bf3")]:
            want = a[np.ix_(idx, idx, idx)]
            assert np.array_equal(a, want), (action, name)
