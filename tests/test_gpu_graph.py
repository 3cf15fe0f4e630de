"""Graph replay of the device-dt RK3 step (grmhd_rk_steps_graph): every
replay is checked against eager steps bit for bit, with the program's own
eager work and synchronisations between the replays; the graph is dropped and
captured again when the launch sequence changes.  Box and torus, and every
kernel form: FP32, fourth-order derivative on four ghost layers, MP7, WENO5,
PLM, the learned guess's list pass (the fallback's: test_gpu_fallback.py)."""
import numpy as np
import pytest

gpu = pytest.mark.gpu
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _grids(g, d, tab=None, **kw):
    import torch
    from paper_1810_04597_amd.grid import Grid
    out = []
    for _ in range(2):
        G = Grid(g, tables=tab, stream=torch.cuda.Stream(), **kw)
        G.curl_potential(d)
        G.set_primitives(d)
        out.append(G)
    return out


def _same(A, B):
    a, b = A.to_numpy("cons"), B.to_numpy("cons")
    pa, pb = A.to_numpy("prim"), B.to_numpy("prim")
    for k in CONS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    for k in pa:
        assert np.array_equal(pa[k], pb[k], equal_nan=True), k
    da, db = A.diagnostics(), B.diagnostics()
    assert da["t"] == db["t"] and da["dt"] == db["dt"] and da["step"] == db["step"]


@gpu
def test_graph_replays_equal_eager_steps_box():
    """Periodic 24^3 box (the update and the inversion write the ghost
    images): one eager step, then single-step replays with reads, a torch
    reduction and host synchronisation between them, each equal to the
    eager grid's state bit for bit; then a multi-step replay."""
    torch = _torch()
    from workloads import box
    g, d = box.turbulent_box(24)
    E, R = _grids(g, d)
    for rep in range(4):
        E.rk_step()
        R.rk_steps_graph(1)
        _same(E, R)
        float(torch.sum(R.cons))          # eager work on torch's stream
        torch.cuda.synchronize()
    for _ in range(3):
        E.rk_step()
    R.rk_steps_graph(3)
    _same(E, R)
    E.close()
    R.close()


@gpu
def test_graph_replays_equal_eager_steps_torus():
    """Torus 32x16x16 (outflow and axis boundaries: ghost fills inside the
    step, floors): replays equal eager steps bit for bit."""
    _torch()
    from workloads.torus import torus
    g, d, tab = torus(32, 16, 16)
    E, R = _grids(g, d, tab)
    for rep in range(3):
        E.rk_step()
        R.rk_steps_graph(1)
        _same(E, R)
    E.close()
    R.close()


@gpu
def test_graph_after_state_change_and_split_change():
    """A new state between replays (the next step reduces the CFL step
    eagerly, then replays), and a change of the Newton split (the graph is
    captured again): still equal to eager steps."""
    _torch()
    from workloads import box
    g, d = box.turbulent_box(16)
    _, d2 = box.turbulent_box(16, seed=7)
    E, R = _grids(g, d)
    E.rk_step()
    R.rk_steps_graph(1)
    for G in (E, R):
        G.curl_potential(d2)
        G.set_primitives(d2)
    for _ in range(2):
        E.rk_step()
    R.rk_steps_graph(2)
    _same(E, R)
    for G in (E, R):
        G.set_newton_split(1)
    for _ in range(2):
        E.rk_step()
    R.rk_steps_graph(2)
    _same(E, R)
    E.close()
    R.close()


@gpu
@pytest.mark.parametrize("variant", ["fp32", "d4_ng4", "mp7_ng6", "weno5", "plm", "learned_all"])
def test_graph_replays_equal_eager_steps_variants(variant):
    """The other kernel forms in a captured step (16^3 box): the FP32 form,
    the fourth-order derivative on four ghost layers, MP7 on six, WENO5,
    PLM, and the learned guess with every zone deferred to the network pass
    (its list filled by atomics in any order; untrained weights): replays
    equal eager steps bit for bit, with eager work between them."""
    torch = _torch()
    from workloads import box
    from workloads.mlp_data import init_weights
    from paper_1810_04597_amd import _lib as L
    kw, ng = {}, 5
    if variant == "fp32":
        kw = dict(precision=1)
    elif variant == "d4_ng4":
        kw, ng = dict(deriv_order=4), 4
    elif variant == "mp7_ng6":
        kw, ng = dict(recon="mp7"), 6
    elif variant in ("weno5", "plm"):
        kw = dict(recon=variant)
    else:
        kw = dict(guess=L.GUESS_MLP)
    g, d = box.turbulent_box(16, ng=ng)
    E, R = _grids(g, d, **kw)
    if variant == "learned_all":
        w = L.mlp_pack(init_weights())
        for G in (E, R):
            G.mlp_set_weights(w, np.ones(32, np.float32))
            G.set_learned_guess(0.0)
    for rep in range(3):
        E.rk_step()
        R.rk_steps_graph(1)
        _same(E, R)
        float(torch.sum(R.cons))          # eager work on torch's stream
        torch.cuda.synchronize()
    E.close()
    R.close()


@gpu
def test_graph_refusals():
    """Kernel timing on, or the null stream: ESTATE, and nothing ran."""
    torch = _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g, d = box.turbulent_box(8)
    G = Grid(g, stream=torch.cuda.Stream())
    G.curl_potential(d)
    G.set_primitives(d)
    G.set_profiling(True)
    with pytest.raises(L.GrmhdError):
        G.rk_steps_graph(2)
    G.set_profiling(False)
    assert G.diagnostics()["step"] == 0
    G.close()
    N = Grid(g)
    if N.stream.cuda_stream == 0:
        N.curl_potential(d)
        N.set_primitives(d)
        with pytest.raises(L.GrmhdError):
            N.rk_steps_graph(1)
    N.close()
