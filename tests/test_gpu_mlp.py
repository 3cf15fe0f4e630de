"""Learned Newton guess on the GPU: training pairs, BF16 MFMA forward and
gradients against the FP64 oracle, training, and the gain of the trained
network over the method's cold start."""
import numpy as np
import pytest

gpu = pytest.mark.gpu
GAM = 4.0 / 3.0


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) >> 16
    return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _grid():
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(16)
    G = Grid(g)
    G.curl_potential(d)
    G.set_primitives(d)
    return g, d, G


def _setup(n, seed=5):
    from workloads.mlp_data import sample_prims, init_weights
    from oracle import mlp
    from paper_1810_04597_amd import _lib as L
    prims = sample_prims(n, seed=seed)
    f, t = mlp.features_targets(prims, GAM)
    fm, fs = mlp.standardise_stats(f)
    tm, ts = mlp.standardise_stats(t)
    params = init_weights()
    norm = L.mlp_norm_pack(fm, fs, tm, ts)
    return prims, f, t, params, norm


def _emulated_forward(params, x):
    """FP64 forward with the GPU's roundings: bf16 weights and layer inputs."""
    h = bf16(x)
    acts = [h]
    for li, (w, b) in enumerate(params):
        z = h @ bf16(w).T + b
        if li < 3:
            h = np.tanh(z)
            acts.append(h)
            h = bf16(h)
        else:
            h = z
    return h


@gpu
def test_datagen_matches_oracle():
    _torch()
    from oracle import mlp
    prims, f, t, params, norm = _setup(4096)
    g, d, G = _grid()
    feat, targ = G.mlp_datagen(prims)
    fg = feat.cpu().numpy()
    tg = targ.cpu().numpy()[:, :5]
    assert np.max(np.abs(fg - f) / (np.abs(f) + 1e-3)) < 1e-5
    assert np.max(np.abs(tg - t) / (np.abs(t) + 1e-3)) < 1e-5


@gpu
def test_forward_matches_emulated_oracle():
    _torch()
    from paper_1810_04597_amd import _lib as L
    prims, f, t, params, norm = _setup(2000)
    g, d, G = _grid()
    G.mlp_set_weights(L.mlp_pack(params), norm)
    feat, targ = G.mlp_datagen(prims)
    out = G.mlp_forward(feat).cpu().numpy()[:, :5]
    fm, fs = norm[0:8].astype(np.float64), norm[8:16].astype(np.float64)
    x = (feat.cpu().numpy().astype(np.float64) - fm) / fs
    ref = _emulated_forward(params, x.astype(np.float32))
    # same roundings on both sides: FP32 vs FP64 accumulation and tanh
    assert np.max(np.abs(out - ref)) < 2e-3, np.max(np.abs(out - ref))


@gpu
def test_gradients_match_oracle():
    """BF16 GPU gradients against the FP64 oracle on the same bf16-rounded
    weights and inputs: norm-relative difference per layer <= 2e-2."""
    _torch()
    from oracle import mlp
    from paper_1810_04597_amd import _lib as L
    prims, f, t, params, norm = _setup(4096)
    g, d, G = _grid()
    G.mlp_set_weights(L.mlp_pack(params), norm)
    feat, targ = G.mlp_datagen(prims)
    grad, loss = G.mlp_gradient(feat, targ)
    gl = L.mlp_unpack(grad)
    fm, fs = norm[0:8].astype(np.float64), norm[8:16].astype(np.float64)
    tm, ts = norm[16:21].astype(np.float64), norm[24:29].astype(np.float64)
    x = bf16(((feat.cpu().numpy().astype(np.float64) - fm) / fs).astype(np.float32))
    y = (targ.cpu().numpy()[:, :5].astype(np.float64) - tm) / ts
    pq = [(bf16(w.astype(np.float32)), b) for w, b in params]
    loss_o, grads_o = mlp.loss_and_grads(pq, x, y)
    assert abs(loss / loss_o - 1) < 2e-2, (loss, loss_o)
    for li in range(4):
        for a, b in ((gl[li][0], grads_o[li][0]), (gl[li][1], grads_o[li][1])):
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert rel < 2e-2, (li, rel)


def _train(G, n_train, epochs, batch=4096, seed=1810):
    from workloads.mlp_data import sample_prims, init_weights
    from paper_1810_04597_amd import _lib as L
    prims = sample_prims(n_train, seed=seed)
    G.mlp_set_weights(L.mlp_pack(init_weights()), np.ones(32, np.float32))
    feat, targ = G.mlp_datagen(prims, set_norm=True)
    losses = []
    for epoch in range(epochs):
        lr = 1e-3 if epoch < (2 * epochs) // 3 else 3e-4
        for s0 in range(0, feat.shape[0], batch):
            l = G.mlp_train_step(feat[s0:s0 + batch], targ[s0:s0 + batch], lr, want_loss=(s0 == 0))
            if s0 == 0:
                losses.append(l)
    return losses


@gpu
def test_training_reduces_loss_and_beats_cold_start():
    """Train on 2^20 seeded samples, then invert 2^16 unseen samples of the
    same distribution from the cold start (Gamma U) and from the network's
    guess: the guess needs fewer Newton iterations, and both reach the same
    primitives."""
    torch = _torch()
    from workloads.mlp_data import sample_prims
    g, d, G = _grid()
    losses = _train(G, 1 << 20, 9)
    print("training loss per epoch:", losses)
    assert losses[-1] < 0.3 * losses[0]
    test = sample_prims(1 << 16, seed=99)
    feat, targ, cons = G.mlp_datagen(test, want_cons=True)
    out = G.mlp_forward(feat)
    _, norm = G.mlp_get_weights()
    t0 = out[:, 0].double() * float(norm[24]) + float(norm[16])
    y0 = ((cons[:, 4] + cons[:, 0]) * torch.pow(10.0, t0)).contiguous()
    p_cold, it_cold = G.cons2prim_points(cons)
    p_mlp, it_mlp = G.cons2prim_points(cons, y0)
    ic, im = it_cold.cpu().numpy(), it_mlp.cpu().numpy()
    ok = (ic > 0) & (im > 0)
    assert ok.mean() > 0.999
    print("mean Newton iterations: cold %.3f learned %.3f" % (ic[ok].mean(), im[ok].mean()))
    assert im[ok].mean() < ic[ok].mean()
    a, b = p_mlp.cpu().numpy()[ok], p_cold.cpu().numpy()[ok]
    assert np.max(np.abs(a[:, 0] / b[:, 0] - 1)) < 1e-10


@gpu
def test_grid_inversion_with_learned_guess_matches_oracle():
    """Torus grid, learned guess in the inversion: the primitives agree with
    the oracle's (same root), fallbacks are counted."""
    _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    g0, d0, G0 = _grid()
    _train(G0, 1 << 18, 4)
    flat, norm = G0.mlp_get_weights()
    g, d, tab = torus(32, 16, 16)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    G = Grid(g, tables=tab, guess=L.GUESS_MLP)
    G.mlp_set_weights(flat, norm)
    G.curl_potential(d)
    G.set_primitives(d)
    dt = s.cfl_dt()
    s.rk_step(dt)
    G.rk_step(dt)
    from helpers import max_rel, interior
    P = {k: interior(v) for k, v in s.P.items()}
    e = max_rel(G.to_numpy("prim", interior=True), P, ("rho", "u1", "u2", "u3", "p"))
    dg = G.diagnostics()
    print("learned-guess torus: max rel err", e, "fallbacks", dg["n_mlp_fallback"], "iters",
          dg["newton_iters_sum"] / g.zones)
    assert max(e.values()) < 1e-10, e


@gpu
def test_learned_start_wins_when_warm_start_is_poor():
    """Torus grid whose stored primitives (the warm start) are replaced by a
    uniform state after the conserved variables were set: with the learned
    guess as the second candidate, most zones start from it, the inversion
    needs fewer Newton iterations than from the poor warm start, and both
    reach the oracle's inversion of the same conserved state (same root,
    same floors)."""
    torch = _torch()
    from workloads.torus import torus
    from oracle.scheme import Solver
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    from helpers import max_rel, interior
    g0, d0, G0 = _grid()
    _train(G0, 1 << 18, 4)
    flat, norm = G0.mlp_get_weights()
    g, d, tab = torus(32, 16, 16)
    s = Solver(g, tab)
    s.curl_potential(d)
    s.set_primitives(d)
    s.cons2prim()
    P = {k: interior(v) for k, v in s.P.items()}
    res = {}
    for guess in (L.GUESS_WARM, L.GUESS_MLP):
        G = Grid(g, tables=tab, guess=guess)
        if guess == L.GUESS_MLP:
            G.mlp_set_weights(flat, norm)
        G.curl_potential(d)
        G.set_primitives(d)
        for f, val in ((0, 1.0), (1, 0.0), (2, 0.0), (3, 0.0), (4, 1.0)):
            G._interior(G.field_view(G.prim, f)).fill_(val)
        assert G.cons2prim() == 0
        dg = G.diagnostics()
        gp = G.to_numpy("prim", interior=True)
        # u^2 of the initial torus is zero up to round-off: absolute bound
        e = max_rel(gp, P, ("rho", "u1", "u3", "p"))
        e["u2"] = float(np.max(np.abs(gp["u2"] - P["u2"])))
        assert max(e.values()) < 1e-10, (guess, e)
        res[guess] = dg
    warm, learned = res[L.GUESS_WARM], res[L.GUESS_MLP]
    print("poor warm start: iterations warm %d learned %d, learned chosen %d of %d, fallbacks %d" % (
        warm["newton_iters_sum"], learned["newton_iters_sum"], learned["n_mlp_chosen"], g.zones,
        learned["n_mlp_fallback"]))
    assert learned["n_mlp_chosen"] > g.zones // 2
    assert learned["newton_iters_sum"] < warm["newton_iters_sum"]


@gpu
def test_network_start_beats_cold_start_on_the_torus():
    """What the trained network itself gains on its workload, the Kerr-Schild
    torus (64 x 32 x 32): the torus' conserved state inverted with every zone
    started from the network's guess alone (every zone deferred to the
    learned pass, no warm candidate) against every zone from the method's
    cold start Gamma U.  Both reach the same primitives; the network's start
    needs fewer Newton iterations.  With the default policy and the exact
    previous primitives as the warm start, no zone is deferred."""
    _torch()
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    from helpers import max_rel
    g0, d0, G0 = _grid()
    _train(G0, 1 << 18, 4)
    flat, norm = G0.mlp_get_weights()
    g, d, tab = torus(64, 32, 32)
    res, prims = {}, {}
    for name, guess in (("cold", L.GUESS_COLD), ("network", L.GUESS_MLP), ("default", L.GUESS_MLP)):
        G = Grid(g, tables=tab, guess=guess)
        if guess == L.GUESS_MLP:
            G.mlp_set_weights(flat, norm)
            if name == "network":
                G.set_learned_guess(0.0, L.LEARNED_ONLY)
        G.curl_potential(d)
        G.set_primitives(d)
        G.reset_run_counters()
        assert G.cons2prim() == 0
        res[name] = G.diagnostics()
        prims[name] = G.to_numpy("prim", interior=True)
        G.close()
    c, m, w = res["cold"], res["network"], res["default"]
    print("torus 64x32x32 inversion: Newton iterations cold %d (max %d), network %d (max %d), "
          "network chosen %d fallbacks %d of %d zones; default policy deferred %d" % (
              c["newton_iters_sum"], c["newton_iters_max"], m["newton_iters_sum"], m["newton_iters_max"],
              m["run_mlp_chosen"], m["run_mlp_fallback"], g.zones, w["run_mlp_deferred"]))
    assert m["run_mlp_deferred"] == g.zones and m["run_mlp_chosen"] == g.zones
    assert m["newton_iters_sum"] < c["newton_iters_sum"]
    assert w["run_mlp_deferred"] == 0
    e = max_rel(prims["network"], prims["cold"], ("rho", "u1", "u3", "p"))
    e["u2"] = float(np.max(np.abs(prims["network"]["u2"] - prims["cold"]["u2"])))
    assert max(e.values()) < 1e-10, e
