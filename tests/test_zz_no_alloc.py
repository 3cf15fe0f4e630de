"""The no-allocation CFL step (grmhd_compute_dt_noalloc) against the
allocating path's grmhd_compute_dt, through the C ABI: two calls in a row,
the second on a smaller grid that reuses the device scratch the first one
wrote, each result equal bit for bit to compute_dt's (the same kernels reduce
the same partials in the same order); a grid beyond the scratch's limit is
refused before any launch; captured into a graph and replayed after state
changes, it writes each state's step."""
import numpy as np
import pytest

gpu = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@gpu
def test_compute_dt_noalloc_matches_compute_dt():
    torch = _torch()
    from workloads import box
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    ga, da = box.turbulent_box(96)
    A = Grid(ga)
    A.curl_potential(da)
    A.set_primitives(da)
    gb, db, tab = torus(32, 16, 16)
    B = Grid(gb, tables=tab)
    B.curl_potential(db)
    B.set_primitives(db)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=A.device)
    A.compute_dt_noalloc(out[0:1])
    B.compute_dt_noalloc(out[1:2])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array([A.compute_dt(), B.compute_dt()])
    print("noalloc dt %r, compute_dt %r" % (got.tolist(), want.tolist()))
    assert np.array_equal(got, want), (got, want)
    assert got[0] > 0.0 and got[1] > 0.0
    # again in the opposite order (larger grid after the smaller one)
    out.fill_(-1.0)
    B.compute_dt_noalloc(out[1:2])
    A.compute_dt_noalloc(out[0:1])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    A.close()
    B.close()


@gpu
def test_compute_dt_noalloc_refuses_grids_beyond_its_scratch():
    torch = _torch()
    from workloads.grid import GridSpec
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    # 513 x 512 x 512 interior zones: 2^27 + 2^18, one workgroup row too many
    G = Grid(GridSpec(n=(513, 512, 512)))
    out = torch.zeros((1,), dtype=torch.float64, device=G.device)
    with pytest.raises(L.GrmhdError) as ei:
        G.compute_dt_noalloc(out)
    assert ei.value.code == L.EINVAL and "too large" in str(ei.value)
    G.close()
    del G
    torch.cuda.empty_cache()


@gpu
def test_compute_dt_noalloc_in_a_captured_graph():
    """What the call is for: captured into a graph (torch's graph capture on
    the grid's own stream; the call launches kernels only) and replayed after
    the state has changed, each replay writes the CFL step of the current
    state, equal bit for bit to compute_dt's."""
    torch = _torch()
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.turbulent_box(48)
    G = Grid(g, stream=torch.cuda.Stream())
    G.curl_potential(d)
    G.set_primitives(d)
    out = torch.full((1,), -1.0, dtype=torch.float64, device=G.device)
    G.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=G.stream, capture_error_mode="thread_local"):
        G.compute_dt_noalloc(out)
    seen = []
    for rep in range(3):
        out.fill_(-1.0)                       # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = float(out.item())
        assert got == G.compute_dt(), rep
        seen.append(got)
        G.rk_step(0.0)                        # a new state for the next replay
        G.synchronize()
    print("captured noalloc dt per replay", seen)
    assert len(set(seen)) == 3
    del graph
    G.close()
