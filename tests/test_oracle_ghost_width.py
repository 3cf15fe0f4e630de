"""Pins of the ghost width as a grid parameter with the fourth-order
derivative (oracle/scheme.py: faces and edges from -flo to n + flo - 2).

The oracle's face and edge arrays start as NaN everywhere and are written
only over the range formed, so a derivative that reached a face or edge
outside it would give NaN.  With the fourth-order derivative the faces and
edges [-2, n] suffice, so four ghost layers serve MP5, WENO5 and PLM (five
serve MP7): the right-hand side and three steps on a grid with one layer
fewer equal those on the wider grid bit for bit (box and torus), and a grid
too narrow for its reconstruction and order is refused.
"""
import numpy as np
import pytest

from oracle.scheme import Solver
from workloads import box


def _rhs_and_steps(g, d, recon, tab=None, steps=3):
    s = Solver(g, tab, recon=recon, deriv_order=4)
    if "A1" in d:
        s.curl_potential(d)
    else:
        s.set_face_fields(d)
    s.set_primitives(d)
    L = s.rhs()
    for _ in range(steps):
        s.rk_step(2e-3)
    return L, {k: s.interior(v).copy() for k, v in s.U.items()}, s


@pytest.mark.parametrize("recon,ng", [("mp5", 4), ("weno5", 4), ("plm", 4), ("mp7", 5)])
def test_one_layer_fewer_changes_nothing_with_the_fourth_order(recon, ng):
    out = {}
    for g_ in (ng, ng + 1):
        g, d = box.turbulent_box(12, ng=g_)
        out[g_] = _rhs_and_steps(g, d, recon)
    for k in out[ng][0]:
        assert np.all(np.isfinite(out[ng][0][k])), k
        assert np.array_equal(out[ng][0][k], out[ng + 1][0][k]), k
    for k in out[ng][1]:
        assert np.array_equal(out[ng][1][k], out[ng + 1][1][k]), k
    assert out[ng][2].diagnostics()["max_divb"] <= 1e-12


def test_four_ghost_layers_on_the_torus():
    from workloads.torus import torus
    out = {}
    for ng in (4, 5):
        g, d, tab = torus(24, 12, 12, ng=ng)
        out[ng] = _rhs_and_steps(g, d, "mp5", tab, steps=1)
    for k in out[4][0]:
        assert np.array_equal(out[4][0][k], out[5][0][k]), k
    for k in out[4][1]:
        assert np.array_equal(out[4][1][k], out[5][1][k]), k


def test_too_narrow_grids_are_refused():
    g, d = box.turbulent_box(8, ng=4)
    with pytest.raises(ValueError):
        Solver(g)                               # sixth order needs five layers
    with pytest.raises(ValueError):
        Solver(g, recon="mp7", deriv_order=4)   # MP7 reaches one cell further
    Solver(g, deriv_order=4)
    g5, _ = box.turbulent_box(8, ng=5)
    with pytest.raises(ValueError):
        Solver(g5, recon="mp7")
    Solver(g5, recon="mp7", deriv_order=4)
