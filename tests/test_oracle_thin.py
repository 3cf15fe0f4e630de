"""Oracle pins on degenerate boxes (one zone along some directions).

With one zone along x^2 and x^3 every field varies along x^1 only, and the
periodic ghost layers of those directions are copies of the one interior
row.  The staggered differences across them then vanish exactly: the face
field B^1 = D_2 A_3 - D_3 A_2 of the curl is exactly 0, and the induction
equation dB^1/dt = -D_2 E_3 + D_3 E_2 keeps it 0 through the steps, whatever
the other components do.  A ghost fill that wrapped a thin direction wrongly
(a shifted source, a layer left unfilled) breaks this, and the conservation
of the total mass on the periodic box."""
import numpy as np

from oracle.scheme import Solver
from workloads import box


def _run(shape, steps):
    g, d = box.turbulent_box_shape(*shape)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    U0 = {k: s.interior(v).copy() for k, v in s.U.items()}
    for _ in range(steps):
        s.rk_step(s.cfl_dt())
    return s, U0


def test_one_dimensional_box_keeps_its_normal_field_zero():
    s, U0 = _run((24, 1, 1), 3)
    assert np.all(U0["Bf1"] == 0.0)
    assert np.all(s.interior(s.U["Bf1"]) == 0.0)
    # the transverse field and the hydro state do evolve
    for k in ("Bf2", "Bf3", "S1", "tau"):
        assert np.max(np.abs(s.interior(s.U[k]) - U0[k])) > 1e-6, k
    assert abs(s.interior(s.U["D"]).sum() / U0["D"].sum() - 1) < 1e-14


def test_thin_boxes_conserve_and_keep_div_b():
    for shape in ((16, 12, 1), (1, 10, 14), (9, 2, 7)):
        s, U0 = _run(shape, 3)
        assert abs(s.interior(s.U["D"]).sum() / U0["D"].sum() - 1) < 1e-14, shape
        assert s.diagnostics()["max_divb"] < 1e-13, shape
        for k, v in s.U.items():
            assert np.isfinite(s.interior(v)).all(), (shape, k)
