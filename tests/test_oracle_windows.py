"""The window method used for full-size parity (tests/windows.py): a
sub-box of a periodic grid, stepped by the oracle with outflow ghosts,
reproduces the full-grid step exactly (bit for bit) at its centre, also
when the window wraps across the periodic boundaries."""
import numpy as np

from windows import MARGIN, window_spec, window_data


def test_window_centre_equals_full_step():
    from workloads import box
    from workloads.grid import BC_OUTFLOW
    from oracle.scheme import Solver
    n = 40
    g, d = box.turbulent_box(n)
    dt = 2e-3
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    s.rk_step(dt)
    w = 2
    m = w + 2 * MARGIN
    origin = (n - MARGIN - 1, 3, 17)
    gw = window_spec(g, origin, (m, m, m), (BC_OUTFLOW,) * 6)
    sw = Solver(gw)
    dw = window_data(g, d, origin, (m, m, m), (True, True, True))
    sw.curl_potential(dw)
    sw.set_primitives(dw)
    sw.rk_step(dt)
    idx = [np.arange(origin[a] + MARGIN, origin[a] + MARGIN + w) % n for a in range(3)]
    c = slice(g.ng + MARGIN, g.ng + MARGIN + w)
    for grp_full, grp_win in ((s.U, sw.U), (s.P, sw.P)):
        for k in grp_full:
            full = s.interior(grp_full[k])[np.ix_(idx[2], idx[1], idx[0])]
            assert np.array_equal(full, grp_win[k][c, c, c]), k
