"""Sub-box windows of a full periodic or torus workload, for parity at sizes
the oracle cannot step whole.

One SSP-RK3 step changes a zone only through zones within a bounded
distance: per stage, a cell-centred update reaches 5 cells (MP5 reads 2..3
cells on each side of a face, the flux derivative 3 faces on each side),
and the face field reaches 8 (edge reconstruction, the edge derivative,
then the centred interpolation of the new face field), so 24 per step.
A window with a margin of MARGIN >= 24 zones around its centre, evolved with
any ghost treatment, reproduces the full-grid step in that centre exactly
(same arithmetic, element by element).
"""
import numpy as np

from workloads.grid import GridSpec, BC_OUTFLOW

MARGIN = 26


def _take(a, axis_idx):
    """a[k][j][i] at index arrays (ik, ij, ii) (outer product)."""
    ik, ij, ii = axis_idx
    return a[np.ix_(ik, ij, ii)]


def window_spec(g, origin, size, bc):
    """GridSpec of a window with interior cells origin .. origin + size - 1."""
    x0 = tuple(g.x0[a] + origin[a] * g.dx[a] for a in range(3))
    return GridSpec(n=size, ng=g.ng, coord=g.coord, x0=x0, dx=g.dx, bc=bc,
                    gamma_ad=g.gamma_ad, cfl=g.cfl, rho_fl_a=g.rho_fl_a, rho_fl_n=g.rho_fl_n,
                    p_fl_a=g.p_fl_a, p_fl_n=g.p_fl_n, w_max=g.w_max,
                    newton_maxit=g.newton_maxit, newton_tol=g.newton_tol)


def window_data(g, d, origin, size, wrap):
    """Initial data of a window.  Cell fields [k][j][i] without ghosts,
    potentials A1..A3 with ng ghosts; indices wrap periodically along the
    axes where wrap[a] is set (direction a = 0 is x^1)."""
    ng = g.ng
    def idx(a, lo, hi, ghosts):
        r = np.arange(origin[a] + lo, origin[a] + hi)
        if wrap[a]:
            return r % g.n[a]
        assert r.min() >= -ghosts and r.max() < g.n[a] + ghosts, "window leaves the grid"
        return r
    out = {}
    cells = [idx(a, 0, size[a], 0) for a in range(3)]
    for k in ("rho", "u1", "u2", "u3", "p"):
        out[k] = np.ascontiguousarray(_take(d[k], (cells[2], cells[1], cells[0])))
    for k in ("A1", "A2", "A3"):
        A = d[k]
        ax = []
        for a in range(3):
            r = idx(a, -ng, size[a] + ng, ng)
            ax.append(r + ng if not wrap[a] else (r % g.n[a]) + ng)
        out[k] = np.ascontiguousarray(_take(A, (ax[2], ax[1], ax[0])))
    return out


def centre_slices(origin, size, margin=MARGIN):
    """Interior index ranges (full grid, unwrapped) of the exact centre."""
    return [(origin[a] + margin, origin[a] + size[a] - margin) for a in range(3)]
