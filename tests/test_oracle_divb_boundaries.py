"""Pins of the face fields at non-periodic boundaries (oracle/scheme.py
face_region, oracle/boundary.py fill_faces).

The discrete div B of a cell is the sum of staggered derivatives of the face
fields over faces that reach 3 (2 for the fourth order) faces beyond the
cell; next to an outflow or polar-axis boundary some of those are ghost
faces.  The scheme evolves those ghost faces with the induction equation, as
it does the owned ones, and sets the edge field to zero on the polar axis,
so d(div B)/dt = 0 holds in every interior cell, the ones beside the
boundaries included: a divergence planted in the face fields of the
Kerr-Schild torus keeps its value, cell by cell, over a step (to round-off),
and the axis faces keep theirs.
"""
import numpy as np
import pytest

from oracle.scheme import Solver, FACE
from workloads.torus import torus


def _divb(s):
    return s.div_b()


@pytest.mark.parametrize("order", [6, 4])
def test_planted_divergence_keeps_its_value_next_to_every_boundary(order):
    g, d, tab = torus(24, 12, 12)
    s = Solver(g, tab, deriv_order=order)
    s.curl_potential(d)
    s.set_primitives(d)
    rng = np.random.default_rng(41)
    scale = max(float(np.nanmax(np.abs(s.U[k]))) for k in FACE)
    for nd, k in enumerate(FACE):
        reg = s.face_region(nd)
        s.U[k][reg] += 1e-6 * scale * rng.normal(size=s.U[k][reg].shape)
    from oracle.boundary import fill_faces
    fill_faces(s.U, g, s.flo)
    s.prim2cons()
    d0 = _divb(s).copy()
    ng = g.ng
    axis0 = (s.U["Bf2"][:, ng - 1, ng:-ng].copy(), s.U["Bf2"][:, ng + g.n[1] - 1, ng:-ng].copy())
    s.rk_step(2e-3)
    d1 = _divb(s)
    # planted divergence is O(1e-6 scale / dx) everywhere; it is carried
    # unchanged (round-off of the update: 1e-12 of the face values)
    assert np.max(np.abs(d0)) > 1e-6
    err = np.max(np.abs(d1 - d0))
    assert err < 1e-9 * np.max(np.abs(d0)), (err, np.max(np.abs(d0)))
    # the cells next to the r boundaries and the axis are among them
    edge_cells = np.zeros(d0.shape, dtype=bool)
    edge_cells[:, :3, :] = edge_cells[:, -3:, :] = True
    edge_cells[:, :, :3] = edge_cells[:, :, -3:] = True
    assert np.max(np.abs(d1 - d0)[edge_cells]) < 1e-9 * np.max(np.abs(d0))
    # the axis faces keep their (planted) values: zero edge field on the
    # axis, so L = 0 there and only the RK weights' rounding remains
    for a, b in zip((s.U["Bf2"][:, ng - 1, ng:-ng], s.U["Bf2"][:, ng + g.n[1] - 1, ng:-ng]), axis0):
        assert np.max(np.abs(a - b)) <= 4e-16 * np.max(np.abs(b)), np.max(np.abs(a - b))


def test_planted_divergence_on_an_outflow_box():
    """Outflow in all three directions (the x^3 boundary included, which the
    torus does not have)."""
    from dataclasses import replace
    from workloads import box
    g0, d = box.turbulent_box(12)
    g = replace(g0, bc=(1,) * 6)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    rng = np.random.default_rng(43)
    for nd, k in enumerate(FACE):
        reg = s.face_region(nd)
        s.U[k][reg] += 1e-6 * rng.normal(size=s.U[k][reg].shape)
    from oracle.boundary import fill_faces
    fill_faces(s.U, g, s.flo)
    s.prim2cons()
    d0 = s.div_b().copy()
    s.rk_step(2e-3)
    err = np.max(np.abs(s.div_b() - d0))
    assert np.max(np.abs(d0)) > 1e-6
    assert err < 1e-9 * np.max(np.abs(d0)), (err, np.max(np.abs(d0)))
