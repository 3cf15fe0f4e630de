"""Pins of the oracle's lower-order fallback (Solver.apply_fallback).

  * the corrected face flux G = f - Delta^2 f/24 + 3 Delta^4 f/640 is the flux
    whose difference is the sixth-order staggered derivative: its difference
    equals fd.deriv of the same face data (and the fourth-order form's
    difference the fourth-order derivative);
  * a troubled zone's stage result is the first-order update: its six faces'
    first-order HLL fluxes, assembled here face by face from the pointwise
    physics, replace the high-order derivative (sources untouched);
  * the correction is conservative: on a periodic box the sums of D, S_i, tau
    over the zones are unchanged by it (the zone across the periodic boundary
    takes its share);
  * untroubled zones next to no troubled zone are untouched, and on smooth
    data nothing is troubled (the option then changes nothing);
  * on the 48 x 24 x 24 torus at its CFL step, where WENO5, MP5, MP7 and PLM
    leave failed inversions, the fallback leaves none; the same for the
    unmagnetised blast (pressure jump 3e4) on a 16 x 16 x 8 box;
  * translation invariance across the periodic boundaries: the blast
    centred on the box corner (its troubled zones on both sides of every
    periodic boundary) gives the centred blast's result rolled by half the
    box, bit for bit.
"""
import numpy as np
import pytest

from oracle import fd
from oracle.scheme import Solver, HYDRO, FACE_LOC, rk_combine
from oracle.boundary import fill_centred
from oracle.physics import state, flux, cons, speeds
from oracle.hll import hll_speeds, hll_flux
from workloads import box


@pytest.mark.parametrize("order", [6, 4])
def test_corrected_flux_difference_is_the_staggered_derivative(order):
    g, d = box.turbulent_box(12)
    s = Solver(g, deriv_order=order)
    rng = np.random.default_rng(71)
    f = rng.normal(size=g.shape)
    for dd in range(3):
        G = s.corrected_flux(f, dd)                   # faces -1/2 .. n-1/2
        ax, n = fd.AXIS[dd], g.n[dd]
        up, dn = [slice(None)] * 3, [slice(None)] * 3
        up[ax], dn[ax] = slice(1, n + 1), slice(0, n)
        diff = (G[tuple(up)] - G[tuple(dn)]) / g.dx[dd]
        ref = fd.deriv(f, dd, 0, n, g.dx[dd], g.ng, order)
        assert np.max(np.abs(diff - ref)) < 1e-12 * np.max(np.abs(ref))


def _setup(n=10):
    g, d = box.turbulent_box(n)
    s = Solver(g, fallback=True)
    s.curl_potential(d)
    s.set_primitives(d)
    fill_centred(s.P, s.grid)
    lh, lf, fdat, _ = s.rhs_parts()
    un = {k: s.interior(v).copy() for k, v in s.U.items()}
    return g, s, lh, fdat, un


def _face_flux_1st(s, d, kji_left):
    """First-order HLL hydro flux at the d-face between interior cell
    kji_left and its + neighbour, from the cells' primitives (ghosted arrays)."""
    g = s.g
    k, j, i = kji_left
    left = (k + g, j + g, i + g)
    right = list(left)
    right[fd.AXIS[d]] += 1
    right = tuple(right)
    m = {nm: v[0, j + g, i + g] for nm, v in s.met.loc[FACE_LOC[d]].items()}
    bn = s.U["Bf%d" % (d + 1)][left] / m["sqrtg"]
    sts = []
    for cell in (left, right):
        u = tuple(s.P["u%d" % (t + 1)][cell] for t in range(3))
        b = tuple(bn if t == d else s.P["B%d" % (t + 1)][cell] for t in range(3))
        sts.append(state(s.P["rho"][cell], u, s.P["p"][cell], b, m, s.gam))
    fl, fr = flux(sts[0], m, d), flux(sts[1], m, d)
    ul, ur = cons(sts[0], m), cons(sts[1], m)
    lpl, lml = speeds(sts[0], m, d, s.gam)
    lpr, lmr = speeds(sts[1], m, d, s.gam)
    ap, am = hll_speeds(np.float64(lpl), np.float64(lml), np.float64(lpr), np.float64(lmr))
    return [float(hll_flux(np.float64(fl[q]), np.float64(fr[q]), np.float64(ul[q]), np.float64(ur[q]), ap, am))
            for q in range(5)]


def test_troubled_zone_takes_the_first_order_update_and_sums_are_conserved():
    g, s, lh, fdat, un = _setup(10)
    a, b, dt = 0.75, 0.25, 2e-3
    cur = {k: un[k] * 1.0 for k in HYDRO}
    new = {k: rk_combine(un[k], cur[k], lh[k], a, b, dt) for k in HYDRO}
    # plant an unphysical result in one zone next to the periodic boundary
    # and in one zone in the middle (tau < 0; |S| > U)
    z1, z2 = (0, 4, 9), (5, 5, 5)
    new["tau"][z1] = -0.5 * new["D"][z1]
    new["S2"][z2] = 3.0 * (new["tau"][z2] + new["D"][z2])
    base = {k: v.copy() for k, v in new.items()}
    out = s.apply_fallback(new, fdat, b, dt)
    assert s.n_troubled == 2
    # conservative: the corrections telescope over the periodic box
    for k in HYDRO:
        assert abs(out[k].sum() - base[k].sum()) <= 1e-13 * np.sum(np.abs(base[k])), k
    # the troubled zones: the high-order divergence sum_d D_d F_d replaced by
    # the first-order one, -sum_d (F1_{m+1/2} - F1_{m-1/2}) / Delta_d
    for z in (z1, z2):
        for q, name in enumerate(HYDRO):
            lo = 0.0
            for d in range(3):
                ax, n = fd.AXIS[d], g.n[d]
                left = list(z)
                left[ax] = (z[ax] - 1) % n            # face m-1/2 is the + face of m-1
                lo -= (_face_flux_1st(s, d, z)[q] - _face_flux_1st(s, d, tuple(left))[q]) / g.dx[d]
            want = base[name][z] + b * dt * (lo + _ho_div(s, fdat, name, z))
            assert abs(out[name][z] - want) <= 1e-12 * max(1.0, abs(want)), (z, name, out[name][z], want)
    # a zone far from both troubled zones is untouched
    assert all(out[k][(8, 0, 3)] == base[k][(8, 0, 3)] for k in HYDRO)


def _ho_div(s, fdat, name, z):
    """sum_d D_d F_d at zone z (the high-order flux divergence), restated from
    the six faces with the staggered stencil."""
    k, j, i = z
    g = s.g
    tot = 0.0
    w = (3.0 / 640.0, -25.0 / 384.0, 75.0 / 64.0)
    for d in range(3):
        ax = fd.AXIS[d]
        F = fdat[d]["F_" + name]
        c = [k + g, j + g, i + g]
        def at(off):
            cc = list(c)
            cc[ax] += off
            return F[tuple(cc)]
        # faces m-5/2 .. m+5/2 are stored m-3 .. m+2
        dv = (w[2] * (at(0) - at(-1)) + w[1] * (at(1) - at(-2)) + w[0] * (at(2) - at(-3))) / s.grid.dx[d]
        tot += dv
    return tot


def test_smooth_data_has_no_troubled_zone_and_nothing_changes():
    g, d = box.turbulent_box(12)
    out = []
    for fb in (False, True):
        s = Solver(g, fallback=fb)
        s.curl_potential(d)
        s.set_primitives(d)
        for _ in range(3):
            s.rk_step()
        out.append(s)
    assert out[1].n_troubled == 0
    for k in HYDRO:
        assert np.array_equal(out[0].interior(out[0].U[k]), out[1].interior(out[1].U[k])), k


@pytest.mark.parametrize("recon", ["weno5", "mp5", "mp7", "plm"])
def test_fallback_removes_the_failed_inversions_on_the_coarse_torus(recon):
    from workloads.torus import torus
    g, d, tab = torus(48, 24, 24, ng=6 if recon == "mp7" else 5)
    res = {}
    for fb in (False, True):
        s = Solver(g, tab, recon=recon, fallback=fb)
        s.curl_potential(d)
        s.set_primitives(d)
        s.rk_step(s.cfl_dt())
        res[fb] = (sum(x["n_fail"] for x in s.last_stage_stats), s.n_troubled)
    assert res[False][0] > 0
    assert res[True][0] == 0 and res[True][1] > 0, res


@pytest.mark.parametrize("recon", ["weno5", "mp5"])
def test_fallback_removes_the_failed_inversions_in_the_blast(recon):
    g, d = box.blast_box((16, 16, 8), b0=0.0)
    res = {}
    for fb in (False, True):
        s = Solver(g, recon=recon, fallback=fb)
        s.set_face_fields(d)
        s.set_primitives(d)
        s.rk_step(s.cfl_dt())
        res[fb] = (sum(x["n_fail"] for x in s.last_stage_stats), s.n_troubled)
    assert res[False][0] > 0
    assert res[True][0] == 0 and res[True][1] > 0, res


def test_blast_on_the_corner_is_the_centred_blast_rolled():
    out = {}
    for name, c in (("centre", (0.5, 0.5, 0.5)), ("corner", (0.0, 0.0, 0.0))):
        g, d = box.blast_box((16, 16, 8), b0=0.0, centre=c)
        s = Solver(g, recon="mp5", fallback=True)
        s.set_face_fields(d)
        s.set_primitives(d)
        s.rk_step(2.0e-3)
        out[name] = (s, s.n_troubled)
    assert out["corner"][1] == out["centre"][1] > 0
    sc, sk = out["centre"][0], out["corner"][0]
    for k in HYDRO:
        rolled = np.roll(sc.interior(sc.U[k]), (4, 8, 8), axis=(0, 1, 2))
        assert np.array_equal(sk.interior(sk.U[k]), rolled), k


def test_first_order_flux_through_the_polar_axis_is_zero():
    """The first-order flux at the x^2 faces on the polar axis (sqrt(gamma)
    = 0 there: the faces have no area) is 0, as the high-order one is; the
    faces next to them carry flux."""
    from workloads.torus import torus
    g, d, tab = torus(24, 12, 12)
    s = Solver(g, tab, fallback=True)
    s.curl_potential(d)
    s.set_primitives(d)
    from oracle.boundary import fill_centred
    fill_centred(s.P, s.grid)
    f1 = s.first_order_face_fluxes(1)             # faces -1/2 .. n2-1/2 (stored -1 .. n2-1)
    n2 = g.n[1]
    for name, v in f1.items():
        assert np.all(v[:, 0, :] == 0.0) and np.all(v[:, n2, :] == 0.0), name
    assert np.max(np.abs(f1["D"][:, 1:n2, :])) > 0.0
