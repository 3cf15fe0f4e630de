"""RHS assembly, constrained transport, SSP-RK3 and CFL step (oracle, FP64).

Paper, Introduction: 3-D finite differences with high-order reconstruction,
after ECHO.  One right-hand-side evaluation, in order:
  1. ghost fill of the 8 centred primitives;
  2. for each direction d: MP5 states of rho, p, u^1..3 and the two
     transverse centred B at d-faces f in [-3, n_d + 1] (the faces the
     sixth-order derivative of the edges and fluxes reads; [-2, n_d] for the
     fourth-order one) over the whole transverse ghosted range (reconstructed rho and p are kept at or above
     0.1 times the cell value on their side); normal B = B_face / sqrt(gamma_face);
     pointwise fluxes, conserved variables and speeds of both states; HLL
     flux (0 on faces where sqrt(gamma) = 0); the per-face data for the
     edge field: v^d and v^c (c = d+1 mod 3) of both states and a+-;
  3. edge fields (upwind constrained transport, Londrillo & Del Zanna 2004),
     family e with d = e+1, c = e+2 (mod 3), at edges offset by 1/2 in d
     and c:
       - v^d, v^c of both d-face states and B^d (d-faces) reconstructed
         along c with MP5 (side b), B^c (c-faces) along d (side a);
       - vt = alpha_edge v - beta_edge; E^{ab} = vt^c_{ab} B^{d,b} - vt^d_{ab} B^{c,a};
       - a_d^pm = max over the two d-faces next to the edge, a_c^pm likewise;
       - E_e = sum_ab w^d_a w^c_b E^{ab} + a_d^+ a_d^-/(a_d^+ + a_d^-) (B^{c,R} - B^{c,L})
               - a_c^+ a_c^-/(a_c^+ + a_c^-) (B^{d,R} - B^{d,L}),
         w_L = a^+/(a^+ + a^-), w_R = a^-/(a^+ + a^-) (1/2 and 0 if a^+ + a^- < 1e-300);
     On a polar-axis boundary the edges on the axis (families 1 and 3,
     stored x^2 index -1 and n2-1) are 0: the covariant field there carries
     sqrt(gamma) = 0.
  4. L[hydro] = -sum_d D_d F_d + s (metric sources) at interior cells;
     L[B^n] = -D_{n+1} E_{n+2} + D_{n+2} E_{n+1} at owned faces (indices mod 3)
     and, normal to a non-periodic boundary, at the ghost faces the
     staggered derivative of an interior cell reads (Solver.face_region), so
     that the discrete div B of every interior cell keeps its value; the
     boundary rule fills only the faces beyond those.
SSP-RK3 (Shu & Osher 1988): U^(s) = a_s U^n + b_s (U^(s-1) + dt L(U^(s-1)))
with (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3), every stage followed by the
ghost fill of the face fields and the inversion (with floors) at interior
cells.

Lower-order fallback (option, off by default): the flux derivative is the
difference of corrected face fluxes, D f = (G_{m+1/2} - G_{m-1/2}) / Delta
with G = f - Delta^2 f / 24 + 3 Delta^4 f / 640 (sixth order; the fourth
keeps the first correction).  After a stage's combination, an interior zone
whose hydro state is unphysical -- D <= 0, tau <= 0 or S^2 >= (tau + D)^2
(undensitised, S^2 with the inverse 3-metric) -- is troubled; at every face
next to a troubled zone G is replaced by the first-order HLL flux of the two
cells' states (the stage's primitives, face metric, normal face field; 0
where sqrt(gamma) = 0), and both zones sharing the face take the
difference: U_m -= b dt (F1 - G)/Delta, U_{m+1} += b dt (F1 - G)/Delta
(conservative).  Neighbours across a periodic boundary are the zones at the
other end; ghost zones are not corrected.  Applied once per stage.  dt = C / max_cells sum_d max(|lambda+_d|, |lambda-_d|)/Delta_d from
P^n with the centre metric.
"""
import math
import numpy as np

from . import fd
from .fd import take, deriv, interp
from .recon import face_states, METHODS as RECON_METHODS, NG_OF
from .physics import state, flux, cons, speeds, prim2cons
from .hll import hll_speeds, hll_flux
from .c2p import newton, warm_guess
from .boundary import fill_centred, fill_faces, AXIS as AXIS_BC
from .sources import sources

PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
HYDRO = ("D", "S1", "S2", "S3", "tau")
FACE = ("Bf1", "Bf2", "Bf3")
LOCS = ("C", "F1", "F2", "E3")
GEOM = ("alpha", "beta1", "beta2", "beta3", "g11", "g12", "g13", "g22", "g23", "g33",
        "gu11", "gu12", "gu13", "gu22", "gu23", "gu33", "sqrtg")
DERIV = (["d1_alpha", "d2_alpha", "d1_beta1", "d1_beta2", "d1_beta3",
          "d2_beta1", "d2_beta2", "d2_beta3"]
         + ["d1_" + c for c in ("g11", "g12", "g13", "g22", "g23", "g33")]
         + ["d2_" + c for c in ("g11", "g12", "g13", "g22", "g23", "g33")])
POS_FRAC = 0.1                   # positivity bound of reconstructed rho, p
FACE_LOC = ("F1", "F2", "C")     # metric location of d-faces
EDGE_LOC = ("F2", "F1", "E3")    # metric location of edge family e


class Metric:
    """Metric tables as {loc: {name: array (1, N2, N1)}} plus centre
    derivatives; parsed from the documented table layout."""

    def __init__(self, tables):
        t = np.asarray(tables, dtype=np.float64)
        assert t.shape[0] == 4 * len(GEOM) + len(DERIV)
        self.loc = {}
        for li, loc in enumerate(LOCS):
            self.loc[loc] = {nm: t[li * len(GEOM) + q][None]
                             for q, nm in enumerate(GEOM)}
        base = 4 * len(GEOM)
        self.der = {nm: t[base + q][None] for q, nm in enumerate(DERIV)}

    @staticmethod
    def sel(m, d, lo, hi, g):
        """Restrict a location dict along direction d (x^3 is broadcast)."""
        if d == 2:
            return m
        return {k: take(v, d, lo, hi, g) for k, v in m.items()}

    @staticmethod
    def interior(m, g):
        return {k: v[:, g:-g, g:-g] for k, v in m.items()}


def minkowski_tables(grid):
    g = grid.ng
    t = np.zeros((4 * len(GEOM) + len(DERIV), grid.n[1] + 2 * g, grid.n[0] + 2 * g))
    for li in range(4):
        for nm in ("alpha", "g11", "g22", "g33", "gu11", "gu22", "gu33", "sqrtg"):
            t[li * len(GEOM) + GEOM.index(nm)] = 1.0
    return t


SSPRK3 = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk_combine(un, u, l, a, b, dt):
    """One SSP-RK3 stage: a U^n + b (U + dt L)."""
    return a * un + b * (u + dt * l)


def _nan(shape):
    return np.full(shape, np.nan)


class Solver:
    """precision: "fp64", or "fp32" for the precision form in which the
    reconstruction, face physics, HLL flux and edge field are evaluated in
    float32 from float32-rounded inputs and widened to float64 afterwards
    (derivatives, sources, RK combine and inversion stay float64).
    recon: interface reconstruction, "mp5" (default), "weno5", "plm" or
    "mp7" (the last on grids with six ghost layers).
    deriv_order: order of the staggered derivative and interpolation, 6
    (default) or 4; one order serves the flux derivative, the induction
    equation, the curl of the vector potential, the centred field and div B,
    so the discrete div B stays zero.
    fallback: the lower-order fallback at the faces of troubled zones (module
    docstring); n_troubled counts the troubled zones over all stages."""

    def __init__(self, grid, tables=None, precision="fp64", recon="mp5", deriv_order=6,
                 fallback=False):
        if recon not in RECON_METHODS:
            raise ValueError("unknown reconstruction %r" % (recon,))
        if deriv_order not in (4, 6):
            raise ValueError("deriv_order must be 4 or 6")
        # faces and edges are formed from -flo to n + flo - 2 along their
        # offset directions (the stored indices the staggered derivative reads
        # at the interior: 3 and 2 below and above for the sixth order, 2 and
        # 1 for the fourth); a face reads cells down to flo plus the
        # reconstruction's reach below it (NG_OF is that for the sixth order)
        self.flo = 3 if deriv_order == 6 else 2
        need = NG_OF[recon] - 3 + self.flo
        if grid.ng < need:
            raise ValueError("%s with deriv_order %d needs %d ghost layers" % (recon, deriv_order, need))
        self.recon = recon
        self.order = deriv_order
        self.fallback = fallback
        self.n_troubled = 0
        self.grid = grid
        self.ftype = np.float32 if precision == "fp32" else np.float64
        self.g = grid.ng
        self.gam = grid.gamma_ad
        self.met = Metric(minkowski_tables(grid) if tables is None else tables)
        shp = grid.shape
        self.P = {k: _nan(shp) for k in PRIM}
        self.U = {k: _nan(shp) for k in HYDRO + FACE}
        self.stats = {}
        # radius at centres (interior), for the floors
        g = self.g
        if grid.coord == 1:
            x1 = grid.x0[0] + (np.arange(grid.n[0]) + 0.5) * grid.dx[0]
            self.r_int = np.exp(x1)[None, None, :]
        else:
            self.r_int = None

    # ---------------------------------------------------------- helpers
    def interior(self, a):
        return fd.interior(a, self.g)

    def set_interior(self, a, val):
        g = self.g
        a[g:-g, g:-g, g:-g] = val

    def centre_metric(self):
        return Metric.interior(self.met.loc["C"], self.g)

    # ---------------------------------------------------------- initial data
    def curl_potential(self, A):
        """B_face = curl_D A at the evolved faces (face_region):
        B^n = D_{n+1} A_{n+2} - D_{n+2} A_{n+1}."""
        g, gr = self.g, self.grid
        for nd in range(3):
            d1, d2 = (nd + 1) % 3, (nd + 2) % 3
            t1 = deriv(A["A%d" % (d2 + 1)], d1, 0, gr.n[d1], gr.dx[d1], g, self.order)
            t2 = deriv(A["A%d" % (d1 + 1)], d2, 0, gr.n[d2], gr.dx[d2], g, self.order)
            f = _nan(gr.shape)
            f[self.face_region(nd)] = (self._restrict_face(t1, d1, nd)
                                       - self._restrict_face(t2, d2, nd))
            self.U["Bf%d" % (nd + 1)] = f
        fill_faces(self.U, gr, self.flo)

    def face_region(self, nd):
        """Slices (of a full array) of the faces of the face field normal to
        nd that the scheme evolves: interior in the other two directions;
        along nd the owned faces 0 .. n-1, and where nd is not periodic also
        the ghost faces -flo .. -1 and n .. n + flo - 2 that the staggered
        derivative of an interior cell reads."""
        g, gr = self.g, self.grid
        sl = [slice(g, g + gr.n[t]) for t in (2, 1, 0)]
        if gr.bc[2 * nd] != 0:
            sl[fd.AXIS[nd]] = slice(g - self.flo, g + gr.n[nd] + self.flo - 1)
        return tuple(sl)

    def _restrict_face(self, a, d, nd):
        """Restrict a derivative along d (interior along d, full along the
        others) to face_region(nd)."""
        g, gr = self.g, self.grid
        reg = self.face_region(nd)
        sl = [slice(None)] * 3
        for t in range(3):
            if t != d:
                sl[fd.AXIS[t]] = reg[fd.AXIS[t]]
        return a[tuple(sl)]

    def set_face_fields(self, data):
        for k in FACE:
            self.U[k] = np.array(data["B%sf" % k[-1]], dtype=np.float64)
        fill_faces(self.U, self.grid, self.flo)

    def centred_b(self):
        """B^i = I_i(B_face^i) / sqrt(gamma) at interior cells."""
        g, gr = self.g, self.grid
        sg = self.centre_metric()["sqrtg"]
        out = []
        for d in range(3):
            bi = interp(self.U["Bf%d" % (d + 1)], d, 0, gr.n[d], g, self.order)
            bi = _restrict_others(bi, d, g, gr)
            out.append(bi / sg)
        return out

    def set_primitives(self, data):
        """Interior rho, u^i, p from data; B from the face fields; U from P."""
        for k in ("rho", "u1", "u2", "u3", "p"):
            self.set_interior(self.P[k], data[k])
        self.prim2cons()

    def prim2cons(self):
        b = self.centred_b()
        for i in range(3):
            self.set_interior(self.P["B%d" % (i + 1)], b[i])
        P = {k: self.interior(v) for k, v in self.P.items()}
        c = prim2cons(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"], tuple(b),
                      self.centre_metric(), self.gam)
        for k, v in zip(HYDRO, c):
            self.set_interior(self.U[k], v)
        fill_centred(self.P, self.grid)

    # ---------------------------------------------------------- RHS pieces
    def sweep(self, d):
        g, gr, gam = self.g, self.grid, self.gam
        n = gr.n[d]
        lo, hi = -self.flo, n + self.flo - 1
        c = (d + 1) % 3
        ft = self.ftype
        P = {k: v.astype(ft) for k, v in self.P.items()}
        gam = ft(gam)
        rec = {}
        for k in ("rho", "p", "u1", "u2", "u3"):
            rec[k] = face_states(P[k], d, lo, hi, g, take, self.recon)
        # positivity: a reconstructed rho or p is kept at or above a tenth of
        # the value of the cell on its side of the face (continuous bound)
        for k in ("rho", "p"):
            l, r = rec[k]
            cj = take(P[k], d, lo, hi, g)
            cj1 = take(P[k], d, lo + 1, hi + 1, g)
            rec[k] = (np.maximum(l, ft(POS_FRAC) * cj), np.maximum(r, ft(POS_FRAC) * cj1))
        for t in range(3):
            if t != d:
                rec["B%d" % (t + 1)] = face_states(P["B%d" % (t + 1)], d, lo, hi, g, take, self.recon)
        mf = {k: v.astype(ft) for k, v in Metric.sel(self.met.loc[FACE_LOC[d]], d, lo, hi, g).items()}
        sg = mf["sqrtg"]
        bn_face = take(self.U["Bf%d" % (d + 1)], d, lo, hi, g).astype(ft)
        with np.errstate(divide="ignore", invalid="ignore"):
            bn = np.where(sg != 0.0, bn_face / np.where(sg != 0.0, sg, ft(1.0)), ft(0.0))
        sts = []
        for side in (0, 1):
            u = tuple(rec["u%d" % (t + 1)][side] for t in range(3))
            b = tuple(bn if t == d else rec["B%d" % (t + 1)][side] for t in range(3))
            sts.append(state(rec["rho"][side], u, rec["p"][side], b, mf, gam))
        with np.errstate(divide="ignore", invalid="ignore"):
            fl, fr = flux(sts[0], mf, d), flux(sts[1], mf, d)
            ul, ur = cons(sts[0], mf), cons(sts[1], mf)
        lpl, lml = speeds(sts[0], mf, d, gam)
        lpr, lmr = speeds(sts[1], mf, d, gam)
        ap, am = hll_speeds(lpl, lml, lpr, lmr)
        axis = np.broadcast_to(sg == 0.0, ap.shape)
        out = {}
        with np.errstate(divide="ignore", invalid="ignore"):
            for q, name in enumerate(HYDRO):
                fh = hll_flux(fl[q], fr[q], ul[q], ur[q], ap, am)
                out["F_" + name] = np.where(axis, 0.0, fh)
        out["vdL"], out["vdR"] = sts[0]["v"][d], sts[1]["v"][d]
        out["vcL"], out["vcR"] = sts[0]["v"][c], sts[1]["v"][c]
        out["ap"], out["am"] = ap, am
        full = {}
        for k, v in out.items():
            a = _nan(gr.shape)
            fd.put(a, d, lo, hi, g, np.broadcast_to(v, take(a, d, lo, hi, g).shape).astype(np.float64))
            full[k] = a
        return full

    def edge(self, e, fdat):
        """Edge field E_e from the face data of the d and c sweeps."""
        g, gr = self.g, self.grid
        d, c = (e + 1) % 3, (e + 2) % 3
        nd, nc = gr.n[d], gr.n[c]
        ft = self.ftype
        D = {k: v.astype(ft) for k, v in fdat[d].items()}
        C = {k: v.astype(ft) for k, v in fdat[c].items()}
        UB = {k: self.U[k].astype(ft) for k in FACE}
        lo, hd, hc = -self.flo, nd + self.flo - 1, nc + self.flo - 1
        # reconstruct d-face data along c to the edge (side b)
        def along_c(q):
            l, r = face_states(q, c, lo, hc, g, take, self.recon)
            return take(l, d, lo, hd, g), take(r, d, lo, hd, g)
        vd = {("L", b): x for b, x in zip("LR", along_c(D["vdL"]))}
        vd.update({("R", b): x for b, x in zip("LR", along_c(D["vdR"]))})
        vc = {("L", b): x for b, x in zip("LR", along_c(D["vcL"]))}
        vc.update({("R", b): x for b, x in zip("LR", along_c(D["vcR"]))})
        bd = dict(zip("LR", along_c(UB["Bf%d" % (d + 1)])))
        # reconstruct B^c (c-faces) along d (side a)
        l, r = face_states(UB["Bf%d" % (c + 1)], d, lo, hd, g, take, self.recon)
        bc = {"L": take(l, c, lo, hc, g), "R": take(r, c, lo, hc, g)}
        # speeds: max over the two faces adjacent to the edge
        def adj(q, along, other, h_along, h_other):
            x0 = take(q, along, lo, h_along, g)
            x1 = take(q, along, lo + 1, h_along + 1, g)
            m = np.maximum(x0, x1)
            return take(m, other, lo, h_other, g)
        apd = adj(D["ap"], c, d, hc, hd)
        amd = adj(D["am"], c, d, hc, hd)
        apc = adj(C["ap"], d, c, hd, hc)
        amc = adj(C["am"], d, c, hd, hc)
        me = Metric.sel(Metric.sel(self.met.loc[EDGE_LOC[e]], d, lo, hd, g),
                        c, lo, hc, g)
        me = {k: v.astype(ft) for k, v in me.items()}
        al = me["alpha"]
        betd, betc = me["beta%d" % (d + 1)], me["beta%d" % (c + 1)]
        with np.errstate(divide="ignore", invalid="ignore"):
            sd = apd + amd
            sc = apc + amc
            tiny = ft(1e-300) if ft == np.float64 else ft(1e-37)
            tiny_d, tiny_c = sd < tiny, sc < tiny
            half, zero = ft(0.5), ft(0.0)
            wd = {"L": np.where(tiny_d, half, apd / sd), "R": np.where(tiny_d, half, amd / sd)}
            wc = {"L": np.where(tiny_c, half, apc / sc), "R": np.where(tiny_c, half, amc / sc)}
            kd = np.where(tiny_d, zero, apd * amd / sd)
            kc = np.where(tiny_c, zero, apc * amc / sc)
        ee = ft(0.0)
        for a_ in "LR":
            for b_ in "LR":
                vtd = al * vd[(a_, b_)] - betd
                vtc = al * vc[(a_, b_)] - betc
                eab = vtc * bd[b_] - vtd * bc[a_]
                ee = ee + wd[a_] * wc[b_] * eab
        ee = ee + kd * (bc["R"] - bc["L"]) - kc * (bd["R"] - bd["L"])
        out = _nan(gr.shape)
        sl = [slice(None)] * 3
        sl[fd.AXIS[d]] = slice(lo + g, hd + g)
        sl[fd.AXIS[c]] = slice(lo + g, hc + g)
        out[tuple(sl)] = np.asarray(ee, dtype=np.float64)
        if gr.bc[2] == AXIS_BC and e != 1:
            # edges on the polar axis (x^2 offset, stored -1 and n2-1): the
            # covariant field there carries sqrt(gamma) = 0
            n2 = gr.n[1]
            out[:, g - 1, :] = 0.0
            out[:, g + n2 - 1, :] = 0.0
        return out

    def rhs_parts(self):
        """Returns (L_hydro dict at interior cells, L_face dict at owned faces,
        face data, edges).  P ghosts must be filled."""
        g, gr = self.g, self.grid
        fdat = [self.sweep(d) for d in range(3)]
        edges = [self.edge(e, fdat) for e in range(3)]
        lh = {}
        for name in HYDRO:
            tot = 0.0
            for d in range(3):
                t = deriv(fdat[d]["F_" + name], d, 0, gr.n[d], gr.dx[d], g, self.order)
                tot = tot - _restrict_others(t, d, g, gr)
            lh[name] = tot
        src = sources({k: self.interior(v) for k, v in self.P.items()},
                      self.centre_metric(), Metric.interior(self.met.der, g), self.gam)
        for name in HYDRO:
            lh[name] = lh[name] + src[name]
        # the face fields over face_region (the owned faces and, normal to a
        # non-periodic boundary, the ghost faces the divergence reads)
        lf = {}
        for nd in range(3):
            d1, d2 = (nd + 1) % 3, (nd + 2) % 3
            t1 = self._restrict_face(deriv(edges[d2], d1, 0, gr.n[d1], gr.dx[d1], g, self.order), d1, nd)
            t2 = self._restrict_face(deriv(edges[d1], d2, 0, gr.n[d2], gr.dx[d2], g, self.order), d2, nd)
            lf["Bf%d" % (nd + 1)] = -t1 + t2
        return lh, lf, fdat, edges

    def owned(self, lf, nd):
        """The owned faces (stored 0 .. n-1 along nd) of a face_region array."""
        gr = self.grid
        if gr.bc[2 * nd] == 0:
            return lf
        sl = [slice(None)] * 3
        sl[fd.AXIS[nd]] = slice(self.flo, self.flo + gr.n[nd])
        return lf[tuple(sl)]

    def rhs(self):
        fill_centred(self.P, self.grid)
        lh, lf, _, _ = self.rhs_parts()
        out = dict(lh)
        for nd, name in enumerate(FACE):
            out[name] = self.owned(lf[name], nd)
        return out

    # ---------------------------------------------------------- inversion
    def cons2prim(self, guess="warm"):
        g, gr, gam = self.g, self.grid, self.gam
        m = self.centre_metric()
        b = self.centred_b()
        sg = m["sqrtg"]
        U = {k: self.interior(v) for k, v in self.U.items()}
        P = {k: self.interior(v) for k, v in self.P.items()}
        dd, tau = U["D"] / sg, U["tau"] / sg
        s = (U["S1"] / sg, U["S2"] / sg, U["S3"] / sg)
        if guess == "warm":
            y0 = warm_guess(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"], m, gam)
        else:
            y0 = gam * (tau + dd)
        res = newton(dd, s, tau, b, m, gam, y0, tol=gr.newton_tol, maxit=gr.newton_maxit)
        ok = res["ok"]
        rho = np.where(ok, res["rho"], P["rho"])
        p = np.where(ok, res["p"], P["p"])
        u = [np.where(ok, res["u"][i], P["u%d" % (i + 1)]) for i in range(3)]
        nfl_rho = nfl_p = nwcap = 0
        floored = np.zeros(ok.shape, dtype=bool)
        if gr.rho_fl_a > 0.0 or gr.p_fl_a > 0.0 or gr.w_max > 0.0:
            r = self.r_int if self.r_int is not None else 1.0
            # a failed zone becomes atmosphere: floor density and pressure, at rest
            rho = np.where(ok, rho, gr.rho_fl_a * r ** gr.rho_fl_n)
            p = np.where(ok, p, gr.p_fl_a * r ** gr.p_fl_n)
            u = [np.where(ok, x, 0.0) for x in u]
            floored |= ~ok
            if gr.rho_fl_a > 0.0:
                rfl = gr.rho_fl_a * r ** gr.rho_fl_n
                low = rho < rfl
                rho = np.where(low, rfl, rho)
                floored |= low
                nfl_rho = int(low.sum())
            if gr.p_fl_a > 0.0:
                pfl = gr.p_fl_a * r ** gr.p_fl_n
                low = p < pfl
                p = np.where(low, pfl, p)
                floored |= low
                nfl_p = int(low.sum())
            if gr.w_max > 0.0:
                from .physics import lower
                ul = lower(m, tuple(u))
                uu = ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2]
                wcur = np.sqrt(1.0 + uu)
                cap = wcur > gr.w_max
                fac = np.sqrt((gr.w_max ** 2 - 1.0) / np.where(cap, uu, 1.0))
                u = [np.where(cap, fac * x, x) for x in u]
                floored |= cap
                nwcap = int(cap.sum())
        vals = {"rho": rho, "u1": u[0], "u2": u[1], "u3": u[2], "p": p,
                "B1": b[0], "B2": b[1], "B3": b[2]}
        for k, v in vals.items():
            self.set_interior(self.P[k], np.broadcast_to(v, ok.shape))
        if floored.any():
            c = prim2cons(rho, tuple(u), p, tuple(b), m, gam)
            for k, v in zip(HYDRO, c):
                self.set_interior(self.U[k], np.where(floored, v, U[k]))
        it = res["iters"]
        self.stats = {"n_fail": int((~ok).sum()), "iters_sum": int(it.sum()),
                      "iters_max": int(it.max()) if it.size else 0,
                      "n_floor_rho": nfl_rho, "n_floor_p": nfl_p, "n_wcap": nwcap}
        return self.stats

    # ---------------------------------------------------------- time step
    def cfl_dt(self):
        gr, gam = self.grid, self.gam
        m = self.centre_metric()
        P = {k: self.interior(v) for k, v in self.P.items()}
        st = state(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"],
                   (P["B1"], P["B2"], P["B3"]), m, gam)
        tot = 0.0
        for d in range(3):
            lp, lm = speeds(st, m, d, gam)
            tot = tot + np.maximum(np.abs(lp), np.abs(lm)) / gr.dx[d]
        return gr.cfl / float(np.max(tot))

    # ---------------------------------------------------------- fallback
    def first_order_face_fluxes(self, d):
        """First-order HLL hydro fluxes at the d-faces -1/2 .. n-1/2 (stored
        -1 .. n-1) from the states of the two cells beside each face."""
        g, gr, gam = self.g, self.grid, self.gam
        n = gr.n[d]
        lo, hi = -1, n
        rec = {k: (take(self.P[k], d, lo, hi, g), take(self.P[k], d, lo + 1, hi + 1, g))
               for k in PRIM}
        mf = Metric.sel(self.met.loc[FACE_LOC[d]], d, lo, hi, g)
        sg = mf["sqrtg"]
        bn_face = take(self.U["Bf%d" % (d + 1)], d, lo, hi, g)
        with np.errstate(divide="ignore", invalid="ignore"):
            bn = np.where(sg != 0.0, bn_face / np.where(sg != 0.0, sg, 1.0), 0.0)
        sts = []
        for side in (0, 1):
            u = tuple(rec["u%d" % (t + 1)][side] for t in range(3))
            b = tuple(bn if t == d else rec["B%d" % (t + 1)][side] for t in range(3))
            sts.append(state(rec["rho"][side], u, rec["p"][side], b, mf, gam))
        with np.errstate(divide="ignore", invalid="ignore"):
            fl, fr = flux(sts[0], mf, d), flux(sts[1], mf, d)
            ul, ur = cons(sts[0], mf), cons(sts[1], mf)
        lpl, lml = speeds(sts[0], mf, d, gam)
        lpr, lmr = speeds(sts[1], mf, d, gam)
        ap, am = hll_speeds(lpl, lml, lpr, lmr)
        axis = np.broadcast_to(sg == 0.0, ap.shape)
        out = {}
        with np.errstate(divide="ignore", invalid="ignore"):
            for q, name in enumerate(HYDRO):
                out[name] = np.where(axis, 0.0, hll_flux(fl[q], fr[q], ul[q], ur[q], ap, am))
        return out

    def troubled(self, new):
        """Interior zones whose hydro state `new` (densitised) is unphysical."""
        from .physics import raise_
        m = self.centre_metric()
        sg = m["sqrtg"]
        dd, tau = new["D"] / sg, new["tau"] / sg
        s = (new["S1"] / sg, new["S2"] / sg, new["S3"] / sg)
        su = raise_(m, s)
        s2 = s[0] * su[0] + s[1] * su[1] + s[2] * su[2]
        return (dd <= 0.0) | (tau <= 0.0) | (s2 >= (tau + dd) ** 2)

    def corrected_flux(self, f, d):
        """G at the d-faces -1/2 .. n-1/2 from the face fluxes f."""
        g, n = self.g, self.grid.n[d]
        t = lambda s: take(f, d, -1 + s, n + s, g)
        if self.order == 4:
            return t(0) - (t(1) - 2.0 * t(0) + t(-1)) / 24.0
        return (t(0) - (t(1) - 2.0 * t(0) + t(-1)) / 24.0
                + 3.0 * (t(2) - 4.0 * t(1) + 6.0 * t(0) - 4.0 * t(-1) + t(-2)) / 640.0)

    def apply_fallback(self, new, fdat, b, dt):
        g, gr = self.g, self.grid
        bad = self.troubled(new)
        self.n_troubled += int(bad.sum())
        if not bad.any():
            return new
        out = dict(new)
        for d in range(3):
            ax, n = fd.AXIS[d], gr.n[d]
            periodic = gr.bc[2 * d] == 0
            widths = [(1, 1) if a_ == ax else (0, 0) for a_ in range(3)]
            pad = np.pad(bad, widths, mode="wrap") if periodic else np.pad(bad, widths, constant_values=False)
            lo_sl, hi_sl = [slice(None)] * 3, [slice(None)] * 3
            lo_sl[ax], hi_sl[ax] = slice(0, n + 1), slice(1, n + 2)
            face_bad = pad[tuple(lo_sl)] | pad[tuple(hi_sl)]        # faces -1/2 .. n-1/2
            f1 = self.first_order_face_fluxes(d)
            for name in HYDRO:
                G = _restrict_others(self.corrected_flux(fdat[d]["F_" + name], d), d, g, gr)
                F1 = _restrict_others(f1[name], d, g, gr)
                delta = np.where(face_bad, F1 - G, 0.0)
                up, dn = [slice(None)] * 3, [slice(None)] * 3
                up[ax], dn[ax] = slice(1, n + 1), slice(0, n)
                out[name] = out[name] - b * dt * (delta[tuple(up)] - delta[tuple(dn)]) / gr.dx[d]
        return out

    def stage(self, un, a, b, dt):
        g = self.g
        fill_centred(self.P, self.grid)
        lh, lf, fdat, _ = self.rhs_parts()
        new = {name: rk_combine(self.interior(un[name]), self.interior(self.U[name]), lh[name], a, b, dt)
               for name in HYDRO}
        if self.fallback:
            new = self.apply_fallback(new, fdat, b, dt)
        for name in HYDRO:
            self.set_interior(self.U[name], new[name])
        for nd, name in enumerate(FACE):
            reg = self.face_region(nd)
            self.U[name][reg] = rk_combine(un[name][reg], self.U[name][reg], lf[name], a, b, dt)
        fill_faces(self.U, self.grid, self.flo)
        return self.cons2prim()

    def rk_step(self, dt=None):
        if dt is None or dt <= 0.0:
            dt = self.cfl_dt()
        un = {k: v.copy() for k, v in self.U.items()}
        stats = []
        for a, b in SSPRK3:
            stats.append(self.stage(un, a, b, dt))
        self.last_stage_stats = stats
        return dt

    # ---------------------------------------------------------- diagnostics
    def div_b(self):
        g, gr = self.g, self.grid
        tot = 0.0
        for d in range(3):
            t = deriv(self.U["Bf%d" % (d + 1)], d, 0, gr.n[d], gr.dx[d], g, self.order)
            tot = tot + _restrict_others(t, d, g, gr)
        return tot

    def diagnostics(self):
        """Monitoring values of the current state (interior cells; owned faces
        for the face fields): plain sums of the 8 conserved fields; the
        largest |div_D B| and that value times min(dx) over the largest field
        strength; extrema of rho and p; the largest Lorentz factor
        W = sqrt(1 + u_i u^i) and field strength |B| = sqrt(B_i B^i) with the
        centre metric; the number of non-finite interior primitives.  Extrema
        skip NaN values."""
        from .physics import lower
        out = {}
        for k in HYDRO + FACE:
            out["sum_" + k] = float(np.sum(self.interior(self.U[k])))
        dv = self.div_b()
        out["max_divb"] = float(np.max(np.abs(dv)))
        P = {k: self.interior(v) for k, v in self.P.items()}
        out["rho_min"], out["rho_max"] = float(np.nanmin(P["rho"])), float(np.nanmax(P["rho"]))
        out["p_min"], out["p_max"] = float(np.nanmin(P["p"])), float(np.nanmax(P["p"]))
        m = self.centre_metric()
        u = (P["u1"], P["u2"], P["u3"])
        b = (P["B1"], P["B2"], P["B3"])
        ul, bl = lower(m, u), lower(m, b)
        w = np.sqrt(1.0 + ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2])
        bmag = np.sqrt(np.maximum(bl[0] * b[0] + bl[1] * b[1] + bl[2] * b[2], 0.0))
        out["w_max"] = float(np.nanmax(w))
        out["b_max"] = float(np.nanmax(bmag))
        out["max_divb_norm"] = (out["max_divb"] * min(self.grid.dx) / out["b_max"]
                                if out["b_max"] > 0.0 else 0.0)
        out["n_nonfinite"] = int(sum(int((~np.isfinite(v)).sum()) for v in P.values()))
        return out


def _restrict_others(a, d, g, grid):
    """Restrict an array that is interior along d to the interior along the
    other two directions."""
    sl = [slice(None)] * 3
    for t in range(3):
        if t != d:
            n = grid.n[t]
            ax = fd.AXIS[t]
            if a.shape[ax] == 1:
                continue
            sl[ax] = slice(g, g + n)
    return a[tuple(sl)]


def new_solver(grid, tables=None):
    return Solver(grid, tables)
