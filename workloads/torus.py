"""Thick accretion torus around a Kerr black hole (Kerr-Schild background).

Constant specific angular momentum torus (Abramowicz, Jaroszynski & Sikora
1978; Font & Daigne 2002), the setup of the paper's Figure 1 use case:
  * l = l_K(r_max), l_K(r) = (r^2 - 2 a sqrt(r) + a^2)/(r^1.5 - 2 sqrt(r) + a);
  * Boyer-Lindquist u_t = -[(g_tphi^2 - g_tt g_phiphi)/(g_phiphi + 2 l g_tphi
    + l^2 g_tt)]^(1/2), enthalpy h = u_t(r_in, pi/2) / u_t(r, theta);
    the torus is where h > 1 (and r >= r_in);
  * polytrope p = K rho^Gamma with K set so that max rho = 1;
  * u^r = u^theta = 0, so u^t and u^phi are the same in BL and KS; with the
    KS lapse the Eulerian Lorentz factor is W = alpha u^t and the primitive
    u^i = W v^i is (u^t beta^1, 0, u^phi);
  * seeded density noise rho <- rho (1 + 0.02 xi), xi ~ U(-1, 1), inside;
  * loop field from A_phi = max(rho_bar - 0.2, 0) on the x^3 edges
    (rho_bar: noise-free density / max), scaled so that
    max p / max(b^2/2) = 100, with b^2 estimated from centred second-order
    differences of A_phi (a normalisation recipe only);
  * atmosphere outside: rho = rho_fl, p = p_fl, u = 0, with the floors
    rho_fl = 1e-4 r^-1.5, p_fl = 1e-6 r^-2.5 also used by the scheme.
"""
import numpy as np

from .grid import torus_grid
from .metric import kerr_schild_tables, comp_index

SEED = 1810
R_IN = 6.0
R_MAX = 10.0
SPIN = 0.9
BETA = 100.0
NOISE = 0.02
RHO_FL = (1e-4, -1.5)
P_FL = (1e-6, -2.5)
W_MAX = 10.0


def ell_kepler(r, a):
    sr = np.sqrt(r)
    return (r * r - 2.0 * a * sr + a * a) / (r * sr - 2.0 * sr + a)


def _ut_bl(r, th, a, ell):
    s2 = np.sin(th) ** 2
    sig = r * r + a * a * np.cos(th) ** 2
    delta = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - a * a * delta * s2
    gtt = -(1.0 - 2.0 * r / sig)
    gtp = -2.0 * a * r * s2 / sig
    gpp = big_a * s2 / sig
    den = gpp + 2.0 * ell * gtp + ell * ell * gtt
    num = gtp * gtp - gtt * gpp
    with np.errstate(invalid="ignore", divide="ignore"):
        ut = -np.sqrt(num / den)
    return ut, (sig, delta, big_a)


def torus_fields(r, th, a=SPIN, r_in=R_IN, r_max=R_MAX, gam=4.0 / 3.0):
    """Noise-free torus (rho, p, u^t, u^phi, inside-mask) at BL (r, theta)."""
    ell = ell_kepler(r_max, a)
    ut_in, _ = _ut_bl(np.array(r_in), np.array(np.pi / 2), a, ell)
    ut, (sig, delta, big_a) = _ut_bl(r, th, a, ell)
    with np.errstate(invalid="ignore", divide="ignore"):
        h = ut_in / ut
    inside = np.isfinite(h) & (h > 1.0) & (r >= r_in)
    # maximum enthalpy sits at r_max on the equator
    ut_c, _ = _ut_bl(np.array(r_max), np.array(np.pi / 2), a, ell)
    h_max = ut_in / ut_c
    kpoly = (h_max - 1.0) * (gam - 1.0) / gam
    hh = np.where(inside, h, 1.0)
    rho = np.where(inside, ((hh - 1.0) / (h_max - 1.0)) ** (1.0 / (gam - 1.0)), 0.0)
    p = kpoly * rho ** gam
    s2 = np.sin(th) ** 2
    ssafe = np.where(s2 > 0, s2, 1.0)
    # contravariant u^t, u^phi from u_t and u_phi = -l u_t (BL inverse metric)
    u_t = np.where(inside, ut, -1.0)
    u_p = -ell * u_t
    gtt_u = -big_a / (sig * delta)
    gtp_u = -2.0 * a * r / (sig * delta)
    gpp_u = (delta - a * a * s2) / (sig * delta * ssafe)
    upt = gtt_u * u_t + gtp_u * u_p
    upp = gtp_u * u_t + gpp_u * u_p
    return rho, p, np.where(inside, upt, 0.0), np.where(inside, upp, 0.0), inside, ell


def torus(n1=256, n2=128, n3=128, seed=SEED, ng=5, a=SPIN, noise=NOISE,
          beta=BETA):
    """Torus initial data.  Returns (grid, data, tables): interior primitives
    rho, u1, u2, u3, p ([k][j][i]), ghosted x^3-edge potential A3 (A1 = A2 = 0),
    and the metric tables."""
    gam = 4.0 / 3.0
    grid = torus_grid(n1, n2, n3, ng=ng, rho_fl_a=RHO_FL[0], rho_fl_n=RHO_FL[1],
                      p_fl_a=P_FL[0], p_fl_n=P_FL[1], w_max=W_MAX)
    tab = kerr_schild_tables(grid, a=a)
    g = ng
    x1c = grid.x0[0] + (np.arange(n1) + 0.5) * grid.dx[0]
    x2c = grid.x0[1] + (np.arange(n2) + 0.5) * grid.dx[1]
    X1, TH = np.meshgrid(x1c, x2c)           # [j][i]
    r = np.exp(X1)
    rho, p, upt, upp, inside, ell = torus_fields(r, TH, a=a, gam=gam)
    sl = (slice(g, g + n2), slice(g, g + n1))
    alpha = tab[comp_index("C", "alpha")][sl]
    beta1 = tab[comp_index("C", "beta1")][sl]
    rho_fl = RHO_FL[0] * r ** RHO_FL[1]
    p_fl = P_FL[0] * r ** P_FL[1]
    w = np.where(inside, alpha * upt, 1.0)
    u1 = np.where(inside, upt * beta1, 0.0)
    u3 = np.where(inside, upp, 0.0)
    rho2 = np.where(inside, np.maximum(rho, rho_fl), rho_fl)
    p2 = np.where(inside, np.maximum(p, p_fl), p_fl)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(n3, n2, n1))
    rho3 = rho2[None] * np.where(inside[None], 1.0 + noise * xi, 1.0)
    data = {"rho": rho3, "u1": np.broadcast_to(u1, (n3, n2, n1)).copy(),
            "u2": np.zeros((n3, n2, n1)),
            "u3": np.broadcast_to(u3, (n3, n2, n1)).copy(),
            "p": np.broadcast_to(p2, (n3, n2, n1)).copy()}
    # vector potential on x^3 edges incl. ghosts (mirrored angles)
    i_e = np.arange(-g, n1 + g)
    j_e = np.arange(-g, n2 + g)
    x1e = grid.x0[0] + (i_e + 1.0) * grid.dx[0]
    x2e = grid.x0[1] + (j_e + 1.0) * grid.dx[1]
    X1e, THe = np.meshgrid(x1e, x2e)
    THe = np.where(THe < 0, -THe, THe)
    THe = np.where(THe > np.pi, 2 * np.pi - THe, THe)
    rho_e, _, _, _, _, _ = torus_fields(np.exp(X1e), THe, a=a, gam=gam)
    aphi = np.maximum(rho_e - 0.2, 0.0)
    scale = _beta_scale(grid, tab, aphi, p2, w, u1, u3, beta)
    a3 = scale * aphi
    data["A1"] = np.zeros(grid.shape)
    data["A2"] = np.zeros(grid.shape)
    data["A3"] = np.broadcast_to(a3[None], grid.shape).copy()
    meta = {"ell": float(ell), "spin": a, "r_in": R_IN, "r_max": R_MAX,
            "A_scale": float(scale), "inside_zones_2d": int(inside.sum())}
    grid.meta.update(meta)
    return grid, data, tab


def _beta_scale(grid, tab, aphi, p, w, u1, u3, beta):
    """Scale for A_phi so that max p / max(b^2/2) = beta, with B from centred
    second-order differences of the unscaled A_phi (edges (i+1/2, j+1/2))."""
    g = grid.ng
    n1, n2 = grid.n[0], grid.n[1]
    # A at the four corners of each cell: a[j][i] is edge (i+1/2, j+1/2)
    A = aphi
    jj = slice(g, g + n2)
    ii = slice(g, g + n1)
    jm = slice(g - 1, g - 1 + n2)
    im = slice(g - 1, g - 1 + n1)
    # B^1 ~ d_theta A, B^2 ~ -d_x1 A, averaged over the cell's corners
    dA2 = 0.5 * ((A[jj, ii] - A[jm, ii]) + (A[jj, im] - A[jm, im])) / grid.dx[1]
    dA1 = 0.5 * ((A[jj, ii] - A[jj, im]) + (A[jm, ii] - A[jm, im])) / grid.dx[0]
    sg = tab[comp_index("C", "sqrtg")][jj, ii]
    b1 = dA2 / sg
    b2 = -dA1 / sg
    g11 = tab[comp_index("C", "g11")][jj, ii]
    g22 = tab[comp_index("C", "g22")][jj, ii]
    g13 = tab[comp_index("C", "g13")][jj, ii]
    g33 = tab[comp_index("C", "g33")][jj, ii]
    bsq = g11 * b1 * b1 + g22 * b2 * b2
    # v_i B^i with v^i = u^i / W
    v1 = u1 / w
    v3 = u3 / w
    vb = (g11 * v1 + g13 * v3) * b1
    bb = bsq / (w * w) + vb * vb
    return np.sqrt(p.max() / (beta * 0.5 * bb.max()))
