"""Pointwise 3+1 GRMHD algebra (oracle, FP64).

Paper, Introduction: the code solves the equations of MHD in general
relativity, based on ECHO.  The conservative 3+1 (Valencia / ECHO) form is
used, in units G = c = M = 1 with Heaviside-Lorentz fields (magnetic pressure
B^2/2), ideal gas of index Gamma.

Primitives: rho, u^i = W v^i (contravariant), p, B^i (undensitised).
  u_i = gamma_ij u^j, W = (1 + u_i u^i)^(1/2), v^i = u^i / W,
  v^2 = u_i u^i / (1 + u_i u^i)
  B_i = gamma_ij B^j, B^2 = B_i B^i, (vB) = v_i B^i
  E_i = -sqrt(gamma) [ijk] v^j B^k, E^i = -[ijk] v_j B_k / sqrt(gamma),
  E^2 = B^2 v^2 - (vB)^2
  h = 1 + Gamma/(Gamma-1) p/rho, y = rho h W^2
Conserved: D = rho W, S_i = (y + B^2) v_i - (vB) B_i,
  U = y - p + (B^2 + E^2)/2, tau = U - D;
  evolved densitised: sqrt(gamma) (D, S_i, tau).
Stress (mixed): W^d_i = y v^d v_i - E^d E_i - B^d B_i + [p + (E^2 + B^2)/2] delta^d_i
Fluxes in direction d (densitised):
  F[D] = sqrt(gamma) (alpha v^d - beta^d) D
  F[S_i] = sqrt(gamma) (alpha W^d_i - beta^d S_i)
  F[tau] = sqrt(gamma) (alpha (S^d - v^d D) - beta^d tau),
  S^d = (y + B^2) v^d - (vB) B^d
Fast speeds (Gammie, McKinney & Toth 2003 estimate):
  cs^2 = Gamma p / (rho h), b^2 = B^2/W^2 + (vB)^2, vA^2 = b^2/(rho h + b^2),
  a^2 = cs^2 + vA^2 - cs^2 vA^2,
  lambda^pm_d = alpha/(1 - v^2 a^2) [v^d (1 - a^2) pm sqrt(a^2 (1 - v^2)
                (gamma^dd (1 - v^2 a^2) - (v^d)^2 (1 - a^2)))] - beta^d
  (radicand clamped at 0).
"""
import numpy as np

LOWER = {(1, 1): "g11", (1, 2): "g12", (1, 3): "g13", (2, 2): "g22",
         (2, 3): "g23", (3, 3): "g33"}
UPPER = {(1, 1): "gu11", (1, 2): "gu12", (1, 3): "gu13", (2, 2): "gu22",
         (2, 3): "gu23", (3, 3): "gu33"}


def gl(m, i, j):
    return m[LOWER[(min(i, j), max(i, j))]]


def gu(m, i, j):
    return m[UPPER[(min(i, j), max(i, j))]]


def lower(m, a):
    """gamma_ij a^j for a = (a1, a2, a3)."""
    return tuple(sum(gl(m, i, j) * a[j - 1] for j in (1, 2, 3)) for i in (1, 2, 3))


def raise_(m, a):
    return tuple(sum(gu(m, i, j) * a[j - 1] for j in (1, 2, 3)) for i in (1, 2, 3))


def state(rho, u, p, b, m, gam):
    """All derived pointwise quantities of a primitive state at a location
    with metric m.  u, b: 3-tuples of contravariant components."""
    st = {"rho": rho, "p": p, "u": u, "B": b}
    ul = lower(m, u)
    uu = ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2]
    w = np.sqrt(1.0 + uu)
    v = tuple(x / w for x in u)
    vl = tuple(x / w for x in ul)
    v2 = uu / (1.0 + uu)
    bl = lower(m, b)
    b2 = bl[0] * b[0] + bl[1] * b[1] + bl[2] * b[2]
    vb = vl[0] * b[0] + vl[1] * b[1] + vl[2] * b[2]
    e2 = b2 * v2 - vb * vb
    h = 1.0 + gam / (gam - 1.0) * p / rho
    y = rho * h * w * w
    dd = rho * w
    s = tuple((y + b2) * vl[i] - vb * bl[i] for i in range(3))
    su = tuple((y + b2) * v[i] - vb * b[i] for i in range(3))
    utot = y - p + 0.5 * (b2 + e2)
    st.update(W=w, v=v, vl=vl, v2=v2, Bl=bl, B2=b2, vB=vb, E2=e2, h=h, y=y,
              D=dd, S=s, Su=su, Utot=utot, tau=utot - dd)
    return st


def electric(st, m):
    """Covariant and contravariant electric field (E_i, E^i)."""
    v, vl, b, bl = st["v"], st["vl"], st["B"], st["Bl"]
    sg = m["sqrtg"]
    el = (-sg * (v[1] * b[2] - v[2] * b[1]),
          -sg * (v[2] * b[0] - v[0] * b[2]),
          -sg * (v[0] * b[1] - v[1] * b[0]))
    with np.errstate(divide="ignore", invalid="ignore"):
        eu = (-(vl[1] * bl[2] - vl[2] * bl[1]) / sg,
              -(vl[2] * bl[0] - vl[0] * bl[2]) / sg,
              -(vl[0] * bl[1] - vl[1] * bl[0]) / sg)
    return el, eu


def cons(st, m):
    """Densitised conserved hydro variables (D, S_1, S_2, S_3, tau)."""
    sg = m["sqrtg"]
    return (sg * st["D"], sg * st["S"][0], sg * st["S"][1], sg * st["S"][2],
            sg * st["tau"])


def flux(st, m, d):
    """Densitised fluxes of (D, S_1, S_2, S_3, tau) in direction d (0-based)."""
    sg, al = m["sqrtg"], m["alpha"]
    bd = m["beta%d" % (d + 1)]
    v, vl, b, bl = st["v"], st["vl"], st["B"], st["Bl"]
    el, eu = electric(st, m)
    ptot = st["p"] + 0.5 * (st["E2"] + st["B2"])
    out = [sg * (al * v[d] - bd) * st["D"]]
    for i in range(3):
        wdi = st["y"] * v[d] * vl[i] - eu[d] * el[i] - b[d] * bl[i]
        if i == d:
            wdi = wdi + ptot
        out.append(sg * (al * wdi - bd * st["S"][i]))
    out.append(sg * (al * (st["Su"][d] - v[d] * st["D"]) - bd * st["tau"]))
    return tuple(out)


def speeds(st, m, d, gam):
    """(lambda^+, lambda^-) in direction d."""
    al = m["alpha"]
    bd = m["beta%d" % (d + 1)]
    gdd = gu(m, d + 1, d + 1)
    rhoh = st["rho"] * st["h"]
    cs2 = gam * st["p"] / rhoh
    bb = st["B2"] / (st["W"] * st["W"]) + st["vB"] * st["vB"]
    va2 = bb / (rhoh + bb)
    a2 = cs2 + va2 - cs2 * va2
    v2 = st["v2"]
    vd = st["v"][d]
    den = 1.0 - v2 * a2
    rad = a2 * (1.0 - v2) * (gdd * den - vd * vd * (1.0 - a2))
    rad = np.sqrt(np.maximum(rad, 0.0))
    lp = al / den * (vd * (1.0 - a2) + rad) - bd
    lm = al / den * (vd * (1.0 - a2) - rad) - bd
    return lp, lm


def prim2cons(rho, u, p, b, m, gam):
    return cons(state(rho, u, p, b, m, gam), m)
