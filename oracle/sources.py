"""Metric source terms of the stationary 3+1 GRMHD equations (oracle, FP64).

Paper, Introduction (MHD in general relativity).  For a stationary metric
(Cowling approximation, d_t gamma_ij = 0) the densitised sources are
  s[D]     = 0
  s[S_i]   = sqrt(gamma) (1/2 alpha W^jk d_i gamma_jk + S_j d_i beta^j - U d_i alpha)
  s[tau]   = sqrt(gamma) (1/2 W^jk beta^l d_l gamma_jk + W^j_k d_j beta^k - S^j d_j alpha)
with W^jk = y v^j v^k - E^j E^k - B^j B^k + [p + (E^2 + B^2)/2] gamma^jk,
W^j_k its mixed form, U = tau + D.  The tables are axisymmetric, so only
d_1 and d_2 are non-zero (s[S_3] = 0).
"""
import numpy as np

from .physics import state, electric, gu

GN = {(1, 1): "g11", (1, 2): "g12", (1, 3): "g13", (2, 2): "g22", (2, 3): "g23",
      (3, 3): "g33"}


def sources(P, m, der, gam):
    """Sources at the points of P (interior cells) with centre metric m and
    derivative tables der ({'d1_alpha': ..., ...})."""
    st = state(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"],
               (P["B1"], P["B2"], P["B3"]), m, gam)
    el, eu = electric(st, m)
    v, vl, b, bl = st["v"], st["vl"], st["B"], st["Bl"]
    ptot = st["p"] + 0.5 * (st["E2"] + st["B2"])
    y = st["y"]

    def wup(j, k):
        return (y * v[j - 1] * v[k - 1] - eu[j - 1] * eu[k - 1] - b[j - 1] * b[k - 1]
                + ptot * gu(m, j, k))

    def wmix(j, k):
        out = y * v[j - 1] * vl[k - 1] - eu[j - 1] * el[k - 1] - b[j - 1] * bl[k - 1]
        if j == k:
            out = out + ptot
        return out

    def dg(i, j, k):
        return der["d%d_%s" % (i, GN[(min(j, k), max(j, k))])]

    sg, al = m["sqrtg"], m["alpha"]
    beta = (m["beta1"], m["beta2"], m["beta3"])
    utot = st["Utot"]
    out = {"D": 0.0 * sg}
    for i in (1, 2, 3):
        if i == 3:
            out["S3"] = 0.0 * sg
            continue
        t = 0.0
        for j in (1, 2, 3):
            for k in (1, 2, 3):
                t = t + 0.5 * al * wup(j, k) * dg(i, j, k)
        for j in (1, 2, 3):
            t = t + st["S"][j - 1] * der["d%d_beta%d" % (i, j)]
        t = t - utot * der["d%d_alpha" % i]
        out["S%d" % i] = sg * t
    t = 0.0
    for l in (1, 2):
        for j in (1, 2, 3):
            for k in (1, 2, 3):
                t = t + 0.5 * wup(j, k) * beta[l - 1] * dg(l, j, k)
    for j in (1, 2):
        for k in (1, 2, 3):
            t = t + wmix(j, k) * der["d%d_beta%d" % (j, k)]
    for j in (1, 2):
        t = t - st["Su"][j - 1] * der["d%d_alpha" % j]
    out["tau"] = sg * t
    return out
