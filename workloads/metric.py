"""Tables of the stationary background metric (3+1 split), shared as data.

Table layout (a float64 array of shape (NCOMP, n2 + 2 ng, n1 + 2 ng), indexed
[comp][j][i], axisymmetric: the same for every x^3 index):
  four location families, in this order, 17 components each
      C  : cell centres          (i,       j      )
      F1 : x^1 faces  i + 1/2    (i + 1/2, j      )
      F2 : x^2 faces  j + 1/2    (i,       j + 1/2)
      E3 : x^3 edges             (i + 1/2, j + 1/2)
    components: alpha, beta^1..3, gamma_11, _12, _13, _22, _23, _33,
                gamma^11, ^12, ^13, ^22, ^23, ^33, sqrt(gamma)
  then 20 centre derivatives:
      d1 alpha, d2 alpha, d1 beta^1..3, d2 beta^1..3,
      d1 gamma_11.._33 (6), d2 gamma_11.._33 (6)
Because the tables do not depend on x^3, x^3 faces use the centre entries,
x^1 edges (i, j+1/2, k+1/2) use F2 and x^2 edges (i+1/2, j, k+1/2) use F1.

Kerr-Schild (spin a, mass m) in code coordinates (x^1 = ln r, theta, phi),
standard KS line element with dr = r dx^1:
  Sigma = r^2 + a^2 cos^2 th, z = 2 m r / Sigma, s = sin th
  alpha = (1+z)^(-1/2), beta^1 = z / (r (1+z)), beta^2 = beta^3 = 0
  gamma_11 = r^2 (1+z), gamma_13 = -a r (1+z) s^2, gamma_22 = Sigma,
  gamma_33 = s^2 (Sigma + a^2 (1+z) s^2), gamma_12 = gamma_23 = 0
  inverse (closed form): gamma^11 = (Sigma + a^2 (1+z) s^2) / (r^2 (1+z) Sigma),
  gamma^13 = a / (r Sigma), gamma^22 = 1/Sigma, gamma^33 = 1/(s^2 Sigma)
  sqrt(gamma) = r Sigma s (1+z)^(1/2)
Derivatives use complex-step differentiation of these closed forms (exact to
round-off).  Ghost rows beyond the polar axis use the mirrored angle, so the
tables there equal those of the mirrored interior row (|sin theta|).  On the
axis itself sin theta is set to exactly 0; gamma^33 is infinite there and is
stored as 0 (the scheme never reads it at axis locations).
"""
import numpy as np

LOCS = ("C", "F1", "F2", "E3")
GEOM = ("alpha", "beta1", "beta2", "beta3", "g11", "g12", "g13", "g22", "g23", "g33",
        "gu11", "gu12", "gu13", "gu22", "gu23", "gu33", "sqrtg")
DERIV = (["d1_alpha", "d2_alpha"] + [f"d1_beta{i}" for i in (1, 2, 3)]
         + [f"d2_beta{i}" for i in (1, 2, 3)]
         + [f"d1_{c}" for c in ("g11", "g12", "g13", "g22", "g23", "g33")]
         + [f"d2_{c}" for c in ("g11", "g12", "g13", "g22", "g23", "g33")])
NGEOM = len(GEOM)
NCOMP = 4 * NGEOM + len(DERIV)   # 88


def comp_index(loc, name):
    if name in GEOM:
        return LOCS.index(loc) * NGEOM + GEOM.index(name)
    assert loc == "C"
    return 4 * NGEOM + DERIV.index(name)


def _ks_fields(x1, th, a, m, s_override=None):
    """Closed-form KS quantities at (x1 = ln r, theta); works on complex input."""
    r = np.exp(x1)
    s = np.sin(th) if s_override is None else s_override
    c = np.cos(th)
    sig = r * r + a * a * c * c
    z = 2.0 * m * r / sig
    f = {}
    f["alpha"] = 1.0 / np.sqrt(1.0 + z)
    f["beta1"] = z / (r * (1.0 + z))
    f["beta2"] = 0.0 * r
    f["beta3"] = 0.0 * r
    f["g11"] = r * r * (1.0 + z)
    f["g12"] = 0.0 * r
    f["g13"] = -a * r * (1.0 + z) * s * s
    f["g22"] = sig
    f["g23"] = 0.0 * r
    f["g33"] = s * s * (sig + a * a * (1.0 + z) * s * s)
    f["gu11"] = (sig + a * a * (1.0 + z) * s * s) / (r * r * (1.0 + z) * sig)
    f["gu12"] = 0.0 * r
    f["gu13"] = a / (r * sig)
    f["gu22"] = 1.0 / sig
    f["gu23"] = 0.0 * r
    with np.errstate(divide="ignore", invalid="ignore"):
        gu33 = 1.0 / (s * s * sig)
    f["gu33"] = gu33
    f["sqrtg"] = r * sig * s * np.sqrt(1.0 + z)
    return f


def _mirror_theta(th):
    """Map ghost angles beyond the poles back into [0, pi]."""
    th = np.where(th < 0.0, -th, th)
    th = np.where(th > np.pi, 2.0 * np.pi - th, th)
    return th


def kerr_schild_tables(grid, a=0.9, m=1.0, h=1e-30):
    """Metric tables on a log-spherical grid (see module docstring)."""
    g = grid.ng
    n1, n2 = grid.n[0], grid.n[1]
    i = np.arange(-g, n1 + g, dtype=np.float64)
    j = np.arange(-g, n2 + g, dtype=np.float64)
    x1c = grid.x0[0] + (i + 0.5) * grid.dx[0]
    x1f = grid.x0[0] + (i + 1.0) * grid.dx[0]
    x2c = grid.x0[1] + (j + 0.5) * grid.dx[1]
    x2f = grid.x0[1] + (j + 1.0) * grid.dx[1]
    pos = {"C": (x1c, x2c), "F1": (x1f, x2c), "F2": (x1c, x2f), "E3": (x1f, x2f)}
    tab = np.zeros((NCOMP, n2 + 2 * g, n1 + 2 * g))
    for loc in LOCS:
        X1, TH = np.meshgrid(pos[loc][0], pos[loc][1])
        THm = _mirror_theta(TH)
        s = np.sin(THm)
        on_axis = np.abs(s) < 1e-12
        s = np.where(on_axis, 0.0, s)
        f = _ks_fields(X1, THm, a, m, s_override=s)
        for name in GEOM:
            v = np.asarray(f[name], dtype=np.float64) * np.ones_like(X1)
            if name == "gu33":
                v = np.where(on_axis, 0.0, v)
            tab[comp_index(loc, name)] = v
    # centre derivatives by complex step
    X1, TH = np.meshgrid(x1c, x2c)
    THm = _mirror_theta(TH)
    fd1 = _ks_fields(X1 + 1j * h, THm, a, m)
    fd2 = _ks_fields(X1 + 0j, THm + 1j * h, a, m)
    for nm in ("alpha", "beta1", "beta2", "beta3", "g11", "g12", "g13", "g22", "g23", "g33"):
        tab[comp_index("C", "d1_" + nm)] = np.imag(fd1[nm] * np.ones_like(X1)) / h
        tab[comp_index("C", "d2_" + nm)] = np.imag(fd2[nm] * np.ones_like(X1)) / h
    return tab


def minkowski_tables(grid):
    """Flat Cartesian metric written out as tables (alpha = 1, beta = 0,
    gamma = identity); used to run the table-driven path in flat space."""
    g = grid.ng
    tab = np.zeros((NCOMP, grid.n[1] + 2 * g, grid.n[0] + 2 * g))
    for loc in LOCS:
        for name in ("alpha", "g11", "g22", "g33", "gu11", "gu22", "gu33", "sqrtg"):
            tab[comp_index(loc, name)] = 1.0
    return tab


def unpack(tab):
    """Split a table array into {loc: {name: 2-D array}} and {deriv: array}."""
    out = {loc: {nm: tab[comp_index(loc, nm)] for nm in GEOM} for loc in LOCS}
    der = {nm: tab[4 * NGEOM + q] for q, nm in enumerate(DERIV)}
    return out, der
