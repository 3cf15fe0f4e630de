"""Conservative-to-primitive inversion (oracle, FP64).

Paper, Introduction (the scheme evolves conserved variables; the primitive
variables needed for reconstruction are recovered in every zone).  Reading
taken here: a one-dimensional Newton iteration in y = rho h W^2 with the
magnetic field known (ECHO-style inversion).

Inputs (undensitised with the centre sqrt(gamma)): D, S_i, tau, B^i;
U = tau + D, S^2 = gamma^ij S_i S_j, B^2 = B_i B^i, SB = S_i B^i.
  v^2(y) = [S^2 + SB^2 (2y + B^2)/y^2] / (y + B^2)^2
  p(y)   = (Gamma-1)/Gamma [y (1 - v^2) - D sqrt(1 - v^2)]
  f(y)   = y - p + B^2 (1 + v^2)/2 - SB^2/(2 y^2) - U
  dv2/dy = -2 SB^2 (y + B^2)/(y^3 (y + B^2)^2) - 2 [S^2 + SB^2 (2y + B^2)/y^2]/(y + B^2)^3
  dp/dy  = (Gamma-1)/Gamma [(1 - v^2) - y dv2/dy + D dv2/dy / (2 sqrt(1 - v^2))]
  f'(y)  = 1 - dp/dy + B^2 dv2/dy / 2 + SB^2 / y^3
Safeguarded Newton on the bracket (a, b) = (0, Gamma U): f(b) >= 0 for a
physical state.  Each iterate y in (a, b):
  * if v^2(y) >= 1, y lies below the root: a = y, next y = (a + b)/2;
  * else f(y) < 0 sets a = y, f(y) >= 0 sets b = y; the Newton step
    y - f/f' is taken if it stays inside [a, b], else (a + b)/2.
Stop when |f(y)| is below the round-off bound of its own evaluation,
4 eps (y + |p| + B^2 (1 + v^2)/2 + SB^2/(2 y^2) + U) (then y is the root),
or when the step |dy| <= tol y (tol = 1e-14); at most maxit (50) steps.
Outputs: W = (1 - v^2)^(-1/2), rho = D/W, p = p(y),
v_i = (S_i + (SB/y) B_i)/(y + B^2), u^i = W gamma^ij v_j.
Failure (flagged): D <= 0, U <= 0, non-finite input, no convergence,
v^2 >= 1 or non-finite output.  Without floors the zone keeps its previous
primitives; with floors (accretion-torus runs) it is reset to atmosphere
(floor density and pressure, at rest) and its conserved variables are
recomputed.
Guess: warm y0 = rho h W^2 of the previous primitives (cold: Gamma U);
a guess outside (a, b) is replaced by (a + b)/2.
"""
import numpy as np

EPS4 = 4.0 * 2.0 ** -52


def _v2(y, s2, sb2, b2):
    return (s2 + sb2 * (2.0 * y + b2) / (y * y)) / ((y + b2) * (y + b2))


def newton(dd, s, tau, b, m, gam, y0, tol=1e-14, maxit=50):
    """Vectorised per-zone Newton.  Returns dict with rho, u (3), p, W, y,
    iters, ok (bool) for every zone (values undefined where not ok)."""
    from .physics import lower, raise_
    utot = tau + dd
    su = raise_(m, s)
    s2 = s[0] * su[0] + s[1] * su[1] + s[2] * su[2]
    bl = lower(m, b)
    b2 = bl[0] * b[0] + bl[1] * b[1] + bl[2] * b[2]
    sb = s[0] * b[0] + s[1] * b[1] + s[2] * b[2]
    sb2 = sb * sb
    gf = (gam - 1.0) / gam
    shape = np.broadcast(dd, utot, y0).shape
    a = np.zeros(shape)
    bb = np.broadcast_to(gam * utot, shape).copy()
    finite = np.isfinite(dd) & np.isfinite(utot) & np.isfinite(s2) & np.isfinite(b2) & np.isfinite(sb)
    valid = finite & (dd > 0.0) & (utot > 0.0)
    y = np.broadcast_to(y0, shape).copy()
    outside = ~((y > a) & (y < bb))
    y = np.where(outside, 0.5 * (a + bb), y)
    active = valid.copy()
    conv = np.zeros(shape, dtype=bool)
    iters = np.zeros(shape, dtype=np.int64)
    with np.errstate(all="ignore"):
        for _ in range(maxit):
            if not active.any():
                break
            iters += active
            v2 = _v2(y, s2, sb2, b2)
            bad = v2 >= 1.0
            sq = np.sqrt(1.0 - v2)
            p = gf * (y * (1.0 - v2) - dd * sq)
            f = y - p + 0.5 * b2 * (1.0 + v2) - 0.5 * sb2 / (y * y) - utot
            yb = y + b2
            dv2 = (-2.0 * sb2 * yb / (y ** 3) / (yb * yb)
                   - 2.0 * (s2 + sb2 * (2.0 * y + b2) / (y * y)) / (yb * yb * yb))
            dp = gf * ((1.0 - v2) - y * dv2 + dd * dv2 / (2.0 * sq))
            fp = 1.0 - dp + 0.5 * b2 * dv2 + sb2 / (y ** 3)
            # residual at the round-off level of its own evaluation
            fabs = y + np.abs(p) + 0.5 * b2 * (1.0 + v2) + 0.5 * sb2 / (y * y) + utot
            zero = ~bad & (np.abs(f) <= EPS4 * fabs)
            hit = active & zero
            conv |= hit
            active &= ~zero
            below = bad | (f < 0.0)
            a_new = np.where(active & below, y, a)
            b_new = np.where(active & ~below, y, bb)
            yn = y - f / fp
            use_bis = bad | ~((yn >= a_new) & (yn <= b_new))
            yn = np.where(use_bis, 0.5 * (a_new + b_new), yn)
            dy = yn - y
            a, bb = a_new, b_new
            y = np.where(active, yn, y)
            done = active & (np.abs(dy) <= tol * y)
            conv |= done
            active &= ~done
        v2 = _v2(y, s2, sb2, b2)
        w = 1.0 / np.sqrt(1.0 - v2)
        p = gf * (y * (1.0 - v2) - dd * np.sqrt(1.0 - v2))
        rho = dd / w
        vl = tuple((s[i] + (sb / y) * bl[i]) / (y + b2) for i in range(3))
        vu = raise_(m, vl)
        u = tuple(w * vu[i] for i in range(3))
    ok = conv & valid & (v2 < 1.0) & np.isfinite(rho) & np.isfinite(p)
    for c in u:
        ok &= np.isfinite(c)
    return {"rho": rho, "u": u, "p": p, "W": w, "y": y, "iters": iters, "ok": ok}


def warm_guess(rho, u, p, m, gam):
    from .physics import lower
    ul = lower(m, u)
    uu = ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2]
    h = 1.0 + gam / (gam - 1.0) * p / rho
    return rho * h * (1.0 + uu)
