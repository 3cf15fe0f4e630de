"""HLL Riemann flux (oracle, FP64).

Paper, Introduction (the scheme family's approximate Riemann solver); the
two-wave HLL flux of Harten, Lax & van Leer (1983):
  a+ = max(0, lambda+_L, lambda+_R), a- = max(0, -lambda-_L, -lambda-_R)
  F = [a+ F_L + a- F_R - a+ a- (U_R - U_L)] / (a+ + a-)
with face-densitised U.  If a+ + a- < 1e-300 the flux is the mean
(F_L + F_R)/2.
"""
import numpy as np


def hll_speeds(lp_l, lm_l, lp_r, lm_r):
    ap = np.maximum(0.0, np.maximum(lp_l, lp_r))
    am = np.maximum(0.0, np.maximum(-lm_l, -lm_r))
    return ap, am


def hll_flux(fl, fr, ul, ur, ap, am):
    s = ap + am
    tiny = s < 1e-300
    with np.errstate(divide="ignore", invalid="ignore"):
        out = (ap * fl + am * fr - ap * am * (ur - ul)) / s
    return np.where(tiny, 0.5 * (fl + fr), out)
