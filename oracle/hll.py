"""HLL Riemann flux (oracle, FP64).

Paper, Introduction (the scheme family's approximate Riemann solver); the
two-wave HLL flux of Harten, Lax & van Leer (1983):
  a+ = max(0, lambda+_L, lambda+_R), a- = max(0, -lambda-_L, -lambda-_R)
  F = [a+ F_L + a- F_R - a+ a- (U_R - U_L)] / (a+ + a-)
with face-densitised U.  If a+ + a- < 1e-300 (1e-37 in float32) the flux
is the mean (F_L + F_R)/2.
"""
import numpy as np


def hll_speeds(lp_l, lm_l, lp_r, lm_r):
    z = np.zeros((), dtype=np.result_type(lp_l, lp_r))
    ap = np.maximum(z, np.maximum(lp_l, lp_r))
    am = np.maximum(z, np.maximum(-lm_l, -lm_r))
    return ap, am


def hll_flux(fl, fr, ul, ur, ap, am):
    s = ap + am
    tiny = s < (1e-300 if s.dtype == np.float64 else 1e-37)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = (ap * fl + am * fr - ap * am * (ur - ul)) / s
    return np.where(tiny, s.dtype.type(0.5) * (fl + fr), out)
