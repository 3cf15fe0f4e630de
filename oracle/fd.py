"""Finite-difference operators on a staggered grid (oracle, FP64).

Paper, Introduction: the equations are discretised with finite differences
in three dimensions.  The ECHO family writes the flux derivative as a plain difference of
high-order corrected face fluxes, f_hat = f - Delta^2 f / 24 + 3 Delta^4 f / 640;
expanded, that is the sixth-order staggered derivative below.  Its companion
I_d interpolates face values to the cell centre to sixth order.

  (D f)_m = [75/64 (f_{m+1/2} - f_{m-1/2}) - 25/384 (f_{m+3/2} - f_{m-3/2})
             + 3/640 (f_{m+5/2} - f_{m-5/2})] / Delta
  (I f)_m = [150 (f_{m+1/2} + f_{m-1/2}) - 25 (f_{m+3/2} + f_{m-3/2})
             + 3 (f_{m+5/2} + f_{m-5/2})] / 256

With the face m+1/2 stored at index m, the stencil of cell m reads stored
indices m-3 .. m+2.

A fourth-order member of the same family (order=4) keeps only the first
correction, f_hat = f - Delta^2 f / 24:

  (D4 f)_m = [27/24 (f_{m+1/2} - f_{m-1/2}) - 1/24 (f_{m+3/2} - f_{m-3/2})] / Delta
  (I4 f)_m = [9 (f_{m+1/2} + f_{m-1/2}) - (f_{m+3/2} + f_{m-3/2})] / 16

(stored indices m-2 .. m+1).
"""
import numpy as np

# direction d (0 = x^1) -> numpy axis of a [k][j][i] array
AXIS = (2, 1, 0)


def take(a, d, lo, hi, g):
    """View of `a` with stored interior-relative indices [lo, hi) along
    direction d and everything along the other directions."""
    sl = [slice(None)] * 3
    sl[AXIS[d]] = slice(lo + g, hi + g)
    return a[tuple(sl)]


def deriv(f, d, lo, hi, dx, g, order=6):
    """D_d f at positions m in [lo, hi) (cells, or edges/faces offset in d)."""
    t = lambda s: take(f, d, lo + s, hi + s, g)
    if order == 4:
        return (27.0 / 24.0 * (t(0) - t(-1)) - 1.0 / 24.0 * (t(1) - t(-2))) / dx
    assert order == 6
    return (75.0 / 64.0 * (t(0) - t(-1)) - 25.0 / 384.0 * (t(1) - t(-2))
            + 3.0 / 640.0 * (t(2) - t(-3))) / dx


def interp(f, d, lo, hi, g, order=6):
    """I_d f at cell positions m in [lo, hi) from faces in direction d."""
    t = lambda s: take(f, d, lo + s, hi + s, g)
    if order == 4:
        return (9.0 * (t(0) + t(-1)) - (t(1) + t(-2))) / 16.0
    assert order == 6
    return (150.0 * (t(0) + t(-1)) - 25.0 * (t(1) + t(-2))
            + 3.0 * (t(2) + t(-3))) / 256.0


def interior(a, g):
    return a[g:-g, g:-g, g:-g] if g > 0 else a


def put(dst, d, lo, hi, g, val):
    sl = [slice(None)] * 3
    sl[AXIS[d]] = slice(lo + g, hi + g)
    dst[tuple(sl)] = val


def region(a, g, ranges):
    """a restricted to stored interior-relative ranges ((lo1,hi1),(lo2,hi2),(lo3,hi3))."""
    (l1, h1), (l2, h2), (l3, h3) = ranges
    return a[l3 + g:h3 + g, l2 + g:h2 + g, l1 + g:h1 + g]


__all__ = ["AXIS", "take", "deriv", "interp", "interior", "put", "region", "np"]
