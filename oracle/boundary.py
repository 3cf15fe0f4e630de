"""Ghost-zone fill (oracle, FP64).

Paper, Introduction: the code decomposes the domain into blocks with ghost
zones; on a single block the ghosts are set from the boundary conditions.
Applied one direction after the other (x^1, then x^2, then x^3), each over
the full extent of the other two directions, so edges and corners are filled.

  periodic : ghost index i <- i mod n (cells and faces alike; owned faces are
             the stored indices 0..n-1)
  outflow  : cells copy the nearest interior cell; at the upper x^1 boundary
             u^1 <- max(u^1, 0) (no inflow)
  axis     : polar axis in x^2 = theta (only with periodic x^3 = phi):
             ghost cell row -1-m <- row m, ghost row n+m <- row n-1-m, taken at
             the x^3 index shifted by n3/2; the components u^2, u^3, B^2, B^3
             and the face fields of x^2 and x^3 change sign.
  Faces normal to an outflow or axis boundary: the ghost faces that the
  staggered derivative of an interior cell reads, stored -flo .. -1 and
  n .. n + flo - 2 (flo = 3 for the sixth order, 2 for the fourth), are not
  filled: the scheme evolves them with the induction equation like the owned
  faces (so the discrete div B of every interior cell keeps its value), and
  the axis faces (stored -1 and n-1) with them.  Beyond those: outflow copies
  the outermost evolved face; axis sets ghost face -2-m <- face m and
  n+m <- n-2-m (half a turn away, sign changed).
"""
import numpy as np

PERIODIC, OUTFLOW, AXIS = 0, 1, 2
AX = (2, 1, 0)
FLIP_AXIS = {"u2", "u3", "B2", "B3", "Bf2", "Bf3"}


def _sl(axis, s):
    out = [slice(None)] * 3
    out[axis] = s
    return tuple(out)


def _fill_dir(q, name, grid, d, normal, flo=3):
    """Fill ghosts of array q along direction d.  normal: True if q is a face
    field whose faces are normal to d; flo: evolved ghost face layers below
    the interior (flo - 1 above) of a non-periodic direction."""
    g = grid.ng
    n = grid.n[d]
    ax = AX[d]
    lo_bc, hi_bc = grid.bc[2 * d], grid.bc[2 * d + 1]
    # index helper: stored interior-relative index m -> array index m + g
    def setv(m, val):
        q[_sl(ax, m + g)] = val

    def getv(m):
        return q[_sl(ax, m + g)].copy()

    if lo_bc == PERIODIC:
        assert hi_bc == PERIODIC
        for m in list(range(-g, 0)) + list(range(n, n + g)):
            setv(m, getv(m % n))
        return
    if lo_bc == AXIS:
        assert hi_bc == AXIS and d == 1 and n >= g
        n3 = grid.n[2]
        sign = -1.0 if name in FLIP_AXIS else 1.0

        def shifted(m):
            v = getv(m)                    # shape (N3, N1) after removing axis 1
            inner = v[g:g + n3]
            rolled = np.roll(inner, -(n3 // 2), axis=0)   # rolled[k] = inner[(k + n3/2) % n3]
            out = v.copy()
            out[g:g + n3] = rolled
            return sign * out
        if normal:
            for m in range(flo - 1, g - 1):
                setv(-2 - m, shifted(m))
            for m in range(flo - 1, g):
                setv(n + m, shifted(n - 2 - m))
        else:
            for m in range(0, g):
                setv(-1 - m, shifted(m))
                setv(n + m, shifted(n - 1 - m))
        return
    # outflow (each side may be outflow independently of the other)
    if lo_bc == OUTFLOW:
        first = -flo if normal else 0
        src = getv(first)
        for m in range(-g, min(first, 0)):
            setv(m, src)
    if hi_bc == OUTFLOW:
        last = n + flo - 2 if normal else n - 1
        src = getv(last)
        if d == 0 and name == "u1":
            src = np.maximum(src, 0.0)
        for m in range(last + 1, n + g):
            setv(m, src)


def fill_centred(P, grid, names=None):
    names = names or list(P.keys())
    for name in names:
        for d in range(3):
            _fill_dir(P[name], name, grid, d, normal=False)


def fill_faces(U, grid, flo=3):
    for nd in range(3):
        name = "Bf%d" % (nd + 1)
        for d in range(3):
            _fill_dir(U[name], name, grid, d, normal=(d == nd), flo=flo)
