"""MP5 reconstruction (oracle, FP64).

Paper, Introduction: the scheme reconstructs interface values to high
order.  The scheme family's fifth-order choice is the monotonicity-preserving MP5 limiter of
Suresh & Huynh (1997).  Two readings apply (both listed with the other
readings of the paper):
  * the unlimited value is the degree-4 Lagrange interpolant of the point
    values at the midpoint, (3, -20, 90, 60, -5)/128, because a
    finite-difference scheme reconstructs point values, not cell averages;
  * the limiter's tolerance is 0, so the map is continuous.

Left state at face j+1/2 from q_{j-2}, ..., q_{j+2} (arguments qm2..qp2):
  1. qL  = (3 q_{j-2} - 20 q_{j-1} + 90 q_j + 60 q_{j+1} - 5 q_{j+2}) / 128
  2. qMP = q_j + minmod(q_{j+1} - q_j, 4 (q_j - q_{j-1}))
  3. if (qL - q_j)(qL - qMP) <= 0: return qL
  4. d_m = q_{m-1} - 2 q_m + q_{m+1} for m = j-1, j, j+1
  5. dM4+ = minmod4(4 d_j - d_{j+1}, 4 d_{j+1} - d_j, d_j, d_{j+1})
     dM4- = minmod4(4 d_j - d_{j-1}, 4 d_{j-1} - d_j, d_j, d_{j-1})
  6. qUL = q_j + 4 (q_j - q_{j-1}); qMD = (q_j + q_{j+1})/2 - dM4+/2;
     qLC = q_j + (q_j - q_{j-1})/2 + 4/3 dM4-
  7. qmin = max(min(q_j, q_{j+1}, qMD), min(q_j, qUL, qLC))
     qmax = min(max(q_j, q_{j+1}, qMD), max(q_j, qUL, qLC))
  8. return median(qL, qmin, qmax) = qL + minmod(qmin - qL, qmax - qL)
The right state at j+1/2 is the same map applied to the reversed stencil
q_{j+3}, ..., q_{j-1}.
"""
import numpy as np


def minmod(a, b):
    return 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))


def minmod4(w, x, y, z):
    s = 0.125 * (np.sign(w) + np.sign(x)) * np.abs((np.sign(w) + np.sign(y))
                                                    * (np.sign(w) + np.sign(z)))
    return s * np.minimum(np.minimum(np.abs(w), np.abs(x)),
                          np.minimum(np.abs(y), np.abs(z)))


def unlimited(qm2, qm1, q0, qp1, qp2):
    return (3.0 * qm2 - 20.0 * qm1 + 90.0 * q0 + 60.0 * qp1 - 5.0 * qp2) / 128.0


def mp5(qm2, qm1, q0, qp1, qp2):
    """Limited left state at the face between q0 and qp1."""
    return mp_limit(unlimited(qm2, qm1, q0, qp1, qp2), qm2, qm1, q0, qp1, qp2)


def mp_limit(ql, qm2, qm1, q0, qp1, qp2):
    """Steps 2-8 above: the monotonicity-preserving limit of an unlimited
    face value ql from q_{j-2..j+2} (the same limiter serves every order of
    the unlimited value)."""
    qmp = q0 + minmod(qp1 - q0, 4.0 * (q0 - qm1))
    accept = (ql - q0) * (ql - qmp) <= 0.0
    dm1 = qm2 - 2.0 * qm1 + q0
    d0 = qm1 - 2.0 * q0 + qp1
    dp1 = q0 - 2.0 * qp1 + qp2
    dm4p = minmod4(4.0 * d0 - dp1, 4.0 * dp1 - d0, d0, dp1)
    dm4m = minmod4(4.0 * d0 - dm1, 4.0 * dm1 - d0, d0, dm1)
    qul = q0 + 4.0 * (q0 - qm1)
    qmd = 0.5 * (q0 + qp1) - 0.5 * dm4p
    qlc = q0 + 0.5 * (q0 - qm1) + 4.0 / 3.0 * dm4m
    qmin = np.maximum(np.minimum(np.minimum(q0, qp1), qmd),
                      np.minimum(np.minimum(q0, qul), qlc))
    qmax = np.minimum(np.maximum(np.maximum(q0, qp1), qmd),
                      np.maximum(np.maximum(q0, qul), qlc))
    lim = ql + minmod(qmin - ql, qmax - ql)
    return np.where(accept, ql, lim)


def face_states(q, d, lo, hi, g, take):
    """Left and right MP5 states at faces f in [lo, hi) along direction d
    (face f+1/2 between cells f and f+1)."""
    c = lambda s: take(q, d, lo + s, hi + s, g)
    left = mp5(c(-2), c(-1), c(0), c(1), c(2))
    right = mp5(c(3), c(2), c(1), c(0), c(-1))
    return left, right
