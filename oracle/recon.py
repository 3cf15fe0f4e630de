"""Alternative interface reconstructions (oracle, FP64).  Test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use it.

Paper, Introduction: the scheme offers high-order reconstruction algorithms
(plural).  MP5 (oracle/mp5.py) is the default; two further members of the
same family are provided, both acting on point values at cell centres, as a
finite-difference scheme does:

WENO5 -- weighted essentially non-oscillatory interpolation (Jiang & Shu
1996 smoothness indicators), in its point-value form.  For the left state
at face j+1/2 from q_{j-2}..q_{j+2}:
  * three quadratic interpolants at x_{j+1/2} (exact for degree <= 2):
      p0 = ( 3 q_{j-2} - 10 q_{j-1} + 15 q_j) / 8
      p1 = (  -q_{j-1} +  6 q_j     +  3 q_{j+1}) / 8
      p2 = ( 3 q_j     +  6 q_{j+1} -    q_{j+2}) / 8
  * linear weights d = (1, 10, 5) / 16, for which sum d_k p_k is the
    degree-4 interpolant (3, -20, 90, 60, -5) / 128;
  * smoothness indicators
      b0 = 13/12 (q_{j-2} - 2 q_{j-1} + q_j)^2 + 1/4 (q_{j-2} - 4 q_{j-1} + 3 q_j)^2
      b1 = 13/12 (q_{j-1} - 2 q_j + q_{j+1})^2 + 1/4 (q_{j-1} - q_{j+1})^2
      b2 = 13/12 (q_j - 2 q_{j+1} + q_{j+2})^2 + 1/4 (3 q_j - 4 q_{j+1} + q_{j+2})^2
  * alpha_k = d_k / (eps + b_k)^2, w_k = alpha_k / sum alpha, with
    eps = 1e-6 (the published value), and qL = sum w_k p_k.

MP7 -- the seventh-order member of the monotonicity-preserving family
(Suresh & Huynh 1997): the unlimited value is the degree-6 Lagrange
interpolant of the point values q_{j-3..j+3} at x_{j+1/2},
  qL7 = (-5 q_{j-3} + 42 q_{j-2} - 175 q_{j-1} + 700 q_j + 525 q_{j+1}
         - 70 q_{j+2} + 7 q_{j+3}) / 1024,
limited by the MP limiter of MP5 (its bounds from q_{j-2..j+2}).  Its
stencil reaches three cells past the face on each side, so a grid using it
carries six ghost layers.

PLM-MC -- piecewise linear reconstruction with the monotonized-central
slope limiter (van Leer 1977), the lower-order member:
  qL(j+1/2) = q_j + 1/2 MC(q_j - q_{j-1}, q_{j+1} - q_j),
  MC(a, b) = minmod(2 a, 2 b, (a + b) / 2).

Right states at j+1/2 apply the same maps to the mirrored stencil, as for
MP5.
"""
import numpy as np

from . import mp5 as _mp5

WENO_EPS = 1e-6
WENO_D = (1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0)
METHODS = ("mp5", "weno5", "plm", "mp7")
# ghost layers each method needs with the sixth-order derivative: its
# stencil's reach past the face (3 for the five- and six-cell stencils, 4 for
# MP7's eight) plus the two further faces of that derivative (one fewer with
# the fourth-order derivative, whose stencil reaches one face less)
NG_OF = {"mp5": 5, "weno5": 5, "plm": 5, "mp7": 6}


def mp7_unlimited(qm3, qm2, qm1, q0, qp1, qp2, qp3):
    """Degree-6 interpolant of q_{j-3..j+3} at the face between q0 and qp1."""
    return (-5.0 * qm3 + 42.0 * qm2 - 175.0 * qm1 + 700.0 * q0 + 525.0 * qp1
            - 70.0 * qp2 + 7.0 * qp3) / 1024.0


def mp7(qm3, qm2, qm1, q0, qp1, qp2, qp3):
    """MP7 left state at the face between q0 and qp1."""
    return _mp5.mp_limit(mp7_unlimited(qm3, qm2, qm1, q0, qp1, qp2, qp3), qm2, qm1, q0, qp1, qp2)


def weno5_candidates(qm2, qm1, q0, qp1, qp2):
    p0 = (3.0 * qm2 - 10.0 * qm1 + 15.0 * q0) / 8.0
    p1 = (-qm1 + 6.0 * q0 + 3.0 * qp1) / 8.0
    p2 = (3.0 * q0 + 6.0 * qp1 - qp2) / 8.0
    return p0, p1, p2


def weno5_indicators(qm2, qm1, q0, qp1, qp2):
    b0 = 13.0 / 12.0 * (qm2 - 2.0 * qm1 + q0) ** 2 + 0.25 * (qm2 - 4.0 * qm1 + 3.0 * q0) ** 2
    b1 = 13.0 / 12.0 * (qm1 - 2.0 * q0 + qp1) ** 2 + 0.25 * (qm1 - qp1) ** 2
    b2 = 13.0 / 12.0 * (q0 - 2.0 * qp1 + qp2) ** 2 + 0.25 * (3.0 * q0 - 4.0 * qp1 + qp2) ** 2
    return b0, b1, b2


def weno5(qm2, qm1, q0, qp1, qp2, eps=WENO_EPS):
    """WENO5 left state at the face between q0 and qp1."""
    p = weno5_candidates(qm2, qm1, q0, qp1, qp2)
    b = weno5_indicators(qm2, qm1, q0, qp1, qp2)
    a = [WENO_D[k] / (eps + b[k]) ** 2 for k in range(3)]
    s = a[0] + a[1] + a[2]
    return (a[0] * p[0] + a[1] * p[1] + a[2] * p[2]) / s


def mc_slope(a, b):
    """Monotonized-central limited slope minmod(2a, 2b, (a+b)/2)."""
    c = 0.5 * (a + b)
    same = (np.sign(a) == np.sign(b)) & (np.sign(a) != 0)
    m = np.minimum(np.minimum(np.abs(2.0 * a), np.abs(2.0 * b)), np.abs(c))
    return np.where(same, np.sign(a) * m, 0.0)


def plm(qm1, q0, qp1):
    """PLM-MC left state at the face between q0 and qp1."""
    return q0 + 0.5 * mc_slope(q0 - qm1, qp1 - q0)


def face_states(q, d, lo, hi, g, take, method="mp5"):
    """Left and right states at faces f in [lo, hi) along direction d (face
    f+1/2 between cells f and f+1) with the given reconstruction."""
    if method == "mp5":
        return _mp5.face_states(q, d, lo, hi, g, take)
    c = lambda s: take(q, d, lo + s, hi + s, g)
    if method == "weno5":
        return (weno5(c(-2), c(-1), c(0), c(1), c(2)),
                weno5(c(3), c(2), c(1), c(0), c(-1)))
    if method == "plm":
        return plm(c(-1), c(0), c(1)), plm(c(2), c(1), c(0))
    if method == "mp7":
        return (mp7(c(-3), c(-2), c(-1), c(0), c(1), c(2), c(3)),
                mp7(c(4), c(3), c(2), c(1), c(0), c(-1), c(-2)))
    raise ValueError("unknown reconstruction %r" % (method,))
