"""Grid description: interior size, ghost depth, coordinates and boundaries.

Conventions (shared by every consumer):
  * arrays are indexed [k][j][i] (x^3, x^2, x^1), x^1 fastest;
  * interior cells have i in [0, n1), ghosts extend ng cells on each side;
  * cell i has its centre at x0 + (i + 1/2) dx;
  * the face "i + 1/2" (upper face of cell i) is stored at index i;
  * the edge (i + 1/2, j + 1/2, k) is stored at [k][j][i], and cyclically for
    the other two edge families.
"""
from dataclasses import dataclass, field
import math

CART = 0      # (x, y, z)
LOGSPH = 1    # (ln r, theta, phi)

BC_PERIODIC = 0
BC_OUTFLOW = 1
BC_AXIS = 2


@dataclass
class GridSpec:
    n: tuple                      # interior zones (n1, n2, n3)
    ng: int = 5
    coord: int = CART
    x0: tuple = (0.0, 0.0, 0.0)
    dx: tuple = None
    bc: tuple = (BC_PERIODIC,) * 6   # -x1, +x1, -x2, +x2, -x3, +x3
    gamma_ad: float = 4.0 / 3.0
    cfl: float = 0.4
    # floors: rho_fl = rho_fl_a * r**rho_fl_n, p_fl = p_fl_a * r**p_fl_n (0 = off)
    rho_fl_a: float = 0.0
    rho_fl_n: float = 0.0
    p_fl_a: float = 0.0
    p_fl_n: float = 0.0
    w_max: float = 0.0            # Lorentz-factor cap (0 = off)
    newton_maxit: int = 50
    newton_tol: float = 1e-14
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        if self.dx is None:
            self.dx = tuple(1.0 / v for v in self.n)
        self.dx = tuple(float(v) for v in self.dx)
        self.x0 = tuple(float(v) for v in self.x0)

    @property
    def shape(self):
        """Ghosted array shape in [k][j][i] order."""
        g = self.ng
        return (self.n[2] + 2 * g, self.n[1] + 2 * g, self.n[0] + 2 * g)

    @property
    def zones(self):
        return self.n[0] * self.n[1] * self.n[2]

    def centres(self, axis):
        """Code coordinate of cell centres along axis (0=x1) incl. ghosts."""
        g = self.ng
        return [self.x0[axis] + (i + 0.5) * self.dx[axis]
                for i in range(-g, self.n[axis] + g)]

    def faces(self, axis):
        """Code coordinate of faces i+1/2 (stored at i) along axis incl. ghosts."""
        g = self.ng
        return [self.x0[axis] + (i + 1.0) * self.dx[axis]
                for i in range(-g, self.n[axis] + g)]


def box(n, ng=5, **kw):
    """Periodic Cartesian unit box with n^3 zones."""
    return GridSpec(n=(n, n, n), ng=ng, coord=CART, x0=(0.0, 0.0, 0.0),
                    dx=(1.0 / n,) * 3, bc=(BC_PERIODIC,) * 6, **kw)


def torus_grid(n1, n2, n3, r_in=1.2, r_out=50.0, ng=5, **kw):
    """Log-spherical (ln r, theta, phi) grid: outflow in r, axis in theta,
    periodic in phi."""
    x0 = (math.log(r_in), 0.0, 0.0)
    dx = ((math.log(r_out) - math.log(r_in)) / n1, math.pi / n2,
          2.0 * math.pi / n3)
    return GridSpec(n=(n1, n2, n3), ng=ng, coord=LOGSPH, x0=x0, dx=dx,
                    bc=(BC_OUTFLOW, BC_OUTFLOW, BC_AXIS, BC_AXIS,
                        BC_PERIODIC, BC_PERIODIC), **kw)
