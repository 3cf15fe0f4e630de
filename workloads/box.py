"""Initial data on periodic Cartesian boxes (Minkowski background).

Turbulent box (the SRMHD workloads at 32^3, 256^3 and 512^3):
  * mode set K = {k in Z^3 : 0 < |k|^2 <= 16}, 256 vectors in lexicographic
    order of (k1, k2, k3);
  * one random phase per mode and per field, drawn from
    numpy.random.default_rng(seed).uniform(0, 2 pi) in the field order
    drho, dv1, dv2, dv3, A1, A2, A3;
  * g_f(x) = sum_k cos(2 pi k.x + phi_{f,k});
  * rho = 1 + 0.1 g_rho / max|g_rho|, v^i = 0.1 g_vi / max|g_v|, p = 0.1,
    u^i = W v^i;
  * vector potential A_i = s g_Ai on the edges, s chosen so that the rms of
    the continuum curl of A at cell centres is 0.1.
All maxima and the rms are taken on a fixed 64^3 sampling grid, so the
continuous fields do not depend on the resolution.  Fields are evaluated with
an inverse FFT (exact for n >= 9) or a direct sum (any n).
"""
import itertools
import numpy as np

from .grid import box as box_grid

SEED = 1810
MODES = np.array([k for k in itertools.product(range(-4, 5), repeat=3)
                  if 0 < k[0] ** 2 + k[1] ** 2 + k[2] ** 2 <= 16], dtype=np.int64)
FIELDS = ("drho", "dv1", "dv2", "dv3", "A1", "A2", "A3")
SAMPLE_N = 64


def phases(seed=SEED):
    rng = np.random.default_rng(seed)
    return {f: rng.uniform(0.0, 2.0 * np.pi, size=len(MODES)) for f in FIELDS}


def _eval_fft(phi, n, offs, deriv=None):
    """g on the n^3 grid at positions (m + offs)/n, [k][j][i] order.

    deriv: None or axis index a (0 = x1) for d g / d x^a."""
    X = np.zeros((n, n, n), dtype=np.complex128)
    k1, k2, k3 = MODES[:, 0], MODES[:, 1], MODES[:, 2]
    c = np.exp(1j * phi)
    c = c * np.exp(2j * np.pi * (k1 * offs[0] + k2 * offs[1] + k3 * offs[2]) / n)
    if deriv is not None:
        c = c * (2j * np.pi * MODES[:, deriv])
    np.add.at(X, (k3 % n, k2 % n, k1 % n), c)
    return np.real(np.fft.ifftn(X)) * float(n) ** 3


def _eval_direct(phi, n, offs, deriv=None):
    x = [(np.arange(n) + offs[a]) / n for a in range(3)]
    out = np.zeros((n, n, n))
    for m, k in enumerate(MODES):
        th = (2 * np.pi * (k[2] * x[2][:, None, None] + k[1] * x[1][None, :, None]
                           + k[0] * x[0][None, None, :]) + phi[m])
        if deriv is None:
            out += np.cos(th)
        else:
            out += -2 * np.pi * k[deriv] * np.sin(th)
    return out


def evaluate(phi, n, offs, deriv=None, method="auto"):
    if method == "direct" or (method == "auto" and n < 9):
        return _eval_direct(phi, n, offs, deriv)
    return _eval_fft(phi, n, offs, deriv)


# positions of the edge families relative to the cell index, (x1, x2, x3)
EDGE_OFFS = {"A1": (0.5, 1.0, 1.0), "A2": (1.0, 0.5, 1.0), "A3": (1.0, 1.0, 0.5)}
CENTRE = (0.5, 0.5, 0.5)


def _wrap_ghosts(a, ng):
    """Periodic extension of an n^3 array to (n+2ng)^3."""
    return np.pad(a, ng, mode="wrap")


def normalisation(seed=SEED):
    """Scale factors (rho, v, A) from the 64^3 sampling grid."""
    ph = phases(seed)
    n = SAMPLE_N
    g_rho = evaluate(ph["drho"], n, CENTRE)
    gv = [evaluate(ph[f], n, CENTRE) for f in ("dv1", "dv2", "dv3")]
    vmax = np.sqrt(gv[0] ** 2 + gv[1] ** 2 + gv[2] ** 2).max()
    # continuum curl of g_A at the centres
    d = {(f, a): evaluate(ph[f], n, CENTRE, deriv=a)
         for f in ("A1", "A2", "A3") for a in range(3)}
    bx = d[("A3", 1)] - d[("A2", 2)]
    by = d[("A1", 2)] - d[("A3", 0)]
    bz = d[("A2", 0)] - d[("A1", 1)]
    brms = np.sqrt(np.mean(bx ** 2 + by ** 2 + bz ** 2))
    return {"rho": 0.1 / np.abs(g_rho).max(), "v": 0.1 / vmax, "A": 0.1 / brms}


def turbulent_box(n, seed=SEED, ng=5, method="auto"):
    """Turbulent SRMHD box.  Returns (grid, data) with interior primitives
    rho, u1, u2, u3, p ([k][j][i], n^3) and ghosted edge potentials A1..A3."""
    grid = box_grid(n, ng=ng)
    ph = phases(seed)
    sc = normalisation(seed)
    rho = 1.0 + sc["rho"] * evaluate(ph["drho"], n, CENTRE, method=method)
    v = [sc["v"] * evaluate(ph[f], n, CENTRE, method=method)
         for f in ("dv1", "dv2", "dv3")]
    w = 1.0 / np.sqrt(1.0 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    data = {"rho": rho, "u1": w * v[0], "u2": w * v[1], "u3": w * v[2],
            "p": np.full((n, n, n), 0.1)}
    for f in ("A1", "A2", "A3"):
        data[f] = _wrap_ghosts(sc["A"] * evaluate(ph[f], n, EDGE_OFFS[f], method=method), ng)
    return grid, data


def _eval_direct_shape(phi, n, offs):
    """g on an n[0] x n[1] x n[2] grid at positions (m_a + offs_a)/n_a,
    [k][j][i] order (direct sum over the modes)."""
    x = [(np.arange(n[a]) + offs[a]) / n[a] for a in range(3)]
    out = np.zeros((n[2], n[1], n[0]))
    for m, k in enumerate(MODES):
        out += np.cos(2 * np.pi * (k[2] * x[2][:, None, None] + k[1] * x[1][None, :, None]
                                   + k[0] * x[0][None, None, :]) + phi[m])
    return out


def turbulent_box_shape(n1, n2, n3, seed=SEED, ng=5):
    """The turbulent box's continuous fields sampled on a periodic unit box
    with n1 x n2 x n3 zones (spacings 1/n_a): the same fields as
    turbulent_box(n) when n1 = n2 = n3 = n.  Any n_a >= 1: the ghost layers
    of the potentials wrap as often as a thin direction needs (one zone: a
    direction the fields do not vary along).  Returns (grid, data)."""
    from .grid import GridSpec, CART, BC_PERIODIC
    n = (n1, n2, n3)
    assert min(n) >= 1
    grid = GridSpec(n=n, ng=ng, coord=CART, x0=(0.0, 0.0, 0.0),
                    dx=tuple(1.0 / x for x in n), bc=(BC_PERIODIC,) * 6)
    ph = phases(seed)
    sc = normalisation(seed)
    rho = 1.0 + sc["rho"] * _eval_direct_shape(ph["drho"], n, CENTRE)
    v = [sc["v"] * _eval_direct_shape(ph[f], n, CENTRE) for f in ("dv1", "dv2", "dv3")]
    w = 1.0 / np.sqrt(1.0 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    data = {"rho": rho, "u1": w * v[0], "u2": w * v[1], "u3": w * v[2],
            "p": np.full((n3, n2, n1), 0.1)}
    for f in ("A1", "A2", "A3"):
        data[f] = _wrap_ghosts(sc["A"] * _eval_direct_shape(ph[f], n, EDGE_OFFS[f]), ng)
    return grid, data


def entropy_wave(n, t=0.0, ng=5, amp=0.2, v=(0.3, 0.2, 0.1), p=1.0,
                 b=(0.3, 0.2, 0.1)):
    """Smooth entropy wave rho = 1 + amp sin(2 pi (x+y+z - (v1+v2+v3) t)) with
    uniform v, p and B: an exact solution (advected density).  Returns
    (grid, data) with interior primitives and ghosted face fields B1f..B3f."""
    grid = box_grid(n, ng=ng)
    x = (np.arange(n) + 0.5) / n
    s = x[None, None, :] + x[None, :, None] + x[:, None, None]
    rho = 1.0 + amp * np.sin(2 * np.pi * (s - (v[0] + v[1] + v[2]) * t))
    w = 1.0 / np.sqrt(1.0 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    shp = (n, n, n)
    data = {"rho": rho, "u1": np.full(shp, w * v[0]), "u2": np.full(shp, w * v[1]),
            "u3": np.full(shp, w * v[2]), "p": np.full(shp, p)}
    gs = grid.shape
    for a, f in enumerate(("B1f", "B2f", "B3f")):
        data[f] = np.full(gs, b[a])
    return grid, data


def uniform_state(grid, rho=1.0, p=0.1):
    """Static uniform state with B = 0 on any grid."""
    shp = (grid.n[2], grid.n[1], grid.n[0])
    data = {"rho": np.full(shp, rho), "u1": np.zeros(shp), "u2": np.zeros(shp),
            "u3": np.zeros(shp), "p": np.full(shp, p)}
    for f in ("B1f", "B2f", "B3f"):
        data[f] = np.zeros(grid.shape)
    return data


def entropy_wave_1d(n, axis=0, t=0.0, ng=5, amp=0.2, v=(0.3, 0.2, 0.1), p=1.0,
                    b=(0.3, 0.2, 0.1), ntrans=1):
    """Entropy wave varying along one axis only, on an n x ntrans x ntrans
    (permuted) periodic grid: rho = 1 + amp sin(2 pi (x_a - v_a t))."""
    from .grid import GridSpec
    nn = [ntrans, ntrans, ntrans]
    nn[axis] = n
    grid = GridSpec(n=tuple(nn), ng=ng, dx=tuple(1.0 / x for x in nn))
    x = (np.arange(n) + 0.5) / n
    prof = 1.0 + amp * np.sin(2 * np.pi * (x - v[axis] * t))
    shp = (nn[2], nn[1], nn[0])
    view = [1, 1, 1]
    view[2 - axis] = n
    rho = np.broadcast_to(prof.reshape(view), shp).copy()
    w = 1.0 / np.sqrt(1.0 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    data = {"rho": rho, "u1": np.full(shp, w * v[0]), "u2": np.full(shp, w * v[1]),
            "u3": np.full(shp, w * v[2]), "p": np.full(shp, p)}
    for a, f in enumerate(("B1f", "B2f", "B3f")):
        data[f] = np.full(grid.shape, b[a])
    return grid, data


def blast_box(n, ng=5, rho_in=1e-2, p_in=1.0, rho_out=1e-4, p_out=3e-5, r0=0.08, b0=0.1,
              centre=(0.5, 0.5, 0.5)):
    """Magnetised blast wave (the relativistic MHD blast problem of Komissarov
    1999, scaled to the periodic unit box): a sphere of radius r0 about
    `centre` (periodic distances) at rho_in, p_in in a medium at rho_out,
    p_out, at rest, in a uniform field B = (b0, 0, 0).  n: zones per side, or
    (n1, n2, n3).  The jump of four orders of magnitude in pressure makes the
    high-order update leave unphysical states next to the shell in the first
    steps.  Returns (grid, data) with interior primitives and ghosted face
    fields."""
    from .grid import GridSpec
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    grid = GridSpec(n=nn, ng=ng, dx=tuple(1.0 / x for x in nn))
    x = [(np.arange(nn[a]) + 0.5) / nn[a] - centre[a] for a in range(3)]
    x = [v - np.round(v) for v in x]
    r = np.sqrt(x[0][None, None, :] ** 2 + x[1][None, :, None] ** 2 + x[2][:, None, None] ** 2)
    inside = r < r0
    shp = (nn[2], nn[1], nn[0])
    data = {"rho": np.where(inside, rho_in, rho_out), "u1": np.zeros(shp), "u2": np.zeros(shp),
            "u3": np.zeros(shp), "p": np.where(inside, p_in, p_out)}
    data["B1f"] = np.full(grid.shape, b0)
    data["B2f"] = np.zeros(grid.shape)
    data["B3f"] = np.zeros(grid.shape)
    return grid, data
