"""Shell fluxes through x^1 = const surfaces (oracle, FP64).

A diagnostic of the torus runs (accretion rate, energy flux and magnetic flux
through spheres; the paper's torus use case, Introduction and Fig. 1), not
part of the time step.  In (ln r, theta, phi) coordinates the densitised
x^1-fluxes already include sqrt(gamma) and the Jacobian, so the flux through
the sphere r = r_i is the sum over the shell's cells of the x^1-flux times
dx^2 dx^3:

  F_D[i]   = sum_{j,k} F^1[D](i,j,k) dx^2 dx^3       (accretion rate = -F_D)
  F_tau[i] = sum_{j,k} F^1[tau](i,j,k) dx^2 dx^3
  F^1[D] = sqrt(gamma) D (alpha v^1 - beta^1),
  F^1[tau] = sqrt(gamma) (alpha (S^1 - v^1 D) - beta^1 tau)
           (pointwise fluxes of the cell-centred state, physics.flux)
  Phi[i]   = 1/2 sum_{j,k} |B_face^1(i,j,k)| dx^2 dx^3  (upper x^1 face of cell i)
  Phi_s[i] = sum_{j,k} B_face^1(i,j,k) dx^2 dx^3       (signed)

with B_face^1 the densitised face field.  Sums in NumPy's order; the GPU sums
in another order and rounds the pointwise state differently, so parity is
relative to the size of the terms that cancel in each flux: scale_D =
sum sqrt(gamma) D (|alpha v^1| + |beta^1|) (the two nearly cancel for gas at
rest in the coordinates), scale_tau = sum sqrt(gamma) (alpha (|S^1| + |v^1| D)
+ |beta^1 tau|), scale_B = sum |B_face^1| (all times dx^2 dx^3).
"""
import numpy as np

from . import physics


def shell_fluxes(solver):
    """{F_D, F_tau, Phi, Phi_s, scale_D, scale_tau, scale_B} over the interior
    x^1 index of the solver's current state (scale_*: sums of |terms|)."""
    g = solver.grid
    m = solver.centre_metric()
    P = {k: solver.interior(v) for k, v in solver.P.items()}
    st = physics.state(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"],
                       (P["B1"], P["B2"], P["B3"]), m, g.gamma_ad)
    f = physics.flux(st, m, 0)
    area = g.dx[1] * g.dx[2]
    bf = solver.interior(solver.U["Bf1"])
    sg, al, b1, v1 = m["sqrtg"], m["alpha"], m["beta1"], st["v"][0]
    sd = sg * st["D"] * (np.abs(al * v1) + np.abs(b1))
    st_ = sg * (al * (np.abs(st["Su"][0]) + np.abs(v1) * st["D"]) + np.abs(b1 * st["tau"]))
    shell = lambda a: np.broadcast_to(a, bf.shape).sum(axis=(0, 1)) * area
    return {"F_D": f[0].sum(axis=(0, 1)) * area,
            "F_tau": f[4].sum(axis=(0, 1)) * area,
            "Phi": 0.5 * np.abs(bf).sum(axis=(0, 1)) * area,
            "Phi_s": bf.sum(axis=(0, 1)) * area,
            "scale_D": shell(sd), "scale_tau": shell(st_),
            "scale_B": np.abs(bf).sum(axis=(0, 1)) * area}
