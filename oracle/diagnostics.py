"""Torus-run diagnostics (oracle, FP64): shell fluxes through x^1 = const
surfaces and the MRI resolution.  Test infrastructure: only the tests, the
smoke check and the benchmark's CPU baseline use it.

Shell fluxes.

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


def fluid_frame(st, m):
    """Four-velocity u^mu = (W / alpha, W (v^i - beta^i / alpha)), the field
    in the fluid frame b^mu (b^t, b^i as below), b^2 and the angular velocity
    Omega = u^3 / u^t of a state (physics.state) with 3+1 metric m."""
    al = m["alpha"]
    beta = (m["beta1"], m["beta2"], m["beta3"])
    w_l = st["W"]
    bt = w_l * st["vB"] / al
    b = [st["B"][d] / w_l + bt * (al * st["v"][d] - beta[d]) for d in range(3)]
    return {"ut": w_l / al, "u": [w_l * (st["v"][d] - beta[d] / al) for d in range(3)],
            "bt": bt, "b": b, "b2": st["B2"] / w_l ** 2 + st["vB"] ** 2,
            "Omega": al * st["v"][2] - beta[2]}


def mri_quality(solver, rho_cut, q_min=8.0):
    """MRI resolution of the current state (a diagnostic of the torus runs,
    whose turbulence is driven by the magneto-rotational instability): the
    number of zones per wavelength of the fastest-growing MRI mode along x^2
    (theta) and x^3 (phi),

      Q_d = lambda_d / Delta x^(d),   lambda_d = 2 pi |b^(d)| / (|Omega| sqrt(rho h + b^2)),

    with b^mu the field in the fluid frame, b^(d) = sqrt(g_dd) b^d its
    orthonormal component, Delta x^(d) = sqrt(g_dd) dx^d the proper zone
    width (the metric factors cancel: Q_d = 2 pi |b^d| / (|Omega| dx^d
    sqrt(rho h + b^2))), and Omega = u^3 / u^t the angular velocity.  In
    3+1 form (v the Eulerian velocity, W its Lorentz factor):
      b^t = W (v_i B^i) / alpha,  b^i = B^i / W + b^t (alpha v^i - beta^i),
      b^2 = B^2 / W^2 + (v_i B^i)^2,  Omega = alpha v^3 - beta^3.
    Per x^1 shell i, over the body zones (rho > rho_cut), with the mass weight
    w = rho sqrt(gamma): sum w Q_2, sum w Q_3, sum w, the number of body zones
    and the numbers with Q_2 >= q_min and Q_3 >= q_min.  Returns the per-zone
    Q_2, Q_3 and those six shell arrays."""
    g = solver.grid
    m = solver.centre_metric()
    P = {k: solver.interior(v) for k, v in solver.P.items()}
    st = physics.state(P["rho"], (P["u1"], P["u2"], P["u3"]), P["p"],
                       (P["B1"], P["B2"], P["B3"]), m, g.gamma_ad)
    ff = fluid_frame(st, m)
    bcon, b2, omega = ff["b"], ff["b2"], ff["Omega"]
    den = np.abs(omega) * np.sqrt(P["rho"] * st["h"] + b2)
    # gas at rest without field (Omega = b = 0, outside any body) gives 0/0
    with np.errstate(invalid="ignore", divide="ignore"):
        q2 = 2.0 * np.pi * np.abs(bcon[1]) / (den * g.dx[1])
        q3 = 2.0 * np.pi * np.abs(bcon[2]) / (den * g.dx[2])
    body = P["rho"] > rho_cut
    wt = np.broadcast_to(P["rho"] * m["sqrtg"], q2.shape)
    z = np.zeros_like(q2)
    shell = lambda a: np.where(body, a, z).sum(axis=(0, 1))
    return {"Q2": q2, "Q3": q3,
            "wQ2": shell(wt * q2), "wQ3": shell(wt * q3), "w": shell(wt),
            "n_body": body.sum(axis=(0, 1)).astype(np.float64),
            "n_Q2_ok": (body & (q2 >= q_min)).sum(axis=(0, 1)).astype(np.float64),
            "n_Q3_ok": (body & (q3 >= q_min)).sum(axis=(0, 1)).astype(np.float64)}
