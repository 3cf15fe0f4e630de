"""The GPU path against an exact solution (independent of the oracle): a
smooth entropy wave advected along each axis on an n x 1 x 1 periodic grid
(uniform v, p and B; rho = 1 + 0.2 sin 2 pi (x - v t)), run to t = 0.2 with
a time step shrinking as n^(-5/3) so the third-order time error stays below
the fifth-order space error.  The mean density error falls at fifth order
(MP5 with the sixth-order D), and at fourth order with the fourth-order D."""
import numpy as np
import pytest

gpu = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _wave_error(n, axis, t_end, deriv_order):
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    g, d = box.entropy_wave_1d(n, axis=axis)
    G = Grid(g, deriv_order=deriv_order)
    G.set_face_fields(d)
    G.set_primitives(d)
    dt0 = 0.4 * (1.0 / 16) * (16.0 / n) ** (5.0 / 3.0)
    nsteps = int(np.ceil(t_end / dt0))
    for _ in range(nsteps):
        G.rk_step(t_end / nsteps)
    _, de = box.entropy_wave_1d(n, axis=axis, t=t_end)
    rho = G.to_numpy("prim", interior=True)["rho"]
    G.close()
    return float(np.mean(np.abs(rho - de["rho"])))


@gpu
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fifth_order_convergence_on_gpu(axis):
    _torch()
    errs = [_wave_error(n, axis, 0.2, 6) for n in (16, 32, 64)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] >= 4.7, (errs, orders)


@gpu
def test_fourth_order_convergence_with_d4_on_gpu():
    _torch()
    errs = [_wave_error(n, 0, 0.2, 4) for n in (16, 32, 64)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 3.7 <= orders[-1] <= 4.4, (errs, orders)
