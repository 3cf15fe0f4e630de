"""Precision form (reconstruction, face physics, HLL and edge field in FP32;
derivatives, sources, RK, inversion and metric in FP64): GPU kernels against
the oracle's float32 form, and the error of the form against FP64."""
import numpy as np
import pytest

from helpers import max_rel, interior

gpu = pytest.mark.gpu
PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _grid(g, d, precision):
    from paper_1810_04597_amd.grid import Grid
    G = Grid(g, precision=precision)
    G.curl_potential(d)
    G.set_primitives(d)
    return G


@gpu
def test_fp32_form_rhs_matches_oracle_fp32_form():
    """Same float32 algorithm on both sides: differences are float32
    rounding-order effects, a few ulps of the flux scale."""
    _torch()
    from workloads import box
    from oracle.scheme import Solver
    g, d = box.turbulent_box(16)
    s = Solver(g, precision="fp32")
    s.curl_potential(d)
    s.set_primitives(d)
    L_o = s.rhs()
    G = _grid(g, d, 1)
    L_g = G.read_group(G.rhs(), CONS, interior=True)
    s64 = Solver(g)
    s64.curl_potential(d)
    s64.set_primitives(d)
    L_64 = s64.rhs()
    for k in CONS:
        scale = np.max(np.abs(L_o[k]))
        e32 = np.max(np.abs(L_g[k] - L_o[k])) / scale
        e_form = np.max(np.abs(L_o[k] - L_64[k])) / scale
        # GPU FP32 form is close to the oracle FP32 form, and both differ
        # from FP64 by the float32 rounding level
        assert e32 < 2e-4, (k, e32)
        assert e_form < 2e-4, (k, e_form)


@gpu
def test_fp32_form_error_after_steps():
    """32^3 box, 10 steps with a fixed dt: the FP32 form stays within 1e-6
    (field-max relative) of the FP64 form on the GPU, the same size as the
    oracle's own FP32-vs-FP64 difference."""
    _torch()
    from workloads import box
    g, d = box.turbulent_box(32)
    G64 = _grid(g, d, 0)
    G32 = _grid(g, d, 1)
    for _ in range(10):
        G64.rk_step(2e-3)
        G32.rk_step(2e-3)
    a = G32.to_numpy("prim", interior=True)
    b = G64.to_numpy("prim", interior=True)
    errs = {k: float(np.max(np.abs(a[k] - b[k])) / np.max(np.abs(b[k]))) for k in PRIM}
    print("FP32-form vs FP64 after 10 steps:", errs)
    assert max(errs.values()) < 1e-6, errs
    assert G32.diagnostics()["max_divb"] < 1e-12
