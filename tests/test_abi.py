"""The C-ABI library on the host (no GPU needed): it loads, exports every
function include/grmhd.h declares, the Python binding marshals each of them,
and descriptor validation rejects bad input before any device call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "grmhd.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grmhd_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_1810_04597_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libgrmhd.so is not built (run __graft_entry__.build())")
    return L, L.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("grmhd_init_grid", "grmhd_set_metric", "grmhd_rhs", "grmhd_rk_step",
                     "grmhd_cons2prim", "grmhd_diagnostics", "grmhd_destroy"):
        assert required in names
    assert len(names) >= 20


def test_library_exports_every_declared_function():
    L, lib = _lib()
    raw = C.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(raw, n)]
    assert not missing, missing
    # and the binding sets up every one of them
    assert sorted(L.EXPORTS) == _declared()


def test_binding_structs_match_the_library_layout():
    # the library checks the same sizes with static_assert when it is built
    from paper_1810_04597_amd import _lib as L
    assert C.sizeof(L.GridDesc) == 184
    assert C.sizeof(L.Diag) == 280
    assert L.Diag.run_c2p_fail.offset == 216 and L.Diag.run_troubled.offset == 272
    assert C.sizeof(L.Profile) == 16 * L.PROF_NCLASS


def _desc(L, **kw):
    from workloads.grid import box
    d = L.make_desc(box(8))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,msg", [
    ("ng", 3, "ng must be 4, 5 or 6"),
    ("ng", 7, "ng must be 4, 5 or 6"),
    ("ng", 4, "ng = 4 needs deriv_order 4"),
    ("precision", 7, "bad precision"),
    ("c2p_guess", 3, "bad c2p_guess"),
    ("newton_maxit", 0, "bad newton_maxit"),
    ("gamma_ad", 1.0, "gamma_ad"),
    ("recon", 4, "bad recon"),
    ("recon", -1, "bad recon"),
    ("recon", 3, "MP7 needs ng = 6 (5 with deriv_order 4)"),
    ("deriv_order", 5, "deriv_order"),
    ("fallback", 2, "fallback must be 0 or 1"),
    ("fallback", -1, "fallback must be 0 or 1"),
])
def test_descriptor_validation_before_any_device_call(field, value, msg):
    L, lib = _lib()
    h = C.c_void_p()
    rc = lib.grmhd_init_grid(C.byref(_desc(L, **{field: value})), None, C.byref(h))
    assert rc == L.EINVAL
    assert msg in lib.grmhd_last_error().decode()
    assert not h.value


def test_descriptor_validation_of_boundaries():
    L, lib = _lib()
    h = C.c_void_p()
    d = _desc(L)
    d.bc[0] = L.BC_PERIODIC
    d.bc[1] = L.BC_OUTFLOW
    assert lib.grmhd_init_grid(C.byref(d), None, C.byref(h)) == L.EINVAL
    assert "pairs" in lib.grmhd_last_error().decode()
    d = _desc(L)
    d.bc[2] = d.bc[3] = L.BC_AXIS
    d.n[1] = 4
    assert lib.grmhd_init_grid(C.byref(d), None, C.byref(h)) == L.EINVAL
    assert "n2 >= ng + 1" in lib.grmhd_last_error().decode()


def test_null_handles_are_rejected():
    L, lib = _lib()
    assert lib.grmhd_rk_step(None, C.c_double(0.0), None) == L.EINVAL
    assert lib.grmhd_get_layout(None, None) == L.EINVAL
    assert lib.grmhd_set_profiling(None, 1) == L.EINVAL


def test_profile_class_names():
    L, lib = _lib()
    names = [lib.grmhd_profile_class_name(c).decode() for c in range(L.PROF_NCLASS)]
    for n in ("sweep_x1", "edge_x3", "update", "cons2prim", "learned_guess", "fallback"):
        assert n in names


@pytest.mark.parametrize("ng,order,recon", [(4, 4, 0), (4, 4, 1), (4, 4, 2), (5, 4, 3)])
def test_narrow_grids_pass_validation_with_the_fourth_order(ng, order, recon):
    """Four ghost layers with the fourth-order derivative (five for MP7) get
    past the descriptor checks (without a device the call then fails at its
    first HIP call, with another code)."""
    L, lib = _lib()
    h = C.c_void_p()
    rc = lib.grmhd_init_grid(C.byref(_desc(L, ng=ng, deriv_order=order, recon=recon)), None, C.byref(h))
    if rc == L.OK:
        lib.grmhd_destroy(h)
    else:
        assert rc != L.EINVAL, lib.grmhd_last_error().decode()
