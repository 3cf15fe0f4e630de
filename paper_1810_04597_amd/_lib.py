"""ctypes mirror of include/grmhd.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrmhd.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
CART, LOGSPH = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_AXIS = 0, 1, 2
FP64, FP32_FLUX = 0, 1
GUESS_WARM, GUESS_COLD, GUESS_MLP = 0, 1, 2
METRIC_MINKOWSKI, METRIC_TABLE_AXISYM = 0, 1
METRIC_NCOMP = 88

EXPORTS = ("grmhd_init_grid", "grmhd_get_layout", "grmhd_bind_fields", "grmhd_set_metric",
           "grmhd_curl_potential", "grmhd_prim2cons", "grmhd_rhs", "grmhd_rk_step",
           "grmhd_cons2prim", "grmhd_compute_dt", "grmhd_diagnostics", "grmhd_destroy",
           "grmhd_last_error", "grmhd_set_profiling", "grmhd_get_profile",
           "grmhd_profile_class_name")
PROF_NCLASS = 16


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("ng", C.c_int32), ("coord", C.c_int32),
                ("bc", C.c_int32 * 6), ("precision", C.c_int32), ("c2p_guess", C.c_int32),
                ("newton_maxit", C.c_int32), ("reserved", C.c_int32),
                ("x0", C.c_double * 3), ("dx", C.c_double * 3), ("gamma_ad", C.c_double),
                ("cfl", C.c_double), ("rho_fl_a", C.c_double), ("rho_fl_n", C.c_double),
                ("p_fl_a", C.c_double), ("p_fl_n", C.c_double), ("w_max", C.c_double),
                ("newton_tol", C.c_double)]


class Layout(C.Structure):
    _fields_ = [("dims", C.c_int64 * 3), ("pitch", C.c_int64), ("plane", C.c_int64),
                ("field", C.c_int64), ("offset", C.c_int64), ("prim_doubles", C.c_int64),
                ("cons_doubles", C.c_int64), ("edge_doubles", C.c_int64),
                ("scratch_bytes", C.c_int64)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("dt", C.c_double),
                ("sum_cons", C.c_double * 8), ("max_divb", C.c_double),
                ("max_divb_norm", C.c_double), ("rho_min", C.c_double), ("rho_max", C.c_double),
                ("p_min", C.c_double), ("p_max", C.c_double), ("w_max", C.c_double),
                ("n_floor_rho", C.c_int64), ("n_floor_p", C.c_int64), ("n_wcap", C.c_int64),
                ("n_c2p_fail", C.c_int64), ("n_mlp_fallback", C.c_int64),
                ("newton_iters_sum", C.c_int64), ("newton_iters_max", C.c_int64),
                ("n_nonfinite", C.c_int64)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "sum_cons" else v
        return out


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 16), ("launches", C.c_int64 * 16)]


class GrmhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("grmhd error %d: %s" % (code, msg))
        self.code = code


_LIB = None


def lib():
    """Load libgrmhd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgrmhd.so not built: run paper_1810_04597_amd/build.py "
                           "(the HIP library is required; there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    L.grmhd_init_grid.argtypes = [C.POINTER(GridDesc), P, C.POINTER(P)]
    L.grmhd_get_layout.argtypes = [P, C.POINTER(Layout)]
    L.grmhd_bind_fields.argtypes = [P, P, P, P, C.c_size_t]
    L.grmhd_set_metric.argtypes = [P, C.c_int, D, C.c_size_t]
    L.grmhd_curl_potential.argtypes = [P, P, P, P]
    L.grmhd_prim2cons.argtypes = [P]
    L.grmhd_rhs.argtypes = [P, P]
    L.grmhd_rk_step.argtypes = [P, C.c_double, D]
    L.grmhd_cons2prim.argtypes = [P, C.POINTER(C.c_int64), C.c_int]
    L.grmhd_compute_dt.argtypes = [P, D]
    L.grmhd_diagnostics.argtypes = [P, C.POINTER(Diag)]
    L.grmhd_destroy.argtypes = [P]
    L.grmhd_destroy.restype = None
    L.grmhd_last_error.restype = C.c_char_p
    L.grmhd_set_profiling.argtypes = [P, C.c_int]
    L.grmhd_get_profile.argtypes = [P, C.POINTER(Profile), C.c_int]
    L.grmhd_profile_class_name.argtypes = [C.c_int]
    L.grmhd_profile_class_name.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("grmhd_destroy", "grmhd_last_error", "grmhd_profile_class_name"):
            getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def check(rc):
    if rc != OK:
        msg = lib().grmhd_last_error().decode()
        raise GrmhdError(rc, msg)
    return rc


def make_desc(grid, precision=FP64, guess=GUESS_WARM):
    """GridDesc from a workloads.GridSpec-like object."""
    d = GridDesc()
    for a in range(3):
        d.n[a] = grid.n[a]
        d.x0[a] = grid.x0[a]
        d.dx[a] = grid.dx[a]
    d.ng = grid.ng
    d.coord = grid.coord
    for s in range(6):
        d.bc[s] = grid.bc[s]
    d.precision = precision
    d.c2p_guess = guess
    d.newton_maxit = grid.newton_maxit
    d.reserved = 0
    d.gamma_ad = grid.gamma_ad
    d.cfl = grid.cfl
    d.rho_fl_a, d.rho_fl_n = grid.rho_fl_a, grid.rho_fl_n
    d.p_fl_a, d.p_fl_n = grid.p_fl_a, grid.p_fl_n
    d.w_max = grid.w_max
    d.newton_tol = grid.newton_tol
    return d
