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
LEARNED_BEST, LEARNED_ONLY = 0, 1
RECON_MP5, RECON_WENO5, RECON_PLM, RECON_MP7 = 0, 1, 2, 3
RECON = {"mp5": RECON_MP5, "weno5": RECON_WENO5, "plm": RECON_PLM, "mp7": RECON_MP7}
METRIC_MINKOWSKI, METRIC_TABLE_AXISYM = 0, 1
METRIC_NCOMP = 88

EXPORTS = ("grmhd_init_grid", "grmhd_get_layout", "grmhd_bind_fields", "grmhd_set_metric",
           "grmhd_curl_potential", "grmhd_prim2cons", "grmhd_rhs", "grmhd_rk_step",
           "grmhd_cons2prim", "grmhd_compute_dt", "grmhd_diagnostics", "grmhd_shell_fluxes", "grmhd_destroy",
           "grmhd_last_error", "grmhd_set_profiling", "grmhd_get_profile",
           "grmhd_profile_class_name", "grmhd_mlp_set_weights", "grmhd_mlp_get_weights",
           "grmhd_mlp_datagen", "grmhd_mlp_gradient", "grmhd_mlp_train_step", "grmhd_mlp_forward",
           "grmhd_cons2prim_points", "grmhd_set_newton_split", "grmhd_mri_quality",
           "grmhd_rk_steps_graph", "grmhd_reset_run_counters", "grmhd_compute_dt_noalloc",
           "grmhd_set_learned_guess")
MLP_NPARAM = 10448
MLP_NNORM = 32
PROF_NCLASS = 17


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("ng", C.c_int32), ("coord", C.c_int32),
                ("bc", C.c_int32 * 6), ("precision", C.c_int32), ("c2p_guess", C.c_int32),
                ("newton_maxit", C.c_int32), ("recon", C.c_int32),
                ("x0", C.c_double * 3), ("dx", C.c_double * 3), ("gamma_ad", C.c_double),
                ("cfl", C.c_double), ("rho_fl_a", C.c_double), ("rho_fl_n", C.c_double),
                ("p_fl_a", C.c_double), ("p_fl_n", C.c_double), ("w_max", C.c_double),
                ("newton_tol", C.c_double), ("deriv_order", C.c_int32), ("fallback", C.c_int32)]


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
                ("n_nonfinite", C.c_int64), ("n_mlp_chosen", C.c_int64),
                ("run_c2p_fail", C.c_int64), ("run_floor_rho", C.c_int64),
                ("run_floor_p", C.c_int64), ("run_wcap", C.c_int64),
                ("run_mlp_deferred", C.c_int64), ("run_mlp_chosen", C.c_int64),
                ("run_mlp_fallback", C.c_int64), ("run_troubled", C.c_int64)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "sum_cons" else v
        return out


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * PROF_NCLASS), ("launches", C.c_int64 * PROF_NCLASS)]


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
    L.grmhd_compute_dt_noalloc.argtypes = [P, P]
    L.grmhd_diagnostics.argtypes = [P, C.POINTER(Diag)]
    L.grmhd_reset_run_counters.argtypes = [P]
    L.grmhd_shell_fluxes.argtypes = [P, C.POINTER(C.c_double), C.c_size_t]
    L.grmhd_destroy.argtypes = [P]
    L.grmhd_destroy.restype = None
    L.grmhd_last_error.restype = C.c_char_p
    L.grmhd_set_profiling.argtypes = [P, C.c_int]
    L.grmhd_set_newton_split.argtypes = [P, C.c_int32]
    L.grmhd_set_learned_guess.argtypes = [P, C.c_double, C.c_int]
    L.grmhd_rk_steps_graph.argtypes = [P, C.c_int32]
    L.grmhd_mri_quality.argtypes = [P, C.c_double, C.c_double, C.POINTER(C.c_double), C.c_size_t]
    L.grmhd_get_profile.argtypes = [P, C.POINTER(Profile), C.c_int]
    L.grmhd_profile_class_name.argtypes = [C.c_int]
    L.grmhd_profile_class_name.restype = C.c_char_p
    F = C.POINTER(C.c_float)
    L.grmhd_mlp_set_weights.argtypes = [P, F, C.c_size_t, F, C.c_size_t]
    L.grmhd_mlp_get_weights.argtypes = [P, F, F]
    L.grmhd_mlp_datagen.argtypes = [P, P, C.c_int64, P, P, P, C.c_int]
    L.grmhd_cons2prim_points.argtypes = [P, P, C.c_int64, P, P, P]
    L.grmhd_mlp_gradient.argtypes = [P, P, P, C.c_int64, F, D]
    L.grmhd_mlp_train_step.argtypes = [P, P, P, C.c_int64, C.c_float, D]
    L.grmhd_mlp_forward.argtypes = [P, P, C.c_int64, P]
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


def make_desc(grid, precision=FP64, guess=GUESS_WARM, recon=RECON_MP5, deriv_order=6, fallback=False):
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
    d.recon = recon
    d.gamma_ad = grid.gamma_ad
    d.cfl = grid.cfl
    d.rho_fl_a, d.rho_fl_n = grid.rho_fl_a, grid.rho_fl_n
    d.p_fl_a, d.p_fl_n = grid.p_fl_a, grid.p_fl_n
    d.w_max = grid.w_max
    d.newton_tol = grid.newton_tol
    d.deriv_order = deriv_order
    d.fallback = 1 if fallback else 0
    return d


# ----------------------------------------------------------------- learned guess layout
MLP_SHAPES = (((64, 16), 0), ((64,), 1024), ((64, 64), 1088), ((64,), 5184),
              ((64, 64), 5248), ((64,), 9344), ((16, 64), 9408), ((16,), 10432))


def mlp_pack(params):
    """[(W (out, in), b (out))] x 4 (widths 8-64-64-64-5) -> padded flat float32."""
    import numpy as np
    flat = np.zeros(MLP_NPARAM, dtype=np.float32)
    for li, (w, b) in enumerate(params):
        (ws, wo), (bs, bo) = MLP_SHAPES[2 * li], MLP_SHAPES[2 * li + 1]
        m = np.zeros(ws, dtype=np.float32)
        m[:w.shape[0], :w.shape[1]] = w
        flat[wo:wo + m.size] = m.ravel()
        v = np.zeros(bs, dtype=np.float32)
        v[:b.shape[0]] = b
        flat[bo:bo + v.size] = v
    return flat


def mlp_unpack(flat):
    import numpy as np
    widths = (8, 64, 64, 64, 5)
    out = []
    for li in range(4):
        (ws, wo), (bs, bo) = MLP_SHAPES[2 * li], MLP_SHAPES[2 * li + 1]
        m = np.asarray(flat[wo:wo + ws[0] * ws[1]], dtype=np.float64).reshape(ws)
        v = np.asarray(flat[bo:bo + bs[0]], dtype=np.float64)
        out.append((m[:widths[li + 1], :widths[li]].copy(), v[:widths[li + 1]].copy()))
    return out


def mlp_norm_pack(fmean, fstd, tmean, tstd):
    import numpy as np
    n = np.zeros(MLP_NNORM, dtype=np.float32)
    n[0:8], n[8:16] = fmean, fstd
    n[16:16 + len(tmean)], n[24:24 + len(tstd)] = tmean, tstd
    n[16 + len(tmean):24] = 0.0
    n[24 + len(tstd):32] = 1.0
    return n
