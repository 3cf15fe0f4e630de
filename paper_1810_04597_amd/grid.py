"""Grid: device memory (torch tensors) + the C-ABI calls, argument marshalling only."""
import ctypes as C
import numpy as np
import torch

from . import _lib as L

PRIM = ("rho", "u1", "u2", "u3", "p", "B1", "B2", "B3")
CONS = ("D", "S1", "S2", "S3", "tau", "Bf1", "Bf2", "Bf3")


class Grid:
    def __init__(self, spec, tables=None, precision=L.FP64, guess=L.GUESS_WARM,
                 device="cuda:0", stream=None, recon=L.RECON_MP5, deriv_order=6, fallback=False):
        """recon: reconstruction code (L.RECON_MP5, _WENO5, _PLM, _MP7) or its
        name; deriv_order: 6 or 4 (staggered derivative and interpolation);
        fallback: first-order HLL fluxes at the faces of zones whose new state
        is unphysical (diagnostics run_troubled counts those zones)."""
        if isinstance(recon, str):
            recon = L.RECON[recon]
        if not torch.cuda.is_available():
            raise RuntimeError("Grid needs a HIP device")
        self.lib = L.lib()
        self.spec = spec
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.desc = L.make_desc(spec, precision, guess, recon, deriv_order, fallback)
        h = C.c_void_p()
        self._call(self.lib.grmhd_init_grid, C.byref(self.desc), C.c_void_p(self.stream.cuda_stream),
                                         C.byref(h))
        self.h = h
        lay = L.Layout()
        self._call(self.lib.grmhd_get_layout, self.h, C.byref(lay))
        self.layout = lay
        f64 = dict(dtype=torch.float64, device=self.device)
        self.prim = torch.zeros(int(lay.prim_doubles), **f64)
        self.cons = torch.zeros(int(lay.cons_doubles), **f64)
        self.scratch = torch.zeros(int(lay.scratch_bytes) // 8, **f64)
        self._call(self.lib.grmhd_bind_fields, self.h, C.c_void_p(self.prim.data_ptr()),
                                           C.c_void_p(self.cons.data_ptr()),
                                           C.c_void_p(self.scratch.data_ptr()),
                                           C.c_size_t(int(lay.scratch_bytes)))
        if tables is None:
            self._call(self.lib.grmhd_set_metric, self.h, L.METRIC_MINKOWSKI, None, 0)
        else:
            self.set_metric(tables)

    def _call(self, fn, *args):
        """One library call on the grid's stream.  When that is not torch's
        current stream, the grid stream first waits for torch's pending work
        (uploads, allocations) and torch's stream then waits for the call
        (results read through torch)."""
        cur = torch.cuda.current_stream(self.device)
        other = cur != self.stream
        if other:
            self.stream.wait_stream(cur)
        rc = L.check(fn(*args))
        if other:
            cur.wait_stream(self.stream)
        return rc

    # ------------------------------------------------------------ layout views
    def field_view(self, flat, f):
        """[k][j][i] ghosted view of field f of a group tensor (padding dropped)."""
        lay = self.layout
        d0, d1, d2 = (int(x) for x in lay.dims)
        base = f * int(lay.field)
        return flat.as_strided((d2, d1, d0), (int(lay.plane), int(lay.pitch), 1), base)

    def new_single(self):
        return torch.zeros(int(self.layout.edge_doubles), dtype=torch.float64, device=self.device)

    def _interior(self, v):
        g = self.spec.ng
        return v[g:-g, g:-g, g:-g]

    # ------------------------------------------------------------ API calls
    def set_metric(self, tables):
        t = np.ascontiguousarray(tables, dtype=np.float64)
        self._call(self.lib.grmhd_set_metric, self.h, L.METRIC_TABLE_AXISYM,
                                          t.ctypes.data_as(C.POINTER(C.c_double)), t.size)

    def set_primitives(self, data):
        """Interior rho, u, p (numpy [k][j][i]) -> prim; then prim2cons."""
        for f, name in enumerate(PRIM[:5]):
            v = self._interior(self.field_view(self.prim, f))
            v.copy_(torch.from_numpy(np.ascontiguousarray(data[name], dtype=np.float64)))
        self.prim2cons()

    def set_face_fields(self, data):
        """Ghosted face fields B1f..B3f (numpy, ghosted shape) -> cons."""
        for a in range(3):
            v = self.field_view(self.cons, 5 + a)
            v.copy_(torch.from_numpy(np.ascontiguousarray(data["B%df" % (a + 1)], dtype=np.float64)))

    def curl_potential(self, data):
        arrs = []
        for a in range(3):
            t = self.new_single()
            self.field_view(t, 0).copy_(torch.from_numpy(np.ascontiguousarray(data["A%d" % (a + 1)], dtype=np.float64)))
            arrs.append(t)
        self._call(self.lib.grmhd_curl_potential, self.h, *[C.c_void_p(t.data_ptr()) for t in arrs])
        self.synchronize()

    def prim2cons(self):
        self._call(self.lib.grmhd_prim2cons, self.h)

    def rhs(self):
        out = torch.zeros_like(self.cons)
        self._call(self.lib.grmhd_rhs, self.h, C.c_void_p(out.data_ptr()))
        return out

    def rk_step(self, dt=0.0, want_dt=False):
        v = C.c_double(0.0)
        self._call(self.lib.grmhd_rk_step, self.h, C.c_double(dt), C.byref(v) if want_dt else None)
        return v.value if want_dt else None

    def cons2prim(self, strict=False):
        n = C.c_int64(0)
        self._call(self.lib.grmhd_cons2prim, self.h, C.byref(n), 1 if strict else 0)
        return n.value

    def compute_dt(self):
        v = C.c_double(0.0)
        self._call(self.lib.grmhd_compute_dt, self.h, C.byref(v))
        return v.value

    def compute_dt_noalloc(self, out):
        """CFL step into out (device float64 tensor, >= 1 element), without
        synchronising or allocating."""
        self._call(self.lib.grmhd_compute_dt_noalloc, self.h, C.c_void_p(out.data_ptr()))

    def diagnostics(self):
        d = L.Diag()
        self._call(self.lib.grmhd_diagnostics, self.h, C.byref(d))
        return d.as_dict()

    def reset_run_counters(self):
        """Zero the inversion counters accumulated over every inversion (diag run_*)."""
        self._call(self.lib.grmhd_reset_run_counters, self.h)

    def shell_fluxes(self):
        """{F_D, F_tau, Phi, Phi_s}: fluxes through the x^1 = const shells (numpy, n1 each)."""
        n1 = self.spec.n[0]
        buf = (C.c_double * (4 * n1))()
        self._call(self.lib.grmhd_shell_fluxes, self.h, buf, C.c_size_t(4 * n1))
        a = np.frombuffer(buf, dtype=np.float64).copy()
        return {"F_D": a[0:n1], "F_tau": a[n1:2 * n1], "Phi": a[2 * n1:3 * n1], "Phi_s": a[3 * n1:]}

    def mri_quality(self, rho_cut, q_min=8.0):
        """MRI resolution sums per x^1 shell over the zones with rho > rho_cut
        (numpy, n1 each): wQ2, wQ3, w (w = rho sqrt(gamma)), n_body, n_Q2_ok,
        n_Q3_ok; plus the body's weighted means Q2_mean, Q3_mean and the
        fractions of body zones with Q >= q_min."""
        n1 = self.spec.n[0]
        buf = (C.c_double * (6 * n1))()
        self._call(self.lib.grmhd_mri_quality, self.h, float(rho_cut), float(q_min), buf, C.c_size_t(6 * n1))
        a = np.frombuffer(buf, dtype=np.float64).copy().reshape(6, n1)
        out = dict(zip(("wQ2", "wQ3", "w", "n_body", "n_Q2_ok", "n_Q3_ok"), a))
        w, nb = a[2].sum(), a[3].sum()
        out.update(Q2_mean=a[0].sum() / w if w > 0 else float("nan"),
                   Q3_mean=a[1].sum() / w if w > 0 else float("nan"),
                   frac_Q2_ok=a[4].sum() / nb if nb > 0 else float("nan"),
                   frac_Q3_ok=a[5].sum() / nb if nb > 0 else float("nan"))
        return out

    # ------------------------------------------------------------ learned guess
    def mlp_set_weights(self, flat, norm):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        Fp = C.POINTER(C.c_float)
        self._call(self.lib.grmhd_mlp_set_weights, self.h, flat.ctypes.data_as(Fp), flat.size,
                                               norm.ctypes.data_as(Fp), norm.size)

    def mlp_get_weights(self):
        flat = np.zeros(L.MLP_NPARAM, dtype=np.float32)
        norm = np.zeros(L.MLP_NNORM, dtype=np.float32)
        Fp = C.POINTER(C.c_float)
        self._call(self.lib.grmhd_mlp_get_weights, self.h, flat.ctypes.data_as(Fp), norm.ctypes.data_as(Fp))
        return flat, norm

    def mlp_datagen(self, prims, set_norm=False, want_cons=False):
        """prims: (n, 8) float64 array (host or device) -> (features, targets)
        device float32 tensors (n, 8) [, cons (n, 8) float64]."""
        pr = torch.as_tensor(np.ascontiguousarray(prims, dtype=np.float64) if isinstance(prims, np.ndarray) else prims,
                             dtype=torch.float64).to(self.device).contiguous()
        n = pr.shape[0]
        feat = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        targ = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        cons = torch.empty((n, 8), dtype=torch.float64, device=self.device) if want_cons else None
        self._call(self.lib.grmhd_mlp_datagen, self.h, C.c_void_p(pr.data_ptr()), n,
                                           C.c_void_p(feat.data_ptr()), C.c_void_p(targ.data_ptr()),
                                           C.c_void_p(cons.data_ptr()) if want_cons else None,
                                           1 if set_norm else 0)
        self.synchronize()
        return (feat, targ, cons) if want_cons else (feat, targ)

    def cons2prim_points(self, cons, y0=None):
        """Batched point-wise inversion (flat frame): cons (n, 8) device float64;
        y0 (n,) device float64 or None (cold start).  -> (prims (n, 8), iterations)."""
        n = cons.shape[0]
        prim = torch.empty((n, 8), dtype=torch.float64, device=self.device)
        it = torch.empty((n,), dtype=torch.int32, device=self.device)
        self._call(self.lib.grmhd_cons2prim_points, self.h, C.c_void_p(cons.data_ptr()), n,
                                                C.c_void_p(y0.data_ptr()) if y0 is not None else None,
                                                C.c_void_p(prim.data_ptr()), C.c_void_p(it.data_ptr()))
        self.synchronize()
        return prim, it

    def mlp_gradient(self, feat, targ):
        g = np.zeros(L.MLP_NPARAM, dtype=np.float32)
        loss = C.c_double(0.0)
        self._call(self.lib.grmhd_mlp_gradient, self.h, C.c_void_p(feat.data_ptr()), C.c_void_p(targ.data_ptr()),
                                            feat.shape[0], g.ctypes.data_as(C.POINTER(C.c_float)),
                                            C.byref(loss))
        return g, loss.value

    def mlp_train_step(self, feat, targ, lr, want_loss=False):
        loss = C.c_double(0.0)
        self._call(self.lib.grmhd_mlp_train_step, self.h, C.c_void_p(feat.data_ptr()), C.c_void_p(targ.data_ptr()),
                                              feat.shape[0], C.c_float(lr),
                                              C.byref(loss) if want_loss else None)
        return loss.value if want_loss else None

    def mlp_forward(self, feat):
        out = torch.empty((feat.shape[0], 8), dtype=torch.float32, device=self.device)
        self._call(self.lib.grmhd_mlp_forward, self.h, C.c_void_p(feat.data_ptr()), feat.shape[0],
                                           C.c_void_p(out.data_ptr()))
        self.synchronize()
        return out

    def rk_steps_graph(self, nsteps):
        """nsteps device-dt RK3 steps replayed from a captured HIP graph of
        one step (the grid needs its own stream: Grid(..., stream=...))."""
        self._call(self.lib.grmhd_rk_steps_graph, self.h, int(nsteps))

    def set_newton_split(self, iters):
        """Split inversion: at most iters Newton iterations in the first pass,
        the rest of the slow zones in a second, compact pass (0: off)."""
        self._call(self.lib.grmhd_set_newton_split, self.h, int(iters))

    def set_learned_guess(self, defer_tol=1e-2, start=L.LEARNED_BEST):
        """Learned-guess pass policy: defer_tol (0: every zone) and start
        (L.LEARNED_BEST or L.LEARNED_ONLY)."""
        self._call(self.lib.grmhd_set_learned_guess, self.h, float(defer_tol), int(start))

    def set_profiling(self, on=True):
        self._call(self.lib.grmhd_set_profiling, self.h, 1 if on else 0)

    def profile(self, reset=True):
        """{kernel class: (total ms, launches)} since the last reset."""
        p = L.Profile()
        self._call(self.lib.grmhd_get_profile, self.h, C.byref(p), 1 if reset else 0)
        out = {}
        for c in range(L.PROF_NCLASS):
            if p.launches[c]:
                out[self.lib.grmhd_profile_class_name(c).decode()] = (p.ms[c], int(p.launches[c]))
        return out

    def synchronize(self):
        self.stream.synchronize()

    # ------------------------------------------------------------ readback
    def read_group(self, flat, names, interior=False):
        self.synchronize()
        out = {}
        for f, name in enumerate(names):
            v = self.field_view(flat, f)
            if interior:
                v = self._interior(v)
            out[name] = v.cpu().numpy().copy()
        return out

    def to_numpy(self, which="prim", interior=False):
        self.synchronize()
        flat = self.prim if which == "prim" else self.cons
        names = PRIM if which == "prim" else CONS
        out = {}
        for f, name in enumerate(names):
            v = self.field_view(flat, f)
            if interior:
                v = self._interior(v)
            out[name] = v.cpu().numpy().copy()
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.grmhd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
