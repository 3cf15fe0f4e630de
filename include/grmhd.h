/*
 * grmhd.h -- C ABI of the MI355X GRMHD right-hand-side and time-update library.
 *
 * The library advances the 3+1 general-relativistic MHD equations on one
 * block of a 3-D finite-difference grid, the method the paper states in its
 * Introduction (3-D finite differences, high-order reconstruction, after the
 * ECHO scheme): MP5 reconstruction (WENO5, PLM-MC and MP7 selectable), HLL
 * fluxes, a sixth-order (or fourth-order) staggered finite-difference flux
 * derivative with metric source terms, an upwind constrained-transport edge
 * field (div B constant to round-off), SSP-RK3 stages with an optional
 * lower-order fallback at zones the high-order update leaves unphysical, and
 * a per-zone Newton conservative-to-primitive inversion.  The
 * paper's multi-node domain decomposition reduces here to one block whose
 * ghost zones are filled on the device.
 *
 * Conventions
 *  - Memory: field arrays are caller-owned device memory (for instance torch
 *    tensors).  The library keeps non-owning pointers from grmhd_bind_fields
 *    until grmhd_destroy or the next bind; the caller keeps them alive and
 *    unmoved.  The library owns only metric tables, reduction buffers, the
 *    device time step and learned-guess weights, and frees them in
 *    grmhd_destroy.
 *  - Layout (grmhd_get_layout): structure of arrays, field-major, x^1 fastest,
 *    ghost zones included.  Element (i, j, k) of field f, with interior
 *    indices starting at 0 and ghosts at -ng, sits at
 *        base + f * field + offset + k * plane + j * pitch + i.
 *    The face "i + 1/2" of a face-centred field is stored at index i; the edge
 *    (i + 1/2, j + 1/2, k) at [k][j][i] (cyclically for the other families).
 *  - Field groups: prim = 8 fields (rho, u^1, u^2, u^3, p, B^1, B^2, B^3;
 *    u^i = W v^i contravariant, B undensitised, at cell centres);
 *    cons = 8 fields (sqrt(gamma) D, sqrt(gamma) S_1..3, sqrt(gamma) tau at
 *    centres; sqrt(gamma) B^1, B^2, B^3 on the x^1, x^2, x^3 faces).
 *  - Face fields at non-periodic boundaries: the field normal to an outflow
 *    or polar-axis boundary is state (not filled from the owned faces) at
 *    the ghost faces the staggered derivative of an interior cell reads,
 *    stored -3 .. -1 and n .. n+1 (-2 .. -1 and n with deriv_order 4), the
 *    polar axis faces among them: the step evolves them with the induction
 *    equation like the owned faces, so the discrete div B of the cells
 *    beside the boundary keeps its value; grmhd_curl_potential sets them, a
 *    caller binding its own face fields supplies them.  The edge field on a
 *    polar axis is 0.  Every other ghost is filled by the boundary rule.
 *  - Streams: every call enqueues work on the stream given at init (a
 *    hipStream_t, 0 = null stream) and returns at once.  Only calls with a
 *    host out-pointer (dt_used, n_fail, diagnostics, loss) synchronise it.
 *  - Errors: negative return codes, never exceptions or aborts across the
 *    ABI.  Arguments are checked before any launch; grmhd_last_error() gives
 *    the message of the last failing call of the calling thread.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct grmhd_grid grmhd_grid;

enum {
  GRMHD_OK = 0,
  GRMHD_EINVAL = -1,       /* bad argument, detected before any launch      */
  GRMHD_ENOMEM = -2,       /* device allocation of library-owned memory     */
  GRMHD_EHIP = -3,         /* HIP runtime error (message says which)        */
  GRMHD_ESTATE = -4,       /* call order: fields or metric not set          */
  GRMHD_ENOCONV = -5,      /* strict inversion requested and a zone failed  */
  GRMHD_EUNSUPPORTED = -6  /* valid request the library does not provide     */
};

enum { GRMHD_CART = 0, GRMHD_LOGSPH = 1 };          /* (x,y,z) | (ln r, theta, phi) */
enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1, GRMHD_BC_AXIS = 2 };
enum { GRMHD_FP64 = 0, GRMHD_FP32_FLUX = 1 };
enum { GRMHD_GUESS_WARM = 0, GRMHD_GUESS_COLD = 1, GRMHD_GUESS_MLP = 2 };
/* Interface reconstruction (paper, Introduction: high-order reconstruction
 * algorithms), applied to point values at cell centres on the six cells
 * f-2 .. f+3 around face f+1/2: MP5 (Suresh & Huynh 1997, point-value
 * interpolant, zero limiter tolerance; the default), WENO5 (Jiang & Shu 1996
 * indicators, point-value form, eps = 1e-6), PLM with the monotonized-central
 * limiter (second order, the lower-order member); MP7 (the same limiter on
 * the degree-6 interpolant of the seven cells f-3 .. f+3, seventh order;
 * eight-cell stencils f-3 .. f+4, so it needs ng = 6, or 5 with
 * deriv_order 4). */
enum { GRMHD_RECON_MP5 = 0, GRMHD_RECON_WENO5 = 1, GRMHD_RECON_PLM = 2, GRMHD_RECON_MP7 = 3 };
enum { GRMHD_METRIC_MINKOWSKI = 0, GRMHD_METRIC_TABLE_AXISYM = 1 };

/* Number of float64 components of an axisymmetric metric table per (j, i):
 * four location families (centre, x^1 face, x^2 face, x^3 edge) x 17
 * components (alpha, beta^1..3, gamma_11,12,13,22,23,33,
 * gamma^11,12,13,22,23,33, sqrt(gamma)), then 20 centre derivatives
 * (d1 alpha, d2 alpha, d1 beta^1..3, d2 beta^1..3, d1 gamma_ij (6),
 * d2 gamma_ij (6)).  Table array: [comp][j][i], j in [-ng, n2+ng),
 * i in [-ng, n1+ng), the same for every x^3 index. */
#define GRMHD_METRIC_NCOMP 88

typedef struct {
  int32_t n[3];            /* interior zones n1, n2, n3 (each >= 1)              */
  int32_t ng;              /* ghost layers: 5 (MP5/WENO5/PLM + 6th-order D), 6
                              (required by MP7 with the 6th-order D; allowed for
                              the others) or 4 (MP5/WENO5/PLM + 4th-order D:
                              faces and edges are formed at -2 .. n instead of
                              -3 .. n+1)                                      */
  int32_t coord;           /* GRMHD_CART | GRMHD_LOGSPH (floors use r = e^{x^1}) */
  int32_t bc[6];           /* -x1,+x1,-x2,+x2,-x3,+x3; periodic in pairs; axis
                              only on x^2 (n2 >= ng+1) with periodic x^3, n3 even */
  int32_t precision;       /* GRMHD_FP64 | GRMHD_FP32_FLUX                       */
  int32_t c2p_guess;       /* GRMHD_GUESS_WARM | _COLD | _MLP                     */
  int32_t newton_maxit;    /* e.g. 50                                             */
  int32_t recon;           /* GRMHD_RECON_MP5 (0) | _WENO5 | _PLM | _MP7          */
  double x0[3];            /* lower interior edge in code coordinates            */
  double dx[3];            /* uniform spacing (> 0)                              */
  double gamma_ad;         /* ideal-gas index (> 1)                              */
  double cfl;              /* Courant number for the device time step (> 0)      */
  double rho_fl_a, rho_fl_n;  /* rho floor a r^n (a = 0: off)                     */
  double p_fl_a, p_fl_n;      /* p floor a r^n (a = 0: off)                       */
  double w_max;            /* Lorentz-factor cap (0: off, else > 1)              */
  double newton_tol;       /* relative step tolerance, e.g. 1e-14                */
  int32_t deriv_order;     /* staggered derivative / interpolation order: 0 or 6
                              (sixth, the default) or 4 (fourth, the first
                              correction only); one order serves the flux
                              derivative, the induction equation, the curl of
                              the vector potential, the centred field and div B */
  int32_t fallback;        /* 0: off; 1: lower-order fallback at troubled zones. A
                              zone whose new hydro state after a stage's update is
                              unphysical (D <= 0, tau <= 0 or S^2 >= (tau + D)^2)
                              is troubled; at each face of a troubled zone the
                              stage replaces the high-order flux (the face flux G
                              = f - Delta^2 f/24 + 3 Delta^4 f/640 whose difference
                              is the staggered derivative; its first correction
                              alone at deriv_order 4) by the first-order HLL flux
                              of the two cells, in both zones beside the face
                              (conservative).  Off: the step is unchanged bit for
                              bit.  On: the update runs as two launches around the
                              fix (two launches that exit at once when no zone is
                              troubled); library-owned: a flag byte and a list
                              entry (int32) per zone                              */
} grmhd_grid_desc;

typedef struct {
  int64_t dims[3];         /* ghosted extents n_d + 2 ng                         */
  int64_t pitch;           /* elements between x^2 rows (>= dims[0], padded)     */
  int64_t plane;           /* elements between x^3 planes                        */
  int64_t field;           /* elements between fields of a group                 */
  int64_t offset;          /* element offset of interior (0,0,0) in a field      */
  int64_t prim_doubles;    /* size of the prim group  (8 fields)                 */
  int64_t cons_doubles;    /* size of the cons group  (8 fields)                 */
  int64_t edge_doubles;    /* size of one single-field array (potentials)        */
  int64_t scratch_bytes;   /* scratch required by grmhd_bind_fields              */
} grmhd_layout;

typedef struct {
  int64_t step;
  double t, dt;
  double sum_cons[8];      /* plain sums over interior cells / owned faces       */
  double max_divb;         /* max over interior cells of |sum_d D_d B^d|         */
  double max_divb_norm;    /* max_divb * min(dx) / max|B centred|                */
  double rho_min, rho_max, p_min, p_max, w_max;
  int64_t n_floor_rho, n_floor_p, n_wcap;   /* last inversion                     */
  int64_t n_c2p_fail, n_mlp_fallback;        /* last inversion                     */
  int64_t newton_iters_sum, newton_iters_max;/* last inversion                     */
  int64_t n_nonfinite;     /* interior primitives that are not finite            */
  int64_t n_mlp_chosen;    /* last inversion: zones that started from the learned guess */
  /* Accumulated over every inversion (each RK stage, cons2prim, the learned
   * and split passes) since grmhd_init_grid or grmhd_reset_run_counters: */
  int64_t run_c2p_fail;    /* zones whose Newton inversion failed                */
  int64_t run_floor_rho, run_floor_p, run_wcap;  /* floor and W-cap activations  */
  int64_t run_mlp_deferred;  /* zones inverted in the learned-guess pass        */
  int64_t run_mlp_chosen;    /* zones that started from the network's guess     */
  int64_t run_mlp_fallback;  /* learned starts rerun from the warm guess         */
  int64_t run_troubled;    /* zones taken by the lower-order fallback (summed over
                              the stages; 0 unless grmhd_grid_desc.fallback)   */
} grmhd_diag;

/* Create a grid.  desc is copied.  hip_stream: hipStream_t or NULL.
 * Errors: EINVAL (descriptor), ENOMEM/EHIP (device buffers). */
int grmhd_init_grid(const grmhd_grid_desc* desc, void* hip_stream, grmhd_grid** out);

/* Memory layout the caller must allocate with (pure host call). */
int grmhd_get_layout(const grmhd_grid* h, grmhd_layout* out);

/* Bind caller-owned device memory: prim (layout.prim_doubles float64),
 * cons (layout.cons_doubles), scratch (>= layout.scratch_bytes, 256-byte
 * aligned).  EINVAL on NULL, misalignment or a short scratch. */
int grmhd_bind_fields(grmhd_grid* h, double* prim, double* cons, void* scratch,
                      size_t scratch_bytes);

/* Background metric.  kind = GRMHD_METRIC_MINKOWSKI (host_tables NULL,
 * Cartesian only) or GRMHD_METRIC_TABLE_AXISYM: host_tables holds
 * GRMHD_METRIC_NCOMP * (n2+2ng) * (n1+2ng) float64 in the layout above; the
 * library copies them to device memory it owns (synchronous copy).
 * The tables are data: the stationary 3+1 metric, see the paper's
 * Introduction (MHD in general relativity). */
int grmhd_set_metric(grmhd_grid* h, int kind, const double* host_tables, size_t n_doubles);

/* Face fields from an edge vector potential: B^n = D_{n+1} A_{n+2} - D_{n+2} A_{n+1}
 * at owned faces and at the evolved ghost faces of non-periodic boundaries,
 * then the face ghost fill.  A1, A2, A3: device arrays with
 * the single-field layout (edge_doubles each), ghosts included. */
int grmhd_curl_potential(grmhd_grid* h, const double* A1, const double* A2, const double* A3);

/* Centred B = I_d(B_face)/sqrt(gamma) and cons (D, S, tau) from the bound
 * prim (rho, u, p at interior cells) and face fields; fills ghosts of the
 * face fields first and of prim afterwards. */
int grmhd_prim2cons(grmhd_grid* h);

/* Right-hand side L(U) of the bound state: rhs_out (cons layout, 8 fields)
 * receives -sum_d D_d F_d + s at interior cells and -curl_D E at owned
 * faces; other elements are left untouched.  Uses the bound prim/cons.  The
 * lower-order fallback (grmhd_grid_desc.fallback) corrects a stage's result,
 * not L: it does not act here. */
int grmhd_rhs(grmhd_grid* h, double* rhs_out);

/* One SSP-RK3 step of the bound state.  dt > 0: that step; dt <= 0: the CFL
 * step dt = cfl / max sum_d max|lambda_d|/dx_d of the primitives at the
 * start of the step, on the device (no host sync).  A step taken with
 * dt <= 0 also reduces that value for the state it leaves (inside its last
 * inversion), and the next dt <= 0 step reuses it; grmhd_compute_dt does the
 * same.  bind_fields, set_metric, curl_potential, prim2cons and cons2prim
 * drop the stored value; a caller that writes the bound prim/cons directly
 * calls one of the latter two before stepping, as the state must be made
 * consistent anyway (they also leave the ghost zones filled: on a fully
 * periodic grid with every n >= 10 the step itself writes ghost images
 * instead of running separate ghost fills).  dt_used (nullable) receives the step taken
 * (synchronises). */
int grmhd_rk_step(grmhd_grid* h, double dt, double* dt_used);

/* Inversion of the bound cons into the bound prim at interior cells (warm,
 * cold or learned guess as configured; floors applied).  n_fail (nullable)
 * receives the number of failed zones (synchronises).  Failed zones keep
 * their previous primitives.  strict != 0 returns GRMHD_ENOCONV when a zone
 * failed (requires n_fail). */
int grmhd_cons2prim(grmhd_grid* h, int64_t* n_fail, int strict);

/* CFL time step of the bound primitives (synchronises); a following
 * rk_step with dt <= 0 takes this step. */
int grmhd_compute_dt(grmhd_grid* h, double* dt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight stepping loops, harnesses that forbid hipMalloc): the CFL
 * time step of grmhd_compute_dt, written to caller-owned device memory
 * dt_dev (one double) on the grid's stream, without synchronising and
 * without any allocation.  The per-workgroup partial maxima go to a static
 * device array of the library (4 MiB per device, kept until the process
 * ends), so the grid may hold at most 2^27 interior zones (EINVAL beyond).
 * Every call on one device shares that array: calls that overlap on one
 * device (other streams, other threads) race.  The grid's own state,
 * including the time step a following rk_step(dt <= 0) takes, is unchanged.
 * ESTATE before fields and metric are set; EHIP when the array's device
 * address could not be looked up at grmhd_init_grid. */
int grmhd_compute_dt_noalloc(grmhd_grid* h, double* dt_dev);

/* Diagnostics of the bound state (synchronises).  Sums are taken in a fixed
 * order (deterministic). */
int grmhd_diagnostics(grmhd_grid* h, grmhd_diag* out);

/* Zero the accumulated inversion counters (grmhd_diag.run_*); enqueued on
 * the grid's stream.  EINVAL on a NULL handle. */
int grmhd_reset_run_counters(grmhd_grid* h);

/* Fluxes through the surfaces x^1 = const of the bound state, for each
 * interior x^1 index i (synchronises; deterministic order).  A diagnostic of
 * the torus use case (paper, Introduction and Fig. 1: accretion onto the
 * black hole): with x^1 = ln r the densitised x^1-fluxes include sqrt(gamma)
 * and the Jacobian, so summing them times dx^2 dx^3 over a shell gives the
 * flux through the sphere.  host_out (host, n_doubles >= 4 n1) receives
 *   [0, n1)     F_D   = sum F^1[D] dx^2 dx^3 at cell centres (accretion rate -F_D)
 *   [n1, 2n1)   F_tau = sum F^1[tau] dx^2 dx^3 at cell centres
 *   [2n1, 3n1)  Phi   = 1/2 sum |B_face^1| dx^2 dx^3 at the upper x^1 face of cell i
 *   [3n1, 4n1)  sum B_face^1 dx^2 dx^3 (signed; 0 for a closed field)
 * with the pointwise fluxes of the stored primitives (including the centred
 * field).  EINVAL on NULL or a short buffer. */
int grmhd_shell_fluxes(grmhd_grid* h, double* host_out, size_t n_doubles);

/* MRI resolution of the stored state (a diagnostic of the torus runs, whose
 * turbulence the magneto-rotational instability drives; paper, Introduction
 * and Fig. 1): per zone, the number of zones per wavelength of the
 * fastest-growing MRI mode along x^2 and x^3,
 *   Q_d = 2 pi |b^d| / (|Omega| dx^d sqrt(rho h + b^2)),
 * with the field in the fluid frame b^t = W (v.B) / alpha,
 * b^i = B^i / W + b^t (alpha v^i - beta^i), b^2 = B^2 / W^2 + (v.B)^2 and the
 * angular velocity Omega = u^3 / u^t = alpha v^3 - beta^3.  Over the body
 * zones (rho > rho_cut >= 0), with the weight w = rho sqrt(gamma), host_out
 * (host, n_doubles >= 6 n1) receives per x^1 shell i:
 *   [0, n1) sum w Q_2, [n1, 2n1) sum w Q_3, [2n1, 3n1) sum w,
 *   [3n1, 4n1) body zones, [4n1, 5n1) zones with Q_2 >= q_min,
 *   [5n1, 6n1) zones with Q_3 >= q_min.
 * Sums in a fixed order (deterministic).  EINVAL on NULL, a short buffer or
 * a negative rho_cut. */
int grmhd_mri_quality(grmhd_grid* h, double rho_cut, double q_min, double* host_out, size_t n_doubles);

/* nsteps SSP-RK3 steps with the device CFL step (as grmhd_rk_step with
 * dt <= 0), replayed from a HIP graph of one step: the step's ~25 kernel
 * launches go to the device as one graph launch, which removes the gaps
 * between them.  The graph is captured on the grid's stream at the first
 * call and kept; binding fields, setting the metric, the Newton split or
 * the network weights drops it (the next call captures again).  The first
 * step after a state change (curl_potential, prim2cons, cons2prim, a step
 * with a host dt) runs eagerly, as it also reduces the CFL step.  Results
 * equal those of grmhd_rk_step bit for bit.  ESTATE while kernel timing is
 * on or on the null stream (which cannot be captured). */
int grmhd_rk_steps_graph(grmhd_grid* h, int32_t nsteps);

/* Split inversion (load balance of the Newton iteration; paper, section on
 * the OpenMP optimisation: uneven work per zone left threads idle and the
 * fix was a guided schedule).  On the GPU the cost of a wavefront is its
 * slowest zone's iteration count, so with iters > 0 every inversion first
 * runs at most iters Newton iterations per zone; zones not converged by then
 * are appended to a list with their current iterate, and a second pass of
 * compact wavefronts finishes each from that iterate (the warm guess is the
 * fallback if it fails).  The roots, floors and counters are those of the
 * one-pass inversion; grmhd_diag.newton_iters_sum counts the iterations of
 * both passes, newton_iters_max is the largest count of either pass.
 * iters = 0 (the default) turns it off.
 * EINVAL unless 0 <= iters < newton_maxit, or when iters > 0 with
 * c2p_guess = GRMHD_GUESS_MLP (whose deferral already forms a second pass).
 * Enqueued on the grid's stream; no allocation. */
int grmhd_set_newton_split(grmhd_grid* h, int32_t iters);

/* Learned Newton initial guess (a training-system pattern layered on the
 * method; the paper has no counterpart).  An MLP 8 -> 64 -> 64 -> 64 -> 5
 * (tanh hidden layers, linear output) runs on BF16 matrix cores with FP32
 * accumulation; FP32 master weights and Adam moments live in the library.
 * Inputs: [log10 D, log10(tau/D), S_hat/(tau+D), B_hat/sqrt(tau+D)] in the
 * Eulerian orthonormal frame; outputs [log10(y/U), log10(p/D), u_hat] with
 * y = rho h W^2 and U = tau + D; both standardised with the normalisation
 * block.  With c2p_guess = GRMHD_GUESS_MLP the inversion starts every zone
 * from the warm guess (the previous primitives) and defers the zones whose
 * first residual, relative to the magnitude of its terms, exceeds 1e-2 to a
 * second pass: there the network's y0 = U 10^{output 0} is a second candidate
 * start, Newton starts from the candidate with the smaller residual (counted
 * in grmhd_diag.n_mlp_chosen) and is rerun from the warm guess when a learned
 * start does not converge (counted in grmhd_diag.n_mlp_fallback).
 * Parameter block (float32, GRMHD_MLP_NPARAM): W1[64][16] (inputs padded to
 * 16 with zeros), b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
 * W4[16][64] (outputs padded to 16 with zeros), b4[16].  Normalisation block
 * (GRMHD_MLP_NNORM): feature mean[8], std[8], target mean[8], std[8].
 * Sample arrays are device float32: features n x 8, targets n x 8 (5 used),
 * outputs n x 8 (5 used, standardised). */
#define GRMHD_MLP_NPARAM 10448
/* Policy of the learned-guess pass (GRMHD_GUESS_MLP grids only):
 * defer_tol > 0: zones whose warm start leaves a first relative residual
 * above defer_tol go to the network pass (1e-2 by default); defer_tol = 0:
 * every zone goes there (the warm start is not tried first).
 * start = GRMHD_LEARNED_BEST (default): Newton starts from the warm or the
 * network's guess, whichever has the smaller residual; GRMHD_LEARNED_ONLY:
 * from the network's guess alone (rerun from the warm guess if it does not
 * converge), which measures what the network itself gains.
 * EINVAL on another grid, a negative or non-finite defer_tol or another
 * start.  Drops a captured step graph; allocates nothing. */
enum { GRMHD_LEARNED_BEST = 0, GRMHD_LEARNED_ONLY = 1 };
int grmhd_set_learned_guess(grmhd_grid* h, double defer_tol, int start);
#define GRMHD_MLP_NNORM 32
int grmhd_mlp_set_weights(grmhd_grid* h, const float* host_params, size_t n_params,
                          const float* host_norm, size_t n_norm);
int grmhd_mlp_get_weights(grmhd_grid* h, float* host_params, float* host_norm);
/* Training pairs from device primitives prims (n x 8 float64: rho, u^1..3, p,
 * B^1..3, flat local frame) through the method's prim -> cons map; cons_out
 * (nullable, n x 8 float64) receives D, S_1..3, tau, B^1..3; set_norm != 0
 * also sets the normalisation block from these samples. */
int grmhd_mlp_datagen(grmhd_grid* h, const double* prims, int64_t n, float* feat, float* targ,
                      double* cons_out, int set_norm);
/* Batched point-wise inversion in a flat local frame (the safeguarded Newton
 * of the grid inversion): cons rows D, S_1..3, tau, B^1..3 (device, n x 8
 * float64); y0 (device, nullable): Newton guesses, Gamma U when NULL;
 * prim_out rows rho, u^1..3, p, B^1..3; iters_out (nullable, int32): Newton
 * iterations, negative when the zone failed. */
int grmhd_cons2prim_points(grmhd_grid* h, const double* cons, int64_t n, const double* y0,
                           double* prim_out, int32_t* iters_out);
/* Mean-squared-error gradient over n samples (synchronises; no update). */
int grmhd_mlp_gradient(grmhd_grid* h, const float* feat, const float* targ, int64_t n,
                       float* grad_host, double* loss_host);
/* One Adam step (lr; beta 0.9, 0.999; eps 1e-8) on a batch of samples;
 * loss (nullable) receives the batch loss before the step (synchronises). */
int grmhd_mlp_train_step(grmhd_grid* h, const float* feat, const float* targ, int64_t batch,
                         float lr, double* loss);
int grmhd_mlp_forward(grmhd_grid* h, const float* feat, int64_t n, float* out);

/* Kernel timing (observability).  When enabled, every launch the library
 * makes is bracketed by HIP events on the grid's stream (no host sync);
 * grmhd_get_profile synchronises the stream, accumulates the elapsed times
 * per kernel class and returns totals (ms) and launch counts since the last
 * reset.  Class names: grmhd_profile_class_name(0 .. GRMHD_PROF_NCLASS-1). */
#define GRMHD_PROF_NCLASS 17
typedef struct {
  double ms[GRMHD_PROF_NCLASS];
  int64_t launches[GRMHD_PROF_NCLASS];
} grmhd_profile;
int grmhd_set_profiling(grmhd_grid* h, int on);
int grmhd_get_profile(grmhd_grid* h, grmhd_profile* out, int reset);
const char* grmhd_profile_class_name(int cls);

void grmhd_destroy(grmhd_grid* h);

/* Message of the last failing call on this thread ("" if none). */
const char* grmhd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRMHD_H */
