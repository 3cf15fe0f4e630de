// Host runtime of the C ABI declared in include/grmhd.h: argument checks,
// layout, scratch carving, launch sequencing on the caller's stream, error
// strings.  All numerical work happens in the kernels.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "grmhd.h"
#include "grmhd_kernels.hpp"

// the descriptor's layout, which the Python binding mirrors field by field
static_assert(sizeof(grmhd_grid_desc) == 184 && offsetof(grmhd_grid_desc, recon) == 56 &&
                  offsetof(grmhd_grid_desc, newton_tol) == 168 &&
                  offsetof(grmhd_grid_desc, deriv_order) == 176,
              "grmhd_grid_desc layout");
static_assert(sizeof(grmhd_diag) == 280 && offsetof(grmhd_diag, run_c2p_fail) == 216 &&
                  offsetof(grmhd_diag, run_troubled) == 272,
              "grmhd_diag layout, which the Python binding mirrors");
static_assert(sizeof(grmhd_profile) == GRMHD_PROF_NCLASS * 16, "grmhd_profile layout");
static_assert(GRMHD_RECON_MP5 == grmhd::RECON_MP5 && GRMHD_RECON_WENO5 == grmhd::RECON_WENO5 &&
                  GRMHD_RECON_PLM == grmhd::RECON_PLM && GRMHD_RECON_MP7 == grmhd::RECON_MP7,
              "reconstruction codes of the ABI and the kernels agree");
#include "grmhd_mlp.hpp"

using namespace grmhd;

// ------------------------------------------------------------------ no-allocation scratch
// Per-workgroup partial maxima of the CFL reduction for
// grmhd_compute_dt_noalloc: a file-scope device array (4 MiB on every device
// the library runs on, held until the process ends) instead of the grid's
// library-allocated reduction buffer.  One double per 256-zone workgroup:
// grids of up to NOALLOC_MAX_BLOCKS x 256 = 2^27 interior zones (512^3).
// Host code never uses the array's name as an address: its device address is
// looked up once per device at grmhd_init_grid (noalloc_resolve) and kept.
constexpr long NOALLOC_MAX_BLOCKS = 1L << 19;
static __device__ __align__(256) double scratch[NOALLOC_MAX_BLOCKS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device).  Returns nullptr and sets *err when the lookup fails.
double* noalloc_resolve(int dev, std::string* err) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    *err = "device index beyond the no-allocation table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev]) return g_noalloc_ptr[dev];
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return nullptr;
  }
  g_noalloc_ptr[dev] = static_cast<double*>(p);
  return g_noalloc_ptr[dev];
}
}  // namespace

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GRMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return GRMHD_OK;
}

long round_up(long v, long m) { return (v + m - 1) / m * m; }

// scratch carve (in fields of the single-field layout)
constexpr int SCR_STAGE = 0;     // 8 fields: U^(1), U^(2) of the RK stages
constexpr int SCR_FLUX = 8;      // 3 x 5 fields
constexpr int SCR_CTD = 23;      // 3 x 6 fields
constexpr int SCR_EDGE = 41;     // 3 fields
constexpr int SCR_LIST = 44;     // 1 field: list of zones deferred to the learned-guess pass (int)
constexpr int SCR_NFIELDS = 45;
constexpr int MLP_MAX_WAVES = 256;

const char* const PROF_NAMES[GRMHD_PROF_NCLASS] = {
    "bc_centred", "sweep_x1", "sweep_x2", "sweep_x3", "edge_x1", "edge_x2", "edge_x3",
    "update", "bc_faces", "cons2prim", "cfl", "newton_split", "advance", "rhs_out",
    "learned_guess", "learned_train", "fallback"};
}  // namespace

struct grmhd_grid {
  grmhd_grid_desc desc;
  Geom G;
  BCSpec bc;
  hipStream_t stream = nullptr;
  int device = 0;                  // device current at grmhd_init_grid
  double* noalloc_scratch = nullptr;   // that device's `scratch` (nullptr: lookup failed)
  std::string noalloc_err;
  grmhd_layout lay;
  double* prim = nullptr;
  double* cons = nullptr;
  double* scratch = nullptr;
  double* tab = nullptr;
  bool flat = true;
  bool metric_set = false;
  // library-owned device buffers
  double* d_dt = nullptr;        // [0] dt of the current step, [1] time, [2] CFL dt of the state
  bool next_dt_valid = false;    // d_dt[2] holds the CFL dt of the current primitives
  int* d_list_n = nullptr;       // number of zones deferred to the learned-guess pass
  bool img = false;              // periodic box with n >= 2 ng: ghosts written as images
  double* d_part = nullptr;      // per-block partials (cfl, diagnostics)
  long long* d_spart = nullptr;  // per-block inversion statistics
  long long* d_stats = nullptr;  // reduced inversion statistics (8)
  unsigned long long* d_run = nullptr;  // accumulated inversion counters (RUN_SLOTS x RUN_STRIDE)
  unsigned char* d_trouble = nullptr;   // lower-order fallback: a flag per interior zone,
  int* d_tlist = nullptr;               // the flagged zones of the current stage,
  int* d_ntrouble = nullptr;            // and their number
  double* d_diag = nullptr;      // reduced diagnostics (16)
  unsigned nblk = 0;
  int64_t step = 0;
  // profiling: HIP events around launches on the grid's stream
  bool prof_on = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[GRMHD_PROF_NCLASS] = {0};
  int64_t prof_n[GRMHD_PROF_NCLASS] = {0};
  hipEvent_t take_event() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  template <class F> void timed(int cls, F&& launch) {
    if (!prof_on) { launch(); return; }
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) { launch(); return; }
    (void)hipEventRecord(a, stream);
    launch();
    (void)hipEventRecord(b, stream);
    pending.push_back({cls, a, b});
  }
  double* stage_state() const { return scratch + (long)SCR_STAGE * G.field; }
  double* flux() const { return scratch + (long)SCR_FLUX * G.field; }
  double* ctd() const { return scratch + (long)SCR_CTD * G.field; }
  double* edges() const { return scratch + (long)SCR_EDGE * G.field; }
  int* list() const { return reinterpret_cast<int*>(scratch + (long)SCR_LIST * G.field); }
  // last iterates of the zones a split inversion deferred: the first flux
  // field, whose contents are dead while an inversion runs
  double* list_y() const { return scratch + (long)SCR_FLUX * G.field; }
  int split_it = 0;   // Newton iterations of the first pass of a split inversion (0: off)
  // learned guess: relative warm-start residual above which a zone goes to
  // the network pass (0: every zone), and the start policy there
  double mlp_defer_tol = 1e-2;
  int mlp_start = GRMHD_LEARNED_BEST;
  // one captured device-dt step (grmhd_rk_steps_graph); dropped whenever the
  // launch sequence or a pointer in it changes
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  MlpState mlp;
  bool mlp_alloc = false;
};

static void graph_reset(grmhd_grid* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
}

namespace {

int validate(const grmhd_grid_desc* d) {
  if (!d) return fail(GRMHD_EINVAL, "desc is NULL");
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1 || d->n[a] > (1 << 20)) return fail(GRMHD_EINVAL, "n out of range");
    if (!(d->dx[a] > 0.0) || !std::isfinite(d->dx[a])) return fail(GRMHD_EINVAL, "dx must be > 0");
    if (!std::isfinite(d->x0[a])) return fail(GRMHD_EINVAL, "x0 not finite");
  }
  if (d->ng < 4 || d->ng > 6) return fail(GRMHD_EINVAL, "ng must be 4, 5 or 6");
  if (d->coord != GRMHD_CART && d->coord != GRMHD_LOGSPH) return fail(GRMHD_EINVAL, "bad coord");
  for (int s = 0; s < 6; ++s)
    if (d->bc[s] < 0 || d->bc[s] > 2) return fail(GRMHD_EINVAL, "bad boundary code");
  for (int a = 0; a < 3; ++a) {
    const int lo = d->bc[2 * a], hi = d->bc[2 * a + 1];
    if ((lo == GRMHD_BC_PERIODIC) != (hi == GRMHD_BC_PERIODIC))
      return fail(GRMHD_EINVAL, "periodic boundaries must come in pairs");
    if ((lo == GRMHD_BC_AXIS || hi == GRMHD_BC_AXIS) && (a != 1 || lo != hi))
      return fail(GRMHD_EINVAL, "axis boundary only on both x^2 sides");
  }
  if (d->bc[2] == GRMHD_BC_AXIS) {
    if (d->bc[4] != GRMHD_BC_PERIODIC) return fail(GRMHD_EINVAL, "axis needs periodic x^3");
    if (d->n[2] % 2 != 0) return fail(GRMHD_EINVAL, "axis needs an even n3");
    if (d->n[1] < d->ng + 1) return fail(GRMHD_EINVAL, "axis needs n2 >= ng + 1");
  }
  if (!(d->gamma_ad > 1.0)) return fail(GRMHD_EINVAL, "gamma_ad must be > 1");
  if (!(d->cfl > 0.0)) return fail(GRMHD_EINVAL, "cfl must be > 0");
  if (d->precision != GRMHD_FP64 && d->precision != GRMHD_FP32_FLUX)
    return fail(GRMHD_EINVAL, "bad precision");
  if (d->c2p_guess < 0 || d->c2p_guess > 2) return fail(GRMHD_EINVAL, "bad c2p_guess");
  if (d->newton_maxit < 1 || d->newton_maxit > 1000) return fail(GRMHD_EINVAL, "bad newton_maxit");
  if (!(d->newton_tol > 0.0)) return fail(GRMHD_EINVAL, "newton_tol must be > 0");
  if (d->rho_fl_a < 0.0 || d->p_fl_a < 0.0) return fail(GRMHD_EINVAL, "negative floor");
  if (d->w_max != 0.0 && !(d->w_max > 1.0)) return fail(GRMHD_EINVAL, "w_max must be 0 or > 1");
  if (d->recon != GRMHD_RECON_MP5 && d->recon != GRMHD_RECON_WENO5 && d->recon != GRMHD_RECON_PLM &&
      d->recon != GRMHD_RECON_MP7)
    return fail(GRMHD_EINVAL, "bad recon");
  {
    // faces from -3 (sixth-order derivative) or -2 (fourth) read cells down
    // to the reconstruction's reach below them: 2 more, 3 for MP7
    const int need = (d->deriv_order == 4 ? 2 : 3) + (d->recon == GRMHD_RECON_MP7 ? 3 : 2);
    if (d->ng < need)
      return fail(GRMHD_EINVAL, d->recon == GRMHD_RECON_MP7 ? "MP7 needs ng = 6 (5 with deriv_order 4)"
                                                          : "ng = 4 needs deriv_order 4");
  }
  if (d->deriv_order != 0 && d->deriv_order != 4 && d->deriv_order != 6)
    return fail(GRMHD_EINVAL, "deriv_order must be 0, 4 or 6");
  if (d->fallback != 0 && d->fallback != 1) return fail(GRMHD_EINVAL, "fallback must be 0 or 1");
  return GRMHD_OK;
}

void make_layout(const grmhd_grid_desc& d, grmhd_layout& L, Geom& G) {
  for (int a = 0; a < 3; ++a) L.dims[a] = d.n[a] + 2 * d.ng;
  L.pitch = round_up(L.dims[0], 16);               // 128-byte rows
  L.plane = L.pitch * L.dims[1];
  L.field = round_up(L.plane * L.dims[2], 32);     // 256-byte field starts
  L.offset = (long)d.ng * L.plane + (long)d.ng * L.pitch + d.ng;
  L.prim_doubles = NPRIM * L.field;
  L.cons_doubles = NCONS * L.field;
  L.edge_doubles = L.field;
  L.scratch_bytes = (int64_t)SCR_NFIELDS * L.field * (int64_t)sizeof(double);
  for (int a = 0; a < 3; ++a) {
    G.n[a] = d.n[a];
    G.dims[a] = (int)L.dims[a];
    G.dx[a] = d.dx[a];
    G.x0[a] = d.x0[a];
  }
  G.pitch = L.pitch;
  G.plane = L.plane;
  G.field = L.field;
  G.off = L.offset;
  G.gam = d.gamma_ad;
  G.dorder = d.deriv_order == 4 ? 4 : 6;
  G.ng = d.ng;
  G.axis2 = d.bc[2] == GRMHD_BC_AXIS ? 1 : 0;
  G.tab_n1 = (int)L.dims[0];
  G.tab_plane = L.dims[0] * L.dims[1];
}

C2PParams c2p_params(const grmhd_grid* h) {
  const grmhd_grid_desc& d = h->desc;
  C2PParams cp;
  cp.run_acc = h->d_run;
  const bool mlp = d.c2p_guess == GRMHD_GUESS_MLP;
  cp.defer_all = mlp && h->mlp_defer_tol == 0.0 ? 1 : 0;
  cp.learned_only = mlp && h->mlp_start == GRMHD_LEARNED_ONLY ? 1 : 0;
  cp.tol = d.newton_tol;
  cp.maxit = d.newton_maxit;
  cp.guess = d.c2p_guess;
  cp.coord = d.coord;
  cp.rho_fl_a = d.rho_fl_a;
  cp.rho_fl_n = d.rho_fl_n;
  cp.p_fl_a = d.p_fl_a;
  cp.p_fl_n = d.p_fl_n;
  cp.w_max = d.w_max;
  // learned guess: zones whose warm start (the previous primitives) leaves a
  // relative residual above mlp_defer_tol (1e-2 unless set) go to the network
  // pass; elsewhere the warm start is better than the network's accuracy
  cp.defer_tol = mlp && h->mlp_defer_tol > 0.0 ? h->mlp_defer_tol : 0.0;
  cp.img = 0;
  cp.split_it = 0;
  return cp;
}

int ready(grmhd_grid* h) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  if (!h->prim || !h->cons || !h->scratch) return fail(GRMHD_ESTATE, "fields not bound");
  if (!h->metric_set) return fail(GRMHD_ESTATE, "metric not set");
  return GRMHD_OK;
}

}  // namespace

extern "C" {

const char* grmhd_last_error(void) { return g_err.c_str(); }

int grmhd_init_grid(const grmhd_grid_desc* desc, void* hip_stream, grmhd_grid** out) {
  g_err.clear();
  if (!out) return fail(GRMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(desc);
  if (rc) return rc;
  grmhd_grid* h = new grmhd_grid();
  h->desc = *desc;
  make_layout(*desc, h->lay, h->G);
  for (int s = 0; s < 6; ++s) h->bc.bc[s] = desc->bc[s];
  h->img = true;
  for (int s = 0; s < 6; ++s) h->img = h->img && desc->bc[s] == GRMHD_BC_PERIODIC;
  for (int d = 0; d < 3; ++d) h->img = h->img && desc->n[d] >= 2 * desc->ng;
  h->stream = (hipStream_t)hip_stream;
  h->nblk = zone_blocks(h->G);
  // the device address of the no-allocation scratch, once per device; a
  // failed lookup only disables grmhd_compute_dt_noalloc
  if (hipGetDevice(&h->device) == hipSuccess)
    h->noalloc_scratch = noalloc_resolve(h->device, &h->noalloc_err);
  else
    h->noalloc_err = "hipGetDevice failed";
  // reduction partials: diagnostics (nblk x 16), CFL (nblk + learned-pass
  // blocks), shell fluxes (chunk partials, then the 4 n1 results)
  const size_t part = std::max(std::max((size_t)h->nblk * (DIAG_NSUM + DIAG_NMAX),
                                        (size_t)h->nblk + C2P_LIST_BLOCKS),
                               (size_t)std::max(shell_part_doubles(h->G) + 4L * desc->n[0],
                                                mri_part_doubles(h->G) + 6L * desc->n[0])) *
                      sizeof(double);
  const size_t spart = ((size_t)h->nblk + C2P_LIST_BLOCKS) * C2P_NSTAT * sizeof(long long);
  hipError_t e = hipSuccess;
  e = hipMalloc(&h->d_dt, 3 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&h->d_part, part);
  if (e == hipSuccess) e = hipMalloc(&h->d_spart, spart);
  if (e == hipSuccess) e = hipMalloc(&h->d_list_n, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(h->d_spart, 0, spart, h->stream);
  if (e == hipSuccess) e = hipMalloc(&h->d_stats, C2P_NSTAT * sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&h->d_diag, (DIAG_NSUM + DIAG_NMAX) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&h->d_run, (size_t)RUN_SLOTS * RUN_STRIDE * sizeof(unsigned long long));
  if (e == hipSuccess) launch_zero_u64(h->d_run, RUN_SLOTS * RUN_STRIDE, h->stream);
  if (e == hipSuccess && desc->fallback) {
    const size_t nz = (size_t)desc->n[0] * desc->n[1] * desc->n[2];
    e = hipMalloc(&h->d_trouble, nz);
    if (e == hipSuccess) e = hipMalloc(&h->d_tlist, nz * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&h->d_ntrouble, sizeof(int));
    if (e == hipSuccess) launch_zero_int(h->d_ntrouble, h->stream);
  }
  if (e == hipSuccess) e = hipMemsetAsync(h->d_dt, 0, 3 * sizeof(double), h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->d_stats, 0, C2P_NSTAT * sizeof(long long), h->stream);
  if (e != hipSuccess) {
    std::string m = std::string("device buffers: ") + hipGetErrorString(e);
    grmhd_destroy(h);
    return fail(e == hipErrorOutOfMemory ? GRMHD_ENOMEM : GRMHD_EHIP, m);
  }
  *out = h;
  return GRMHD_OK;
}

int grmhd_get_layout(const grmhd_grid* h, grmhd_layout* out) {
  if (!h || !out) return fail(GRMHD_EINVAL, "NULL argument");
  *out = h->lay;
  return GRMHD_OK;
}

int grmhd_bind_fields(grmhd_grid* h, double* prim, double* cons, void* scratch,
                      size_t scratch_bytes) {
  if (!h || !prim || !cons || !scratch) return fail(GRMHD_EINVAL, "NULL argument");
  if (((uintptr_t)prim | (uintptr_t)cons | (uintptr_t)scratch) % 256 != 0)
    return fail(GRMHD_EINVAL, "field pointers must be 256-byte aligned");
  if ((int64_t)scratch_bytes < h->lay.scratch_bytes)
    return fail(GRMHD_EINVAL, "scratch smaller than layout.scratch_bytes");
  graph_reset(h);
  h->prim = prim;
  h->cons = cons;
  h->scratch = (double*)scratch;
  h->next_dt_valid = false;
  return GRMHD_OK;
}

int grmhd_set_metric(grmhd_grid* h, int kind, const double* host_tables, size_t n_doubles) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  h->next_dt_valid = false;
  graph_reset(h);
  if (kind == GRMHD_METRIC_MINKOWSKI) {
    if (h->desc.coord != GRMHD_CART) return fail(GRMHD_EINVAL, "Minkowski kind needs Cartesian coordinates");
    if (h->tab) { (void)hipFree(h->tab); h->tab = nullptr; }
    h->flat = true;
    h->metric_set = true;
    return GRMHD_OK;
  }
  if (kind != GRMHD_METRIC_TABLE_AXISYM) return fail(GRMHD_EUNSUPPORTED, "unknown metric kind");
  const size_t need = (size_t)NCOMP_TAB * h->lay.dims[0] * h->lay.dims[1];
  if (!host_tables || n_doubles != need) return fail(GRMHD_EINVAL, "table size mismatch");
  for (size_t q = 0; q < need; ++q)
    if (!std::isfinite(host_tables[q])) return fail(GRMHD_EINVAL, "non-finite metric table entry");
  double* t = nullptr;
  hipError_t e = hipMalloc(&t, need * sizeof(double));
  if (e != hipSuccess) return fail(GRMHD_ENOMEM, std::string("metric tables: ") + hipGetErrorString(e));
  e = hipMemcpy(t, host_tables, need * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(t); return fail(GRMHD_EHIP, std::string("metric copy: ") + hipGetErrorString(e)); }
  if (h->tab) (void)hipFree(h->tab);
  h->tab = t;
  h->flat = false;
  h->metric_set = true;
  return GRMHD_OK;
}

int grmhd_curl_potential(grmhd_grid* h, const double* A1, const double* A2, const double* A3) {
  int rc = ready(h);
  if (rc) return rc;
  if (!A1 || !A2 || !A3) return fail(GRMHD_EINVAL, "NULL potential");
  h->next_dt_valid = false;
  h->timed(15, [&] {
    launch_curl(h->G, A1, A2, A3, h->cons, h->stream);
    launch_ghost_normal_curl(h->G, h->bc, A1, A2, A3, h->cons, h->stream);
  });
  h->timed(8, [&] { launch_bc_faces(h->G, h->bc, h->cons, h->stream); });
  return hip_check("curl_potential");
}

int grmhd_prim2cons(grmhd_grid* h) {
  int rc = ready(h);
  if (rc) return rc;
  h->next_dt_valid = false;
  h->timed(8, [&] { launch_bc_faces(h->G, h->bc, h->cons, h->stream); });
  h->timed(15, [&] { launch_prim2cons(h->G, h->flat, h->prim, h->cons, h->tab, h->stream); });
  h->timed(0, [&] { launch_bc_centred(h->G, h->bc, h->prim, NPRIM, h->stream); });
  return hip_check("prim2cons");
}

// fill_ghosts: ghost fill of the primitives first (skipped inside rk_step on
// a periodic box, where the inversion writes the ghost images itself).
// cons_cur: the conserved state the right-hand side reads (its face fields):
// the bound cons, or the step's scratch stage buffer.
static void rhs_pieces(grmhd_grid* h, bool fill_ghosts = true, double* cons_cur = nullptr) {
  double* const U = cons_cur ? cons_cur : h->cons;
  const bool fp32 = h->desc.precision == GRMHD_FP32_FLUX;
  if (fill_ghosts) h->timed(0, [&] { launch_bc_centred(h->G, h->bc, h->prim, NPRIM, h->stream); });
  for (int d = 0; d < 3; ++d)
    h->timed(1 + d, [&] {
      launch_sweep(d, h->G, h->flat, fp32, h->desc.recon, h->prim, U, h->tab, h->flux(), h->ctd(),
                   h->stream);
    });
  for (int e = 0; e < 3; ++e)
    h->timed(4 + e, [&] {
      launch_edge(e, h->G, h->flat, fp32, h->desc.recon, U, h->tab, h->ctd(), h->edges(), h->stream);
    });
}

// with_cfl: also reduce the CFL time step of the inverted state into d_dt[2].
// Learned guess: the inversion defers zones with a poor warm start to a list,
// the network pass inverts those; counters and CFL partials of both passes
// are reduced together.
// cons_cur: the conserved state to invert (the bound cons, or the step's
// scratch stage buffer); floored zones are written back to it.
static void c2p_with_guess(grmhd_grid* h, const C2PParams& cp, bool with_cfl = false,
                           double* cons_cur = nullptr) {
  double* const U = cons_cur ? cons_cur : h->cons;
  double* cflp = with_cfl ? h->d_part : nullptr;
  const int nb = (int)h->nblk;
  if (cp.guess == GRMHD_GUESS_MLP) {
    h->timed(9, [&] {
      launch_zero_int(h->d_list_n, h->stream);
      launch_c2p(h->G, h->flat, cp, h->prim, U, h->tab, h->d_spart, cflp, h->list(), h->d_list_n,
                 nullptr, h->stream);
    });
    h->timed(14, [&] {
      mlp_launch_c2p_list(h->G, h->flat, cp, h->prim, U, h->tab, h->mlp, h->list(), h->d_list_n,
                          h->d_spart + (long)nb * C2P_NSTAT, cflp ? cflp + nb : nullptr, h->stream);
    });
    if (with_cfl) launch_dt_final(cflp, nb + C2P_LIST_BLOCKS, h->desc.cfl, h->d_dt + 2, h->stream);
  } else if (h->split_it > 0) {
    C2PParams c1 = cp;
    c1.split_it = h->split_it;
    h->timed(9, [&] {
      launch_zero_int(h->d_list_n, h->stream);
      launch_c2p(h->G, h->flat, c1, h->prim, U, h->tab, h->d_spart, cflp, h->list(), h->d_list_n,
                 h->list_y(), h->stream);
    });
    h->timed(11, [&] {
      launch_c2p_split(h->G, h->flat, cp, h->prim, U, h->tab, h->list(), h->d_list_n, h->list_y(),
                       h->d_spart + (long)nb * C2P_NSTAT, cflp ? cflp + nb : nullptr, h->stream);
    });
    if (with_cfl) launch_dt_final(cflp, nb + C2P_LIST_BLOCKS, h->desc.cfl, h->d_dt + 2, h->stream);
  } else {
    h->timed(9, [&] {
      launch_c2p(h->G, h->flat, cp, h->prim, U, h->tab, h->d_spart, cflp, nullptr, nullptr, nullptr,
                 h->stream);
    });
    if (with_cfl) launch_dt_final(cflp, nb, h->desc.cfl, h->d_dt + 2, h->stream);
  }
}

static int mlp_ready(grmhd_grid* h) {
  if (h->desc.c2p_guess == GRMHD_GUESS_MLP && !h->mlp.weights_set)
    return fail(GRMHD_ESTATE, "learned guess selected but no weights set");
  return GRMHD_OK;
}

int grmhd_rhs(grmhd_grid* h, double* rhs_out) {
  int rc = ready(h);
  if (rc) return rc;
  if (!rhs_out) return fail(GRMHD_EINVAL, "rhs_out is NULL");
  rhs_pieces(h);
  h->timed(13, [&] {
    launch_update(h->G, h->flat, h->desc.precision == GRMHD_FP32_FLUX, 1, h->prim, h->cons, h->stage_state(),
                  h->flux(), h->edges(), h->tab,
                  0.0, 0.0, 0.0, h->d_dt, rhs_out, 1, h->stream);
  });
  return hip_check("rhs");
}

// The three stages of one SSP-RK3 step (dt <= 0: the device CFL step in
// d_dt[2], reduced again by the last inversion for the next step).  Kernel
// launches only, on the grid's stream: a step whose dt is already on the
// device is captured into a graph as it stands.
static void step_stages(grmhd_grid* h, double dt) {
  const bool device_dt = dt <= 0.0;
  const double* dt_src = h->d_dt + 2;
  // Shu-Osher weights: U^(s+1) = A[s] U^n + B[s] (U^(s) + dt L(U^(s)))
  const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
  // periodic box: the update and the inversion write the ghost images of
  // what they produce, so the stage needs no separate ghost fills
  C2PParams cp = c2p_params(h);
  const bool img = h->img && h->flat;
  cp.img = img ? 1 : 0;
  // stage buffers: U^n stays in the bound cons until the last stage writes
  // U^(3) over it; U^(1) and U^(2) live in the scratch buffer S (no copy of U^n)
  double* const Un = h->cons;
  double* const S = h->stage_state();
  for (int s = 0; s < 3; ++s) {
    double* const cur = s == 0 ? Un : S;        // state the stage's RHS reads
    double* const next = s == 2 ? Un : S;       // state the stage produces
    rhs_pieces(h, !img, cur);
    const bool fp32 = h->desc.precision == GRMHD_FP32_FLUX;
    h->timed(7, [&] {
      if (!h->desc.fallback) {
        launch_update(h->G, h->flat, fp32, 0, h->prim, s == 0 ? Un : S, s == 0 ? S : Un, h->flux(),
                      h->edges(), h->tab, A[s], B[s], dt, dt_src, nullptr, s + 1, h->stream, img ? 1 : 0);
      } else {
        // lower-order fallback: the hydro update flags troubled zones, the
        // fix replaces the fluxes at their faces (reading the face fields of
        // the stage's start, which stage 2 updates in place), then the
        // induction update
        UpdateFallback fb{h->d_trouble, h->d_tlist, h->d_ntrouble};
        launch_zero_int(h->d_ntrouble, h->stream);
        launch_update(h->G, h->flat, fp32, 0, h->prim, s == 0 ? Un : S, s == 0 ? S : Un, h->flux(),
                      h->edges(), h->tab, A[s], B[s], dt, dt_src, nullptr, s + 1, h->stream, img ? 1 : 0,
                      UPD_HYDRO, &fb);
      }
    });
    if (h->desc.fallback) {
      h->timed(16, [&] {
        // the face deltas go to the per-face edge-field data, which the
        // stage's edge fields have consumed and the next sweeps overwrite
        launch_fallback(h->G, h->flat, fp32, h->bc, h->prim, cur, next, h->flux(), h->tab, h->d_trouble,
                        h->d_tlist, h->d_ntrouble, h->ctd(), B[s], dt, dt_src, h->d_run, h->stream);
      });
      h->timed(7, [&] {
        launch_update(h->G, h->flat, fp32, 0, h->prim, s == 0 ? Un : S, s == 0 ? S : Un, h->flux(),
                      h->edges(), h->tab, A[s], B[s], dt, dt_src, nullptr, s + 1, h->stream, img ? 1 : 0,
                      UPD_INDUCTION);
      });
    }
    // normal to a non-periodic boundary the ghost faces the divergence of
    // the cells beside it reads evolve with the induction equation too
    if (!img)
      h->timed(7, [&] {
        launch_ghost_normal_update(h->G, h->bc, fp32, s == 0 ? Un : S, s == 0 ? S : Un, h->edges(), A[s], B[s],
                                   dt, dt_src, s + 1, h->stream);
      });
    // dt and time are recorded once the last update has consumed d_dt[2]
    if (s == 2) h->timed(12, [&] { launch_advance(h->d_dt, dt_src, dt, h->stream); });
    if (!img) h->timed(8, [&] { launch_bc_faces(h->G, h->bc, next, h->stream); });
    c2p_with_guess(h, cp, s == 2 && device_dt, next);
  }
}

int grmhd_rk_step(grmhd_grid* h, double dt, double* dt_used) {
  int rc = ready(h);
  if (rc) return rc;
  rc = mlp_ready(h);
  if (rc) return rc;
  if (!std::isfinite(dt)) return fail(GRMHD_EINVAL, "dt not finite");
  // Device time step: the CFL dt of the current primitives.  When the last
  // state change was a step taken in this mode, its final inversion already
  // reduced that value into d_dt[2]; otherwise it is reduced here.
  const bool device_dt = dt <= 0.0;
  if (device_dt && !h->next_dt_valid)
    h->timed(10, [&] { launch_cfl(h->G, h->flat, h->prim, h->tab, h->desc.cfl, h->d_part, h->d_dt + 2, h->stream); });
  h->next_dt_valid = false;
  step_stages(h, dt);
  h->step += 1;
  rc = hip_check("rk_step");
  if (rc) return rc;
  h->next_dt_valid = device_dt;
  if (dt_used) {
    hipError_t e = hipMemcpyAsync(dt_used, h->d_dt, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  }
  return GRMHD_OK;
}

int grmhd_rk_steps_graph(grmhd_grid* h, int32_t nsteps) {
  int rc = ready(h);
  if (rc) return rc;
  rc = mlp_ready(h);
  if (rc) return rc;
  if (nsteps < 0) return fail(GRMHD_EINVAL, "nsteps must be >= 0");
  if (h->prof_on) return fail(GRMHD_ESTATE, "graph replay needs kernel timing off");
  if (h->stream == nullptr) return fail(GRMHD_ESTATE, "graph replay needs a stream other than the null stream");
  int done = 0;
  // the first step after a state change also reduces the CFL step: eager
  if (nsteps > 0 && !h->next_dt_valid) {
    rc = grmhd_rk_step(h, 0.0, nullptr);
    if (rc) return rc;
    done = 1;
  }
  if (done < nsteps && !h->gexec) {
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
    step_stages(h, 0.0);
    e = hipStreamEndCapture(h->stream, &h->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      graph_reset(h);
      return fail(GRMHD_EHIP, hipGetErrorString(e));
    }
  }
  for (; done < nsteps; ++done) {
    hipError_t e = hipGraphLaunch(h->gexec, h->stream);
    if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
    h->step += 1;
    h->next_dt_valid = true;
  }
  return hip_check("rk_steps_graph");
}

int grmhd_cons2prim(grmhd_grid* h, int64_t* n_fail, int strict) {
  int rc = ready(h);
  if (rc) return rc;
  rc = mlp_ready(h);
  if (rc) return rc;
  if (strict && !n_fail) return fail(GRMHD_EINVAL, "strict mode needs n_fail");
  h->next_dt_valid = false;
  C2PParams cp = c2p_params(h);
  cp.img = h->img && h->flat ? 1 : 0;   // leaves the primitive ghosts filled, as rk_step expects
  h->timed(8, [&] { launch_bc_faces(h->G, h->bc, h->cons, h->stream); });
  c2p_with_guess(h, cp);
  rc = hip_check("cons2prim");
  if (rc) return rc;
  if (n_fail) {
    long long st[C2P_NSTAT];
    launch_reduce_stats(h->d_spart, (int)h->nblk + C2P_LIST_BLOCKS, h->d_stats, h->stream);
    hipError_t e = hipMemcpyAsync(st, h->d_stats, sizeof(st), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
    *n_fail = st[0];
    if (strict && st[0] > 0) return fail(GRMHD_ENOCONV, "inversion failed in some zones");
  }
  return GRMHD_OK;
}

int grmhd_compute_dt(grmhd_grid* h, double* dt) {
  int rc = ready(h);
  if (rc) return rc;
  if (!dt) return fail(GRMHD_EINVAL, "dt is NULL");
  h->timed(10, [&] { launch_cfl(h->G, h->flat, h->prim, h->tab, h->desc.cfl, h->d_part, h->d_dt + 2, h->stream); });
  h->next_dt_valid = true;
  hipError_t e = hipMemcpyAsync(dt, h->d_dt + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return hip_check("compute_dt");
}

int grmhd_compute_dt_noalloc(grmhd_grid* h, double* dt_dev) {
  int rc = ready(h);
  if (rc) return rc;
  if (!dt_dev) return fail(GRMHD_EINVAL, "dt_dev is NULL");
  if ((long)h->nblk > NOALLOC_MAX_BLOCKS)
    return fail(GRMHD_EINVAL, "grid too large for the no-allocation scratch (at most 2^27 interior zones)");
  if (!h->noalloc_scratch) return fail(GRMHD_EHIP, "no-allocation scratch unavailable: " + h->noalloc_err);
  launch_cfl(h->G, h->flat, h->prim, h->tab, h->desc.cfl, h->noalloc_scratch, dt_dev, h->stream);
  return hip_check("compute_dt_noalloc");
}

int grmhd_shell_fluxes(grmhd_grid* h, double* host_out, size_t n_doubles) {
  int rc = ready(h);
  if (rc) return rc;
  if (!host_out) return fail(GRMHD_EINVAL, "host_out is NULL");
  if (n_doubles < (size_t)4 * h->G.n[0]) return fail(GRMHD_EINVAL, "host_out needs 4 n1 doubles");
  double* res = h->d_part + shell_part_doubles(h->G);
  launch_shell(h->G, h->flat, h->prim, h->cons, h->tab, h->d_part, res, h->stream);
  hipError_t e = hipMemcpyAsync(host_out, res, (size_t)4 * h->G.n[0] * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return hip_check("shell_fluxes");
}

int grmhd_mri_quality(grmhd_grid* h, double rho_cut, double q_min, double* host_out, size_t n_doubles) {
  int rc = ready(h);
  if (rc) return rc;
  if (!host_out) return fail(GRMHD_EINVAL, "host_out is NULL");
  if (n_doubles < (size_t)6 * h->G.n[0]) return fail(GRMHD_EINVAL, "host_out needs 6 n1 doubles");
  if (!(rho_cut >= 0.0)) return fail(GRMHD_EINVAL, "rho_cut must be >= 0");
  double* res = h->d_part + mri_part_doubles(h->G);
  launch_mri(h->G, h->flat, h->prim, h->tab, rho_cut, q_min, h->d_part, res, h->stream);
  hipError_t e = hipMemcpyAsync(host_out, res, (size_t)6 * h->G.n[0] * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return hip_check("mri_quality");
}

int grmhd_diagnostics(grmhd_grid* h, grmhd_diag* out) {
  int rc = ready(h);
  if (rc) return rc;
  if (!out) return fail(GRMHD_EINVAL, "out is NULL");
  double dg[DIAG_NSUM + DIAG_NMAX];
  long long st[C2P_NSTAT];
  double dtt[2] = {0.0, 0.0};
  launch_diag(h->G, h->flat, h->prim, h->cons, h->tab, h->d_part, h->d_diag, h->stream);
  launch_reduce_stats(h->d_spart, (int)h->nblk + C2P_LIST_BLOCKS, h->d_stats, h->stream);
  hipError_t e = hipMemcpyAsync(dg, h->d_diag, sizeof(dg), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(st, h->d_stats, sizeof(st), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dtt, h->d_dt, sizeof(dtt), hipMemcpyDeviceToHost, h->stream);
  std::vector<unsigned long long> run((size_t)RUN_SLOTS * RUN_STRIDE, 0ull);
  if (e == hipSuccess)
    e = hipMemcpyAsync(run.data(), h->d_run, run.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  rc = hip_check("diagnostics");
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->step = h->step;
  out->t = dtt[1];
  out->dt = dtt[0];
  for (int q = 0; q < 8; ++q) out->sum_cons[q] = dg[q];
  out->max_divb = dg[DIAG_NSUM + 0];
  out->rho_min = -dg[DIAG_NSUM + 1];
  out->rho_max = dg[DIAG_NSUM + 2];
  out->p_min = -dg[DIAG_NSUM + 3];
  out->p_max = dg[DIAG_NSUM + 4];
  out->w_max = dg[DIAG_NSUM + 5];
  const double bmax = dg[DIAG_NSUM + 6];
  double dxmin = h->G.dx[0];
  for (int a = 1; a < 3; ++a) dxmin = dxmin < h->G.dx[a] ? dxmin : h->G.dx[a];
  out->max_divb_norm = bmax > 0.0 ? out->max_divb * dxmin / bmax : 0.0;
  out->n_nonfinite = (int64_t)dg[DIAG_NSUM + 7];
  out->n_c2p_fail = st[0];
  out->newton_iters_sum = st[1];
  out->newton_iters_max = st[2];
  out->n_floor_rho = st[3];
  out->n_floor_p = st[4];
  out->n_wcap = st[5];
  out->n_mlp_fallback = st[6];
  out->n_mlp_chosen = st[7];
  int64_t acc[RUN_NCOUNT] = {0};
  for (int sl = 0; sl < RUN_SLOTS; ++sl)
    for (int q = 0; q < RUN_NCOUNT; ++q) acc[q] += (int64_t)run[(size_t)sl * RUN_STRIDE + q];
  out->run_c2p_fail = acc[0];
  out->run_floor_rho = acc[1];
  out->run_floor_p = acc[2];
  out->run_wcap = acc[3];
  out->run_mlp_deferred = acc[4];
  out->run_mlp_chosen = acc[5];
  out->run_mlp_fallback = acc[6];
  out->run_troubled = acc[7];
  return GRMHD_OK;
}

int grmhd_reset_run_counters(grmhd_grid* h) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  launch_zero_u64(h->d_run, RUN_SLOTS * RUN_STRIDE, h->stream);
  return hip_check("reset_run_counters");
}

static int mlp_alloc(grmhd_grid* h) {
  if (h->mlp_alloc) return GRMHD_OK;
  MlpState& M = h->mlp;
  hipError_t e = hipMalloc(&M.wb, NPARAM * sizeof(unsigned short));
  if (e == hipSuccess) e = hipMalloc(&M.wf, NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M.norm, mlp::NNORM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M.m1, NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M.m2, NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M.part, (size_t)MLP_MAX_WAVES * NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M.part_loss, MLP_MAX_WAVES * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&M.loss, sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&M.dpart, 256 * 32 * sizeof(double));
  if (e == hipSuccess) e = hipMemsetAsync(M.m1, 0, NPARAM * sizeof(float), h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(M.m2, 0, NPARAM * sizeof(float), h->stream);
  if (e != hipSuccess) return fail(GRMHD_ENOMEM, std::string("learned-guess buffers: ") + hipGetErrorString(e));
  h->mlp_alloc = true;
  return GRMHD_OK;
}

int grmhd_mlp_set_weights(grmhd_grid* h, const float* host_params, size_t n_params,
                          const float* host_norm, size_t n_norm) {
  if (!h || !host_params || !host_norm) return fail(GRMHD_EINVAL, "NULL argument");
  if (n_params != (size_t)NPARAM || n_norm != (size_t)mlp::NNORM)
    return fail(GRMHD_EINVAL, "parameter or normalisation size mismatch");
  for (size_t q = 0; q < n_params; ++q)
    if (!std::isfinite(host_params[q])) return fail(GRMHD_EINVAL, "non-finite weight");
  for (size_t q = 0; q < n_norm; ++q)
    if (!std::isfinite(host_norm[q])) return fail(GRMHD_EINVAL, "non-finite normalisation");
  graph_reset(h);
  int rc = mlp_alloc(h);
  if (rc) return rc;
  hipError_t e = hipMemcpy(h->mlp.wf, host_params, NPARAM * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->mlp.norm, host_norm, mlp::NNORM * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(h->mlp.m1, 0, NPARAM * sizeof(float), h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->mlp.m2, 0, NPARAM * sizeof(float), h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  mlp_launch_to_bf16(h->mlp, h->stream);
  h->mlp.step = 0;
  h->mlp.weights_set = true;
  return hip_check("mlp_set_weights");
}

int grmhd_mlp_get_weights(grmhd_grid* h, float* host_params, float* host_norm) {
  if (!h || !host_params || !host_norm) return fail(GRMHD_EINVAL, "NULL argument");
  if (!h->mlp_alloc) return fail(GRMHD_ESTATE, "no learned-guess state");
  hipError_t e = hipMemcpyAsync(host_params, h->mlp.wf, NPARAM * sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(host_norm, h->mlp.norm, mlp::NNORM * sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return GRMHD_OK;
}

int grmhd_mlp_datagen(grmhd_grid* h, const double* prims, int64_t n, float* feat, float* targ,
                      double* cons_out, int set_norm) {
  if (!h || !prims || !feat || !targ || n <= 0) return fail(GRMHD_EINVAL, "bad argument");
  int rc = mlp_alloc(h);
  if (rc) return rc;
  h->timed(15, [&] {
    mlp_launch_datagen(prims, (long)n, h->desc.gamma_ad, feat, targ, cons_out, h->mlp.dpart,
                       set_norm ? h->mlp.norm : nullptr, h->stream);
  });
  return hip_check("mlp_datagen");
}

int grmhd_cons2prim_points(grmhd_grid* h, const double* cons, int64_t n, const double* y0,
                           double* prim_out, int32_t* iters_out) {
  if (!h || !cons || !prim_out || n <= 0) return fail(GRMHD_EINVAL, "bad argument");
  launch_points_c2p(cons, (long)n, h->desc.gamma_ad, y0, h->desc.newton_tol, h->desc.newton_maxit,
                    prim_out, (int*)iters_out, h->stream);
  return hip_check("cons2prim_points");
}

static int nwaves_for(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  return (int)(tiles < MLP_MAX_WAVES ? tiles : MLP_MAX_WAVES);
}

int grmhd_mlp_gradient(grmhd_grid* h, const float* feat, const float* targ, int64_t n,
                       float* grad_host, double* loss_host) {
  if (!h || !feat || !targ || !grad_host || n <= 0) return fail(GRMHD_EINVAL, "bad argument");
  if (!h->mlp.weights_set) return fail(GRMHD_ESTATE, "weights not set");
  const int nw = nwaves_for(n);
  float* g = nullptr;
  hipError_t e = hipMalloc(&g, NPARAM * sizeof(float));
  if (e != hipSuccess) return fail(GRMHD_ENOMEM, hipGetErrorString(e));
  mlp_launch_grad(h->mlp, feat, targ, (long)n, nw, h->stream);
  mlp_launch_reduce(h->mlp, nw, 0, g, 0.f, 1, h->stream);
  e = hipMemcpyAsync(grad_host, g, NPARAM * sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && loss_host) e = hipMemcpyAsync(loss_host, h->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(g);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return hip_check("mlp_gradient");
}

int grmhd_mlp_train_step(grmhd_grid* h, const float* feat, const float* targ, int64_t batch,
                         float lr, double* loss) {
  if (!h || !feat || !targ || batch <= 0 || !(lr > 0.f)) return fail(GRMHD_EINVAL, "bad argument");
  if (!h->mlp.weights_set) return fail(GRMHD_ESTATE, "weights not set");
  const int nw = nwaves_for(batch);
  h->mlp.step += 1;
  h->timed(15, [&] {
    mlp_launch_grad(h->mlp, feat, targ, (long)batch, nw, h->stream);
    mlp_launch_reduce(h->mlp, nw, 1, nullptr, lr, h->mlp.step, h->stream);
  });
  int rc = hip_check("mlp_train_step");
  if (rc) return rc;
  if (loss) {
    hipError_t e = hipMemcpyAsync(loss, h->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  }
  return GRMHD_OK;
}

int grmhd_mlp_forward(grmhd_grid* h, const float* feat, int64_t n, float* out) {
  if (!h || !feat || !out || n <= 0) return fail(GRMHD_EINVAL, "bad argument");
  if (!h->mlp.weights_set) return fail(GRMHD_ESTATE, "weights not set");
  mlp_launch_forward(h->mlp, feat, (long)n, out, h->stream);
  return hip_check("mlp_forward");
}

int grmhd_set_newton_split(grmhd_grid* h, int32_t iters) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  if (iters < 0 || iters >= h->desc.newton_maxit)
    return fail(GRMHD_EINVAL, "split iterations must be in [0, newton_maxit)");
  if (iters > 0 && h->desc.c2p_guess == GRMHD_GUESS_MLP)
    return fail(GRMHD_EINVAL, "the split inversion is not combined with the learned guess");
  if (iters == h->split_it) return GRMHD_OK;
  graph_reset(h);
  h->split_it = iters;
  // the second pass's counter slots must read zero whenever it does not run
  hipError_t e = hipMemsetAsync(h->d_spart + (long)h->nblk * C2P_NSTAT, 0,
                                (size_t)C2P_LIST_BLOCKS * C2P_NSTAT * sizeof(long long), h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  return GRMHD_OK;
}

int grmhd_set_learned_guess(grmhd_grid* h, double defer_tol, int start) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  if (h->desc.c2p_guess != GRMHD_GUESS_MLP) return fail(GRMHD_EINVAL, "the grid does not use the learned guess");
  if (!(defer_tol >= 0.0) || !std::isfinite(defer_tol)) return fail(GRMHD_EINVAL, "defer_tol must be finite and >= 0");
  if (start != GRMHD_LEARNED_BEST && start != GRMHD_LEARNED_ONLY) return fail(GRMHD_EINVAL, "bad start policy");
  if (defer_tol == h->mlp_defer_tol && start == h->mlp_start) return GRMHD_OK;
  graph_reset(h);
  h->mlp_defer_tol = defer_tol;
  h->mlp_start = start;
  return GRMHD_OK;
}

int grmhd_set_profiling(grmhd_grid* h, int on) {
  if (!h) return fail(GRMHD_EINVAL, "grid handle is NULL");
  h->prof_on = on != 0;
  return GRMHD_OK;
}

int grmhd_get_profile(grmhd_grid* h, grmhd_profile* out, int reset) {
  if (!h || !out) return fail(GRMHD_EINVAL, "NULL argument");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GRMHD_EHIP, hipGetErrorString(e));
  for (auto& r : h->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      h->prof_ms[r.cls] += ms;
      h->prof_n[r.cls] += 1;
    }
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
  }
  h->pending.clear();
  for (int c = 0; c < GRMHD_PROF_NCLASS; ++c) {
    out->ms[c] = h->prof_ms[c];
    out->launches[c] = h->prof_n[c];
    if (reset) { h->prof_ms[c] = 0.0; h->prof_n[c] = 0; }
  }
  return GRMHD_OK;
}

const char* grmhd_profile_class_name(int cls) {
  if (cls < 0 || cls >= GRMHD_PROF_NCLASS) return "";
  return PROF_NAMES[cls];
}

void grmhd_destroy(grmhd_grid* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream); else (void)hipDeviceSynchronize();
  graph_reset(h);
  for (auto& r : h->pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto ev : h->pool) (void)hipEventDestroy(ev);
  if (h->mlp_alloc) {
    (void)hipFree(h->mlp.wb); (void)hipFree(h->mlp.wf); (void)hipFree(h->mlp.norm);
    (void)hipFree(h->mlp.m1); (void)hipFree(h->mlp.m2); (void)hipFree(h->mlp.part);
    (void)hipFree(h->mlp.part_loss); (void)hipFree(h->mlp.loss); (void)hipFree(h->mlp.dpart);
  }
  (void)hipFree(h->tab);
  (void)hipFree(h->d_dt);
  (void)hipFree(h->d_list_n);
  (void)hipFree(h->d_part);
  (void)hipFree(h->d_spart);
  (void)hipFree(h->d_stats);
  (void)hipFree(h->d_diag);
  (void)hipFree(h->d_run);
  (void)hipFree(h->d_trouble);
  (void)hipFree(h->d_tlist);
  (void)hipFree(h->d_ntrouble);
  delete h;
}

}  // extern "C"
