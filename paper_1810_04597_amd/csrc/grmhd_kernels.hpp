// Host-side launchers of the GRMHD kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include "grmhd_device.hpp"

namespace grmhd {

// Parameters of the inversion and floors.
struct C2PParams {
  double tol;
  int maxit;
  int guess;            // 0 warm, 1 cold, 2 learned
  int coord;            // 0 Cartesian, 1 log-spherical (r = exp(x^1))
  double rho_fl_a, rho_fl_n, p_fl_a, p_fl_n, w_max;
  double defer_tol;     // learned guess: relative warm residual above which a zone is deferred
  int img;              // all directions periodic, n >= 2 ng: also write the ghost images
  int split_it;         // > 0: defer zones not converged after this many iterations to a second pass
  // nullable: counters accumulated over every inversion (RUN_SLOTS slots of
  // RUN_STRIDE words, RUN_NCOUNT used)
  unsigned long long* run_acc;
  int defer_all;        // learned guess: every zone goes to the network pass
  int learned_only;     // learned guess: the network's start alone (warm start as fallback)
};

// Accumulated inversion counters: a block adds its non-zero counts to slot
// (block mod RUN_SLOTS) so that concurrent blocks rarely hit one address;
// each slot sits on its own 128-byte line.  The host sums the slots.
// Counters: failed zones, rho floors, p floors, W caps, zones inverted in the
// learned-guess pass, zones started from the network's guess, learned starts
// rerun from the warm guess, zones taken by the lower-order fallback.
constexpr int RUN_NCOUNT = 8;
constexpr int RUN_TROUBLED = 7;
constexpr int RUN_SLOTS = 64;
constexpr int RUN_STRIDE = 16;

// Per-block partial results of the inversion (reduced on the device).
constexpr int C2P_NSTAT = 8;   // fail, iters_sum, iters_max, floor_rho, floor_p, wcap, learned fallback, learned chosen
// Workgroups of the learned-guess pass over the deferred zones; its per-block
// partials follow the inversion's nblk partials.
constexpr int C2P_LIST_BLOCKS = 512;
constexpr int DIAG_NSUM = 8;   // plain sums of the 8 conserved fields
constexpr int DIAG_NMAX = 8;   // max|divB|, -rho_min, rho_max, -p_min, p_max, w_max, max|B|, nonfinite

struct BCSpec {
  int bc[6];
};

void launch_bc_centred(const Geom& G, const BCSpec& bc, double* prim, int nfields, hipStream_t s);
void launch_bc_faces(const Geom& G, const BCSpec& bc, double* cons, hipStream_t s);
// recon: RECON_MP5 | RECON_WENO5 | RECON_PLM | RECON_MP7 (grmhd_device.hpp)
void launch_sweep(int d, const Geom& G, bool flat, bool fp32, int recon, const double* prim,
                  const double* cons, const double* tab, double* flux, double* ctd, hipStream_t s);
void launch_edge(int e, const Geom& G, bool flat, bool fp32, int recon, const double* cons,
                 const double* tab, const double* ctd, double* edges, hipStream_t s);
// mode 0: SSP-RK3 stage `stage` (1, 2, 3) over the distinct buffers x, y
// (stage 1: x = U^n -> y; stage 2: x updated in place, U^n read from y;
// stage 3: x -> y, overwriting U^n); dt from d_dt when dt_host <= 0.
// mode 1: write L of the state in x into out (cons layout).
// img (flat metric, mode 0): all directions periodic with n >= 2 ng; the new
// face fields are also written to their ghost images (no separate face fill).
// fp32: flux and edges hold float fields (the FP32 form's storage), read at
// the same element offsets.
// parts (mode 0): UPD_ALL, or the hydro fields alone (UPD_HYDRO, which with
// fb also writes the fallback's flag per interior zone, 1 where the new state
// is unphysical, and counts those zones into fb->count) or the face fields
// alone (UPD_INDUCTION, with the ghost images when img).
enum { UPD_HYDRO = 1, UPD_INDUCTION = 2, UPD_ALL = 3 };
struct UpdateFallback {
  unsigned char* flags;   // n1 n2 n3 bytes, x^1 fastest
  int* list;              // n1 n2 n3 ints: the flagged zones (any order)
  int* count;             // their number; zeroed before the launch
};
void launch_update(const Geom& G, bool flat, bool fp32, int mode, const double* prim, double* x, double* y,
                   const double* flux, const double* edges, const double* tab, double a, double b,
                   double dt_host, const double* d_dt, double* out, int stage, hipStream_t s,
                   int img = 0, int parts = UPD_ALL, const UpdateFallback* fb = nullptr);
// Lower-order fallback of one stage (after the UPD_HYDRO update, before the
// UPD_INDUCTION one), two launches.  (1) Over the listed zones' faces (a
// fixed grid walking 6 count items): (F1 - G) of the five hydro fields at
// each face of a flagged zone, written to `delta` (15 face fields, the
// layout of the fluxes; each face once, and at its periodic image when it
// lies on a periodic boundary), F1 the first-order HLL flux from the
// primitives of the two cells and the face field in `cur`, G the corrected
// flux of the stored face fluxes.  (2) Each interior zone with a flagged
// zone on either side of one of its faces (periodic directions wrap;
// elsewhere zones outside count as unflagged) subtracts b dt times the
// difference of those faces' deltas over the cell from its new hydro state
// in `next`.  Both exit at once when count is 0; the second adds count to
// the accumulated counters (run_acc, nullable).
void launch_fallback(const Geom& G, bool flat, bool fp32, const BCSpec& bc, const double* prim,
                     const double* cur, double* next, const double* flux, const double* tab,
                     const unsigned char* flags, const int* list, const int* count, double* delta,
                     double b, double dt_host, const double* d_dt, unsigned long long* run_acc,
                     hipStream_t s);
// The face field normal to each non-periodic direction at the ghost faces
// the staggered derivative of an interior cell reads (-flo .. -1 and
// n .. n + flo - 2, interior in the other directions): the RK stage of the
// induction equation into x / y as launch_update (mode 0) does at the owned
// faces, after it; or the curl of the edge potentials into cons (after
// launch_curl).  The face ghost fill leaves these faces alone.
void launch_ghost_normal_update(const Geom& G, const BCSpec& bc, bool fp32, double* x, double* y,
                                const double* edges, double a, double b, double dt_host, const double* d_dt,
                                int stage, hipStream_t s);
void launch_ghost_normal_curl(const Geom& G, const BCSpec& bc, const double* a1, const double* a2,
                              const double* a3, double* cons, hipStream_t s);
void launch_advance(double* d_dt, const double* src, double dt_host, hipStream_t s);
// Inversion of all interior zones; per-block counters into partials[0, nblk),
// CFL partials (nullable) into cfl_partials[0, nblk).  list != nullptr: defer
// zones with a poor warm start into list / list_n (learned guess).
// list / list_n: zones deferred by the learned-guess residual test or by
// cp.split_it (appended in any order); list_y: their last iterates (split).
void launch_c2p(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                const double* tab, long long* partials, double* cfl_partials, int* list, int* list_n,
                double* list_y, hipStream_t s);
// Second pass of a split inversion: the listed zones, each from its stored
// iterate, C2P_LIST_BLOCKS workgroups (partials at their block index).
void launch_c2p_split(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                      const double* tab, const int* list, const int* list_n, const double* list_y,
                      long long* partials, double* cfl_partials, hipStream_t s);
void launch_zero_int(int* p, hipStream_t s);
void launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// Shell fluxes through x^1 = const: out[4 n1] = F_D, F_tau, Phi (|B|/2), Phi
// signed; part: shell_part_doubles(G) doubles of chunk partials.
void launch_shell(const Geom& G, bool flat, const double* prim, const double* cons, const double* tab,
                  double* part, double* out, hipStream_t s);
long shell_part_doubles(const Geom& G);
// MRI resolution sums per x^1 shell (6 n1 doubles into out; part holds
// mri_part_doubles(G) chunk partials).
void launch_mri(const Geom& G, bool flat, const double* prim, const double* tab, double rho_cut,
                double q_min, double* part, double* out, hipStream_t s);
long mri_part_doubles(const Geom& G);
void launch_dt_final(const double* cfl_partials, int nb, double cfl, double* d_dt, hipStream_t s);
void launch_prim2cons(const Geom& G, bool flat, double* prim, double* cons, const double* tab,
                      hipStream_t s);
void launch_cfl(const Geom& G, bool flat, const double* prim, const double* tab, double cfl,
                double* partials, double* d_dt, hipStream_t s);
void launch_curl(const Geom& G, const double* a1, const double* a2, const double* a3,
                 double* cons, hipStream_t s);
void launch_reduce_stats(const long long* partials, int nblk, long long* out, hipStream_t s);
void launch_diag(const Geom& G, bool flat, const double* prim, const double* cons,
                 const double* tab, double* partials, double* out, hipStream_t s);
unsigned zone_blocks(const Geom& G);

}  // namespace grmhd
