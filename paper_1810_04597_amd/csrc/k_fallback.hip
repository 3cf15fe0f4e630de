// Lower-order fallback at troubled zones (gfx950).
//
// Paper, Introduction: the scheme family carries reconstruction algorithms
// of several orders; here the first-order member (the cell values
// themselves, with the same HLL solver) serves as a fallback, applied after
// a stage's update where the high-order update left a hydro state that no
// physical primitives can give (D <= 0, tau <= 0 or S^2 >= (tau + D)^2; the
// update kernel flags those zones).
//
// The high-order update differences face values: the staggered derivative
// of the face fluxes f equals the difference, over the cell, of the
// corrected face flux G = f - Delta^2 f / 24 + 3 Delta^4 f / 640 (its first
// correction alone for the fourth-order derivative), the flux form of the
// scheme.  At every face of a troubled zone the stage's G is replaced by the
// first-order HLL flux F1 of the two cells beside it, in both zones: the new
// state of a zone changes by -b dt sum_d [(F1 - G)_{+1/2} - (F1 - G)_{-1/2}]
// / Delta_d over its replaced faces, so the step stays conservative.
//
// Two launches.  The update lists the troubled zones; a fixed grid walks
// the six faces of each listed zone (face-major, so a wavefront mostly takes
// one direction) and writes (F1 - G) of each face once to face fields laid
// out like the fluxes (a face shared by two troubled zones is written by the
// lower one; a face on a periodic boundary also at its image, so both zones
// beside it read the one value and the step stays conservative).  Then one
// thread per interior zone gathers the values of its replaced faces, so no
// two threads write one value.  When no zone is troubled (the usual case)
// both exit after reading the count.
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"
#include "grmhd_c2p.hpp"

namespace grmhd {

// (F1 - G) of the five hydro fields at the DIR-face stored at (fi, fj, fk)
// (the face +1/2 of that cell): F1 from the primitives of cells (fi, fj, fk)
// and its DIR neighbour and the face field of the stage's start state cur;
// G from the stored face fluxes of faces -2 .. +2 around it (-1 .. +1 for the
// fourth-order form).
template <int DIR, class MET, typename FS, int DO>
__device__ __forceinline__ void face_delta(const Geom& G, const double* __restrict__ prim,
                                           const double* __restrict__ cur, const FS* __restrict__ flux,
                                           const double* __restrict__ tab, int fi, int fj, int fk,
                                           double* __restrict__ out) {
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  const long c = G.idx(fi, fj, fk);
  const long st = G.stride(DIR);
  MET m;
  if constexpr (!MET::flat) {
    constexpr int loc = DIR == 0 ? LOC_F1 : (DIR == 1 ? LOC_F2 : LOC_C);
    m.load(tab, G.tab_plane, loc, G.tidx(fi, fj));
  }
  const int fields[7] = {P_RHO, P_P, P_U1, P_U2, P_U3, P_B1 + T1, P_B1 + T2};
  auto qs = [&](int v, int s) { return prim[(long)fields[v] * G.field + c + s * st]; };
  const double bface = cur[(long)(C_BF1 + DIR) * G.field + c];
  bool axis = false;
  double bn = bface;
  if constexpr (!MET::flat) {
    axis = m.sg == 0.0;
    bn = axis ? 0.0 : bface / m.sg;
  }
  double fh[5], cd[6];
  face_body_q<DIR, RECON_PCM>(qs, bn, axis, m, G.gam, fh, cd);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const FS* fp = flux + ((long)DIR * 5 + q) * G.field + c;
    const double fm1 = fp[-st], f0 = fp[0], fp1 = fp[st];
    double g = f0 - (fp1 - 2.0 * f0 + fm1) / 24.0;
    if constexpr (DO == 6) {
      const double fm2 = fp[-2 * st], fp2 = fp[2 * st];
      g = g + 3.0 * (fp2 - 4.0 * fp1 + 6.0 * f0 - 4.0 * fm1 + fm2) / 640.0;
    }
    out[q] = fh[q] - g;
  }
}

// Whether interior zone w (w[d] may be one past either end) is flagged: a
// periodic direction wraps, elsewhere zones outside count as unflagged.
__device__ __forceinline__ bool flagged(const Geom& G, const BCSpec& bc, const unsigned char* __restrict__ flags,
                                        int w0, int w1, int w2) {
  int w[3] = {w0, w1, w2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (w[d] < 0 || w[d] >= G.n[d]) {
      if (bc.bc[2 * d] != 0) return false;   // not periodic (0)
      w[d] = w[d] < 0 ? w[d] + G.n[d] : w[d] - G.n[d];
    }
  }
  return flags[w[0] + (long)G.n[0] * (w[1] + (long)G.n[1] * w[2])] != 0;
}

// Workgroups of the face pass (a fixed grid; each thread walks items).
constexpr int FB_FACE_BLOCKS = 1024;

template <int DIR, class MET, typename FS, int DO>
__device__ __forceinline__ void store_face_delta(const Geom& G, const BCSpec& bc, const double* __restrict__ prim,
                                                 const double* __restrict__ cur, const FS* __restrict__ flux,
                                                 const double* __restrict__ tab, int f0, int f1, int f2,
                                                 double* __restrict__ delta) {
  double dl[5];
  face_delta<DIR, MET, FS, DO>(G, prim, cur, flux, tab, f0, f1, f2, dl);
  int f[3] = {f0, f1, f2};
  const long c = G.idx(f0, f1, f2);
#pragma unroll
  for (int q = 0; q < 5; ++q) delta[((long)DIR * 5 + q) * G.field + c] = dl[q];
  // the same face seen from the other side of a periodic boundary: stored at
  // -1 (face -1/2) and at n - 1 (face n - 1/2)
  if (bc.bc[2 * DIR] == 0 && (f[DIR] == -1 || f[DIR] == G.n[DIR] - 1)) {
    f[DIR] = f[DIR] == -1 ? G.n[DIR] - 1 : -1;
    const long ci = G.idx(f[0], f[1], f[2]);
#pragma unroll
    for (int q = 0; q < 5; ++q) delta[((long)DIR * 5 + q) * G.field + ci] = dl[q];
  }
}

template <class MET, typename FS, int DO>
__global__ __launch_bounds__(256) void k_fallback_faces(Geom G, BCSpec bc, const double* __restrict__ prim,
                                                        const double* __restrict__ cur,
                                                        const FS* __restrict__ flux,
                                                        const double* __restrict__ tab,
                                                        const unsigned char* __restrict__ flags,
                                                        const int* __restrict__ list,
                                                        const int* __restrict__ count,
                                                        double* __restrict__ delta) {
  const long nt = *count;
  if (nt == 0) return;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < 6 * nt; w += stride) {
    const int face = (int)(w / nt);           // direction face / 2; side face % 2 (0: -1/2, 1: +1/2)
    const int z = list[w - face * nt];
    int ijk[3];
    ijk[0] = z % G.n[0];
    ijk[1] = (z / G.n[0]) % G.n[1];
    ijk[2] = z / (G.n[0] * G.n[1]);
    const int d = face >> 1;
    if ((face & 1) == 0) {
      // the -1/2 face is stored at the lower neighbour, which writes it
      // itself (as its +1/2 face) when it is flagged too
      int nb[3] = {ijk[0], ijk[1], ijk[2]};
      nb[d] -= 1;
      if (flagged(G, bc, flags, nb[0], nb[1], nb[2])) continue;
      ijk[d] -= 1;
    }
    if (d == 0) store_face_delta<0, MET, FS, DO>(G, bc, prim, cur, flux, tab, ijk[0], ijk[1], ijk[2], delta);
    else if (d == 1) store_face_delta<1, MET, FS, DO>(G, bc, prim, cur, flux, tab, ijk[0], ijk[1], ijk[2], delta);
    else store_face_delta<2, MET, FS, DO>(G, bc, prim, cur, flux, tab, ijk[0], ijk[1], ijk[2], delta);
  }
}

// The corrections of direction DIR at zone c: faces -1/2 (stored at the DIR
// neighbour below) where lo, +1/2 where hi.
template <int DIR>
__device__ __forceinline__ void correct_dir(const Geom& G, const double* __restrict__ delta, long c, bool lo,
                                            bool hi, double bdt, double v[5]) {
  if (!lo && !hi) return;
  double dlo[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, dhi[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const long st = G.stride(DIR);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double* f = delta + ((long)DIR * 5 + q) * G.field + c;
    if (lo) dlo[q] = f[-st];
    if (hi) dhi[q] = f[0];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = v[q] - bdt * (dhi[q] - dlo[q]) / G.dx[DIR];
}

__global__ __launch_bounds__(256) void k_fallback(Geom G, BCSpec bc, double* __restrict__ next,
                                                  const double* __restrict__ delta,
                                                  const unsigned char* __restrict__ flags,
                                                  const int* __restrict__ count, double b,
                                                  double dt_host, const double* __restrict__ d_dt,
                                                  unsigned long long* __restrict__ run_acc) {
  const int nt = *count;
  if (blockIdx.x == 0 && threadIdx.x == 0 && run_acc != nullptr && nt > 0)
    atomicAdd(run_acc + RUN_TROUBLED, (unsigned long long)nt);
  if (nt == 0) return;
  const long t = flat_thread();
  if (t >= (long)G.n[0] * G.n[1] * G.n[2]) return;
  int i, j, k;
  zone_of(G, t, i, j, k);
  const bool self = flags[t] != 0;
  bool lo[3], hi[3];
  bool any = self;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = self || flagged(G, bc, flags, i - (d == 0), j - (d == 1), k - (d == 2));
    hi[d] = self || flagged(G, bc, flags, i + (d == 0), j + (d == 1), k + (d == 2));
    any = any || lo[d] || hi[d];
  }
  if (!any) return;
  const long c = G.idx(i, j, k);
  const double bdt = b * (dt_host > 0.0 ? dt_host : *d_dt);
  double v[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = next[(long)q * G.field + c];
  correct_dir<0>(G, delta, c, lo[0], hi[0], bdt, v);
  correct_dir<1>(G, delta, c, lo[1], hi[1], bdt, v);
  correct_dir<2>(G, delta, c, lo[2], hi[2], bdt, v);
#pragma unroll
  for (int q = 0; q < 5; ++q) next[(long)q * G.field + c] = v[q];
}

template <class MET, typename FS>
static void launch_faces_m(const Geom& G, const BCSpec& bc, const double* prim, const double* cur,
                           const FS* flux, const double* tab, const unsigned char* flags, const int* list,
                           const int* count, double* delta, hipStream_t s) {
  if (G.dorder == 4)
    hipLaunchKernelGGL((k_fallback_faces<MET, FS, 4>), dim3(FB_FACE_BLOCKS), dim3(256), 0, s, G, bc, prim, cur,
                       flux, tab, flags, list, count, delta);
  else
    hipLaunchKernelGGL((k_fallback_faces<MET, FS, 6>), dim3(FB_FACE_BLOCKS), dim3(256), 0, s, G, bc, prim, cur,
                       flux, tab, flags, list, count, delta);
}

void launch_fallback(const Geom& G, bool flat, bool fp32, const BCSpec& bc, const double* prim,
                     const double* cur, double* next, const double* flux, const double* tab,
                     const unsigned char* flags, const int* list, const int* count, double* delta,
                     double b, double dt_host, const double* d_dt, unsigned long long* run_acc,
                     hipStream_t s) {
  const float* ff = reinterpret_cast<const float*>(flux);
  if (flat && fp32)
    launch_faces_m<FlatMet<double>, float>(G, bc, prim, cur, ff, tab, flags, list, count, delta, s);
  else if (flat)
    launch_faces_m<FlatMet<double>, double>(G, bc, prim, cur, flux, tab, flags, list, count, delta, s);
  else if (fp32)
    launch_faces_m<TabMet<double>, float>(G, bc, prim, cur, ff, tab, flags, list, count, delta, s);
  else
    launch_faces_m<TabMet<double>, double>(G, bc, prim, cur, flux, tab, flags, list, count, delta, s);
  hipLaunchKernelGGL(k_fallback, dim3(zone_blocks(G)), dim3(256), 0, s, G, bc, next, delta, flags, count, b,
                     dt_host, d_dt, run_acc);
}

}  // namespace grmhd
