// Face sweeps and constrained-transport edge fields (gfx950).
//
// k_sweep<DIR>: one thread per DIR-face, faces f in [-3, n_DIR + 1] over the
// whole ghosted transverse range, flattened with x^1 fastest so a wavefront
// reads 64 consecutive x^1 cells (coalesced).  Per face: MP5 left/right
// states of rho, p, u^1..3 and the two transverse centred B (paper,
// Introduction: high-order reconstruction; rho and p bounded below by 0.1 of
// the cell value on their side), normal B from the face field,
// pointwise state, fluxes, conserved variables and fast speeds of both
// states, HLL flux (0 where sqrt(gamma) = 0, the polar axis).  Writes the
// five hydro fluxes and the six per-face quantities the edge field needs
// (v^d and v^c of both states, a+ and a-), c = d+1 mod 3.
//
// k_edge<E>: one thread per edge of family E (offsets 1/2 in d = E+1 and
// c = E+2 mod 3), over d, c in [-3, n + 1] and interior x^E: upwind
// constrained transport (Londrillo & Del Zanna 2004) from MP5 along c of the
// d-face velocities and B^d, MP5 along d of B^c, and the speeds of the two
// adjacent faces of each family.
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"

namespace grmhd {

template <int DIR, class MET, typename T>
__global__ __launch_bounds__(256) void k_sweep(Geom G, const double* __restrict__ prim,
                                               const double* __restrict__ cons,
                                               const double* __restrict__ tab,
                                               double* __restrict__ flux,
                                               double* __restrict__ ctd) {
  int ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ext[a] = (a == DIR) ? G.n[a] + 5 : G.dims[a];
  const long t = flat_thread();
  const long total = (long)ext[0] * ext[1] * ext[2];
  if (t >= total) return;
  // traversal order: x^1 fastest; for the x^3 sweep x^3 comes next, so the
  // six planes of a stencil are read by neighbouring workgroups (L2 reuse)
  constexpr int MID = DIR == 2 ? 2 : 1, SLOW = DIR == 2 ? 1 : 2;
  int ii[3];
  ii[0] = (int)(t % ext[0]);
  const long r = t / ext[0];
  ii[MID] = (int)(r % ext[MID]);
  ii[SLOW] = (int)(r / ext[MID]);
#pragma unroll
  for (int a = 0; a < 3; ++a) ii[a] += (a == DIR) ? -3 : -NG;
  const long c = G.idx(ii[0], ii[1], ii[2]);
  const long st = G.stride(DIR);
  const T gam = T(G.gam);
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;

  // face metric: x^1 faces -> F1, x^2 faces -> F2, x^3 faces -> centre tables
  MET m;
  if constexpr (!MET::flat) {
    constexpr int loc = DIR == 0 ? LOC_F1 : (DIR == 1 ? LOC_F2 : LOC_C);
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }

  T q[7][6];
  {
    const int fields[7] = {P_RHO, P_P, P_U1, P_U2, P_U3, P_B1 + T1, P_B1 + T2};
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const double* p = prim + (long)fields[v] * G.field + c;
#pragma unroll
      for (int s = 0; s < 6; ++s) q[v][s] = T(p[(s - 2) * st]);
    }
  }
  const double bface = cons[(long)(C_BF1 + DIR) * G.field + c];
  T bn;
  bool axis = false;
  if constexpr (MET::flat) {
    bn = T(bface);
  } else {
    axis = (m.sg == T(0));
    bn = axis ? T(0) : T(bface) / m.sg;
  }
  T fh[5], cd[6];
  face_body<DIR>(q, bn, axis, m, gam, fh, cd);
#pragma unroll
  for (int q5 = 0; q5 < 5; ++q5) flux[(long)q5 * G.field + c] = double(fh[q5]);
#pragma unroll
  for (int q6 = 0; q6 < 6; ++q6) ctd[(long)q6 * G.field + c] = double(cd[q6]);
}

// Edge field of family E.  ctd_d / ctd_c: per-face data of the d and c sweeps.
template <int E, class MET, typename T>
__global__ __launch_bounds__(256) void k_edge(Geom G, const double* __restrict__ cons,
                                              const double* __restrict__ tab,
                                              const double* __restrict__ ctd_d,
                                              const double* __restrict__ ctd_c,
                                              double* __restrict__ edge) {
  constexpr int D = (E + 1) % 3, C = (E + 2) % 3;
  int ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ext[a] = (a == E) ? G.n[a] : G.n[a] + 5;
  const long t = flat_thread();
  const long total = (long)ext[0] * ext[1] * ext[2];
  if (t >= total) return;
  // families 1 and 2 reconstruct along x^3: traverse x^3 before x^2
  constexpr int MID = E == 2 ? 1 : 2, SLOW = E == 2 ? 2 : 1;
  int ii[3];
  ii[0] = (int)(t % ext[0]);
  const long r = t / ext[0];
  ii[MID] = (int)(r % ext[MID]);
  ii[SLOW] = (int)(r / ext[MID]);
#pragma unroll
  for (int a = 0; a < 3; ++a) ii[a] += (a == E) ? 0 : -3;
  const long b = G.idx(ii[0], ii[1], ii[2]);
  const long sd = G.stride(D), sc = G.stride(C);

  T qd[5][6], qc[6];
  {
    const double* src[5] = {ctd_d, ctd_d + G.field, ctd_d + 2 * G.field, ctd_d + 3 * G.field,
                            cons + (long)(C_BF1 + D) * G.field};
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int s = 0; s < 6; ++s) qd[v][s] = T(src[v][b + (s - 2) * sc]);
    const double* bcs = cons + (long)(C_BF1 + C) * G.field;
#pragma unroll
    for (int s = 0; s < 6; ++s) qc[s] = T(bcs[b + (s - 2) * sd]);
  }
  MET m;
  if constexpr (!MET::flat) {
    // x^3 edges -> E3 tables, x^1 edges (i, j+1/2, k+1/2) -> F2, x^2 edges -> F1
    constexpr int loc = E == 2 ? LOC_E3 : (E == 0 ? LOC_F2 : LOC_F1);
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }
  const T ee = edge_body<E>(qd, qc, T(ctd_d[4 * G.field + b]), T(ctd_d[4 * G.field + b + sc]),
                            T(ctd_d[5 * G.field + b]), T(ctd_d[5 * G.field + b + sc]),
                            T(ctd_c[4 * G.field + b]), T(ctd_c[4 * G.field + b + sd]),
                            T(ctd_c[5 * G.field + b]), T(ctd_c[5 * G.field + b + sd]), m);
  edge[b] = double(ee);
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblocks(long total) { return (unsigned)((total + 255) / 256); }

template <class MET, typename T>
static void launch_sweep_t(int d, const Geom& G, const double* prim, const double* cons,
                           const double* tab, double* flux, double* ctd, hipStream_t s) {
  long total = 1;
  for (int a = 0; a < 3; ++a) total *= (a == d) ? G.n[a] + 5 : G.dims[a];
  double* fl = flux + (long)d * 5 * G.field;
  double* cd = ctd + (long)d * 6 * G.field;
  if (d == 0) hipLaunchKernelGGL((k_sweep<0, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, prim, cons, tab, fl, cd);
  if (d == 1) hipLaunchKernelGGL((k_sweep<1, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, prim, cons, tab, fl, cd);
  if (d == 2) hipLaunchKernelGGL((k_sweep<2, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, prim, cons, tab, fl, cd);
}

template <class MET, typename T>
static void launch_edge_t(int e, const Geom& G, const double* cons, const double* tab,
                          const double* ctd, double* edges, hipStream_t s) {
  long total = 1;
  for (int a = 0; a < 3; ++a) total *= (a == e) ? G.n[a] : G.n[a] + 5;
  const int d = (e + 1) % 3, c = (e + 2) % 3;
  const double* cd = ctd + (long)d * 6 * G.field;
  const double* cc = ctd + (long)c * 6 * G.field;
  double* ed = edges + (long)e * G.field;
  if (e == 0) hipLaunchKernelGGL((k_edge<0, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, cons, tab, cd, cc, ed);
  if (e == 1) hipLaunchKernelGGL((k_edge<1, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, cons, tab, cd, cc, ed);
  if (e == 2) hipLaunchKernelGGL((k_edge<2, MET, T>), dim3(nblocks(total)), dim3(256), 0, s, G, cons, tab, cd, cc, ed);
}

void launch_sweep(int d, const Geom& G, bool flat, bool fp32, const double* prim, const double* cons,
                  const double* tab, double* flux, double* ctd, hipStream_t s) {
  if (flat && !fp32) launch_sweep_t<FlatMet<double>, double>(d, G, prim, cons, tab, flux, ctd, s);
  if (flat && fp32) launch_sweep_t<FlatMet<float>, float>(d, G, prim, cons, tab, flux, ctd, s);
  if (!flat && !fp32) launch_sweep_t<TabMet<double>, double>(d, G, prim, cons, tab, flux, ctd, s);
  if (!flat && fp32) launch_sweep_t<TabMet<float>, float>(d, G, prim, cons, tab, flux, ctd, s);
}

void launch_edge(int e, const Geom& G, bool flat, bool fp32, const double* cons, const double* tab,
                 const double* ctd, double* edges, hipStream_t s) {
  if (flat && !fp32) launch_edge_t<FlatMet<double>, double>(e, G, cons, tab, ctd, edges, s);
  if (flat && fp32) launch_edge_t<FlatMet<float>, float>(e, G, cons, tab, ctd, edges, s);
  if (!flat && !fp32) launch_edge_t<TabMet<double>, double>(e, G, cons, tab, ctd, edges, s);
  if (!flat && fp32) launch_edge_t<TabMet<float>, float>(e, G, cons, tab, ctd, edges, s);
}

}  // namespace grmhd
