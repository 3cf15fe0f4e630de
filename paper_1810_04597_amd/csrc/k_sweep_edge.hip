// Face sweeps and constrained-transport edge fields (gfx950).
//
// k_sweep<DIR>: one thread per DIR-face, faces f in [-3, n_DIR + 1] over the
// whole ghosted transverse range, flattened with x^1 fastest so a wavefront
// reads 64 consecutive x^1 cells (coalesced).  Per face: MP5 left/right
// states of rho, p, u^1..3 and the two transverse centred B (paper,
// Introduction: high-order reconstruction), normal B from the face field,
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
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)ext[0] * ext[1] * ext[2];
  if (t >= total) return;
  int ii[3];
  ii[0] = (int)(t % ext[0]);
  const long r = t / ext[0];
  ii[1] = (int)(r % ext[1]);
  ii[2] = (int)(r / ext[1]);
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

  PState<T> sl, sr;
  {
    T q[6];
    auto rec = [&](int f, T& l, T& rr) {
      const double* p = prim + (long)f * G.field + c;
#pragma unroll
      for (int s = 0; s < 6; ++s) q[s] = T(p[(s - 2) * st]);
      mp5_lr(q, l, rr);
    };
    // a non-positive rho or p state falls back to the cell on its side
    rec(P_RHO, sl.rho, sr.rho);
    if (sl.rho <= T(0)) sl.rho = q[2];
    if (sr.rho <= T(0)) sr.rho = q[3];
    rec(P_P, sl.p, sr.p);
    if (sl.p <= T(0)) sl.p = q[2];
    if (sr.p <= T(0)) sr.p = q[3];
    rec(P_U1, sl.u[0], sr.u[0]);
    rec(P_U2, sl.u[1], sr.u[1]);
    rec(P_U3, sl.u[2], sr.u[2]);
    rec(P_B1 + T1, sl.B[T1], sr.B[T1]);
    rec(P_B1 + T2, sl.B[T2], sr.B[T2]);
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
  sl.B[DIR] = bn;
  sr.B[DIR] = bn;
  make_state(sl, m, gam);
  make_state(sr, m, gam);
  T fl[5], fr[5], ul[5], ur[5];
  flux_of(sl, m, DIR, fl);
  flux_of(sr, m, DIR, fr);
  cons_of(sl, m, ul);
  cons_of(sr, m, ur);
  T lpl, lml, lpr, lmr;
  speeds_of(sl, m, DIR, gam, lpl, lml);
  speeds_of(sr, m, DIR, gam, lpr, lmr);
  const T ap = fmax(T(0), fmax(lpl, lpr));
  const T am = fmax(T(0), fmax(-lml, -lmr));
  const T s = ap + am;
  const bool tiny = s < tiny_speed<T>();
  const T inv_s = tiny ? T(0) : T(1) / s;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    T fh = hll(fl[q], fr[q], ul[q], ur[q], ap, am, inv_s, tiny);
    if (axis) fh = T(0);
    flux[(long)q * G.field + c] = double(fh);
  }
  ctd[0 * G.field + c] = double(sl.v[DIR]);
  ctd[1 * G.field + c] = double(sr.v[DIR]);
  ctd[2 * G.field + c] = double(sl.v[T1]);
  ctd[3 * G.field + c] = double(sr.v[T1]);
  ctd[4 * G.field + c] = double(ap);
  ctd[5 * G.field + c] = double(am);
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
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)ext[0] * ext[1] * ext[2];
  if (t >= total) return;
  int ii[3];
  ii[0] = (int)(t % ext[0]);
  const long r = t / ext[0];
  ii[1] = (int)(r % ext[1]);
  ii[2] = (int)(r / ext[1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) ii[a] += (a == E) ? 0 : -3;
  const long b = G.idx(ii[0], ii[1], ii[2]);
  const long sd = G.stride(D), sc = G.stride(C);

  T q[6];
  // d-face quantities reconstructed along c (side b of the edge)
  auto along_c = [&](const double* __restrict__ src, T& l, T& rr) {
#pragma unroll
    for (int s = 0; s < 6; ++s) q[s] = T(src[b + (s - 2) * sc]);
    mp5_lr(q, l, rr);
  };
  T vd[2][2], vc[2][2], bd[2], bc[2];   // [a][b]
  along_c(ctd_d + 0 * G.field, vd[0][0], vd[0][1]);
  along_c(ctd_d + 1 * G.field, vd[1][0], vd[1][1]);
  along_c(ctd_d + 2 * G.field, vc[0][0], vc[0][1]);
  along_c(ctd_d + 3 * G.field, vc[1][0], vc[1][1]);
  along_c(cons + (long)(C_BF1 + D) * G.field, bd[0], bd[1]);
  {
    const double* src = cons + (long)(C_BF1 + C) * G.field;
#pragma unroll
    for (int s = 0; s < 6; ++s) q[s] = T(src[b + (s - 2) * sd]);
    mp5_lr(q, bc[0], bc[1]);
  }
  const T apd = fmax(T(ctd_d[4 * G.field + b]), T(ctd_d[4 * G.field + b + sc]));
  const T amd = fmax(T(ctd_d[5 * G.field + b]), T(ctd_d[5 * G.field + b + sc]));
  const T apc = fmax(T(ctd_c[4 * G.field + b]), T(ctd_c[4 * G.field + b + sd]));
  const T amc = fmax(T(ctd_c[5 * G.field + b]), T(ctd_c[5 * G.field + b + sd]));

  MET m;
  if constexpr (!MET::flat) {
    // x^3 edges -> E3 tables, x^1 edges (i, j+1/2, k+1/2) -> F2, x^2 edges -> F1
    constexpr int loc = E == 2 ? LOC_E3 : (E == 0 ? LOC_F2 : LOC_F1);
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }
  const T sdd = apd + amd, scc = apc + amc;
  const bool tiny_d = sdd < tiny_speed<T>(), tiny_c = scc < tiny_speed<T>();
  const T isd = tiny_d ? T(0) : T(1) / sdd;
  const T isc = tiny_c ? T(0) : T(1) / scc;
  const T wd[2] = {tiny_d ? T(0.5) : apd * isd, tiny_d ? T(0.5) : amd * isd};
  const T wc[2] = {tiny_c ? T(0.5) : apc * isc, tiny_c ? T(0.5) : amc * isc};
  const T kd = tiny_d ? T(0) : apd * amd * isd;
  const T kc = tiny_c ? T(0) : apc * amc * isc;
  T ee = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const T vtd = m.tvel(vd[a][bb], D);
      const T vtc = m.tvel(vc[a][bb], C);
      const T eab = vtc * bd[bb] - vtd * bc[a];
      ee = ee + wd[a] * wc[bb] * eab;
    }
  }
  ee = ee + kd * (bc[1] - bc[0]) - kc * (bd[1] - bd[0]);
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
