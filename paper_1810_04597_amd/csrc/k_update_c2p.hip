// Cell-centred kernels: RK stage update with metric sources, conservative-to-
// primitive inversion with floors, prim->cons, CFL step, curl of a potential,
// ghost fill and deterministic reductions (gfx950).
//
// Method references (paper, Introduction: GRMHD with 3-D finite differences
// after ECHO; standard published forms):
//   update : L = -sum_d D_d F_d + s, SSP-RK3 stage a U^n + b (U + dt L)
//            (Shu & Osher 1988); induction -curl_D E on the owned faces;
//   sources: stationary-metric 3+1 sources
//            s[S_i] = sqrt(g) (alpha W^jk d_i g_jk / 2 + S_j d_i beta^j - U d_i alpha),
//            s[tau] = sqrt(g) (W^jk beta^l d_l g_jk / 2 + W^j_k d_j beta^k - S^j d_j alpha);
//   c2p    : safeguarded 1-D Newton in y = rho h W^2 on (0, Gamma U], bisection
//            when a step leaves the bracket or v^2 >= 1, stop at a round-off
//            residual or |dy| <= tol y; failed zones keep their primitives.
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"
#include "grmhd_c2p.hpp"

namespace grmhd {

static inline unsigned nblk(long total) { return (unsigned)((total + 255) / 256); }

// ------------------------------------------------------------------ block reductions
// ------------------------------------------------------------------ metric sources
template <class MET>
__device__ __forceinline__ void sources_of(const PState<double>& s, const MET& m,
                                           const double* __restrict__ tab, long tplane, long tt,
                                           double src[5]) {
  const double* dp = tab + (long)DER_BASE * tplane + tt;
  auto der = [&](int q) { return dp[(long)q * tplane]; };
  // electric field, both index positions
  double el[3], eu[3];
  el[0] = m.e_lo(-(s.v[1] * s.B[2] - s.v[2] * s.B[1]));
  el[1] = m.e_lo(-(s.v[2] * s.B[0] - s.v[0] * s.B[2]));
  el[2] = m.e_lo(-(s.v[0] * s.B[1] - s.v[1] * s.B[0]));
  eu[0] = m.e_up(-(s.vl[1] * s.Bl[2] - s.vl[2] * s.Bl[1]));
  eu[1] = m.e_up(-(s.vl[2] * s.Bl[0] - s.vl[0] * s.Bl[2]));
  eu[2] = m.e_up(-(s.vl[0] * s.Bl[1] - s.vl[1] * s.Bl[0]));
  const double ptot = s.p + 0.5 * (s.E2 + s.B2);
  // W^jk and d_i gamma_jk are symmetric: the sum over j, k is the sum over
  // j <= k with the off-diagonal terms doubled.  Each term is formed and
  // consumed at once (no 3x3 arrays held), which keeps the register count of
  // the update low.  a_i = sum_jk W^jk d_i gamma_jk for i = 1, 2.
  constexpr int JJ[6] = {0, 0, 0, 1, 1, 2}, KK[6] = {0, 1, 2, 1, 2, 2};   // 11,12,13,22,23,33
  const double gu[6] = {m.u11, m.u12, m.u13, m.u22, m.u23, m.u33};
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int j = JJ[q], k = KK[q];
    double w = s.y * s.v[j] * s.v[k] - eu[j] * eu[k] - s.B[j] * s.B[k] + ptot * gu[q];
    if (j != k) w = 2.0 * w;
    a0 = a0 + w * der(D1_G11 + q);
    a1 = a1 + w * der(D2_G11 + q);
  }
  const double utot = s.tau + s.D;
  src[0] = 0.0 * m.sg;
  src[3] = 0.0 * m.sg;
  {
    double t1 = 0.5 * m.al * a0, t2 = 0.5 * m.al * a1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      t1 = t1 + s.S[j] * der(D1_B1 + j);
      t2 = t2 + s.S[j] * der(D2_B1 + j);
    }
    src[1] = m.sg * (t1 - utot * der(D1_AL));
    src[2] = m.sg * (t2 - utot * der(D2_AL));
  }
  // energy: W^jk beta^l d_l gamma_jk / 2 + W^j_k d_j beta^k - S^j d_j alpha (l, j over the
  // two axisymmetric directions)
  double t = 0.5 * (m.b[0] * a0 + m.b[1] * a1);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double wm = s.y * s.v[j] * s.vl[k] - eu[j] * el[k] - s.B[j] * s.Bl[k] + (j == k ? ptot : 0.0);
      t = t + wm * der((j == 0 ? D1_B1 : D2_B1) + k);
    }
  for (int j = 0; j < 2; ++j) t = t - s.Su[j] * der(j == 0 ? D1_AL : D2_AL);
  src[4] = m.sg * t;
}

// ------------------------------------------------------------------ zone order
// Zone order of the one-thread-per-zone kernels that read x^3 stencils (the
// update on a tabulated metric reads F^3, E_1 and E_2 over planes k-3 .. k+2;
// the inversion's centred field reads the x^3 face field there).  In the
// plain order (x^1 fastest, then x^2, then x^3) the x^3 neighbours of a row
// are n_2 rows apart, more than one XCD's L2 holds, so those fields are
// fetched from HBM once per stencil point.  Here the (j, k) rows are walked
// in strips of S rows of x^2 with k advancing once per strip: x^3 neighbours
// are S rows apart, x^2 neighbours inside a strip 1-3 rows apart, and only
// the strip edges re-read x^2 rows.  A bijection on the interior zones (the
// last strip may be narrower).
template <int S>
__device__ __forceinline__ long strip_zone_order(const Geom& G, long t) {
  const long n0 = G.n[0];
  const long r = t / n0;                        // logical row
  const int i = (int)(t - r * n0);
  const long per = (long)S * G.n[2];            // rows in a full strip
  const int st = (int)(r / per);
  const int w = (int)(r - st * per);
  const int h = min(S, G.n[1] - st * S);
  const int k = w / h;
  const int j = st * S + (w - k * h);
  return i + n0 * (j + (long)G.n[1] * k);
}
constexpr int UPDATE_STRIP = 16;
constexpr int C2P_STRIP = 32;

// ------------------------------------------------------------------ RK update
// RK stage store over two distinct buffers x and y (SSP-RK3, Shu-Osher form,
// U^(s+1) = a U^n + b (U^(s) + dt L)), so that U^n is never copied:
//   stage 1 (a = 0): reads U^n from x, writes U^(1) to y;
//   stage 2: reads U^(1) from x and U^n from y, writes U^(2) to x;
//   stage 3: reads U^(2) from x and U^n from y, writes U^(3) to y.
// The caller's buffer holds U^n and receives U^(3); the other is scratch.
// Returns the stored value.  ST is a template argument so that a
// z-iteration of the update below is one basic block: the scheduler can then
// issue every field's stencil loads ahead of the earlier fields' stores.
template <int ST>
__device__ __forceinline__ double rk_store(double* __restrict__ x, double* __restrict__ y, long o,
                                           double a, double b, double dt, double L) {
  const double old = x[o];
  if constexpr (ST == 1) {
    const double v = b * (old + dt * L);   // a = 0
    y[o] = v;
    return v;
  } else {
    const double v = a * y[o] + b * (old + dt * L);
    if constexpr (ST == 2) x[o] = v; else y[o] = v;
    return v;
  }
}

__device__ __forceinline__ double rk_store_rt(double* __restrict__ x, double* __restrict__ y, long o,
                                              double a, double b, double dt, double L, int stage) {
  if (stage == 1) return rk_store<1>(x, y, o, a, b, dt, L);
  if (stage == 2) return rk_store<2>(x, y, o, a, b, dt, L);
  return rk_store<3>(x, y, o, a, b, dt, L);
}

// Troubled state of the lower-order fallback: the new (densitised) hydro
// state nv = (D, S_1..3, tau) has D <= 0, tau <= 0 or S^2 >= (tau + D)^2 (no
// physical primitives can give it); the comparisons are false for NaN.
template <class MET>
__device__ __forceinline__ bool troubled_state(const double nv[5], const MET& m) {
  const double dd = m.undens(nv[0]), tau = m.undens(nv[4]);
  const double sl[3] = {m.undens(nv[1]), m.undens(nv[2]), m.undens(nv[3])};
  double su[3];
  m.raise(sl, su);
  const double s2 = sl[0] * su[0] + sl[1] * su[1] + sl[2] * su[2];
  const double u = tau + dd;
  return dd <= 0.0 || tau <= 0.0 || s2 >= u * u;
}

// flags (nullable: then nothing is recorded): one byte per interior zone,
// x^1 fastest; the flagged zones' indices are appended to list, count holds
// their number.
__device__ __forceinline__ void flag_zone(const Geom& G, int i, int j, int k, bool bad,
                                          unsigned char* __restrict__ flags, int* __restrict__ list,
                                          int* __restrict__ count) {
  if (!flags) return;
  const int z = i + G.n[0] * (j + G.n[1] * k);
  flags[z] = bad ? 1 : 0;
  if (bad) list[atomicAdd(count, 1)] = z;
}

// FS: storage type of the fluxes and edge fields (double, or float in the
// FP32 form), widened to double on load.  PARTS: UPD_ALL, UPD_HYDRO (with the
// fallback's flags) or UPD_INDUCTION.
template <class MET, int DO, typename FS, int PARTS>
__global__ __launch_bounds__(256) void k_update(Geom G, int mode, const double* __restrict__ prim,
                                                double* __restrict__ x,
                                                double* __restrict__ y,
                                                const FS* __restrict__ flux,
                                                const FS* __restrict__ edges,
                                                const double* __restrict__ tab, double a, double b,
                                                double dt_host, const double* __restrict__ d_dt,
                                                double* __restrict__ out, int stage,
                                                unsigned char* __restrict__ tflags,
                                                int* __restrict__ tlist, int* __restrict__ tcount) {
  const long t = flat_thread();
  if (t >= (long)G.n[0] * G.n[1] * G.n[2]) return;
  int i, j, k;
  zone_of(G, strip_zone_order<UPDATE_STRIP>(G, t), i, j, k);
  const long c = G.idx(i, j, k);
  auto stage_dt = [&]() { return (mode != 0) ? 0.0 : (dt_host > 0.0 ? dt_host : *d_dt); };
  double dt = 0.0, f[6];
  if constexpr ((PARTS & UPD_HYDRO) != 0) {
    double src[5] = {0, 0, 0, 0, 0};
    if constexpr (!MET::flat) {
      const long tt = G.tidx(i, j);
      MET m;
      m.load(tab, G.tab_plane, LOC_C, tt);
      PState<double> s;
      s.rho = prim[P_RHO * G.field + c];
      s.p = prim[P_P * G.field + c];
      for (int q = 0; q < 3; ++q) {
        s.u[q] = prim[(P_U1 + q) * G.field + c];
        s.B[q] = prim[(P_B1 + q) * G.field + c];
      }
      make_state(s, m, G.gam);
      sources_of(s, m, tab, G.tab_plane, tt, src);
    }
    dt = stage_dt();
    double nv[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double L = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const FS* fp = flux + ((long)d * 5 + q) * G.field + c;
        const long st = G.stride(d);
#pragma unroll
        for (int s = 0; s < 6; ++s) f[s] = fp[(s - 3) * st];
        L = L - fd_deriv_o<DO>(f, 1.0 / G.dx[d]);
      }
      L = L + src[q];
      const long o = (long)q * G.field + c;
      if (mode == 0)
        nv[q] = rk_store_rt(x, y, o, a, b, dt, L, stage);
      else
        out[o] = L;
    }
    if constexpr (PARTS == UPD_HYDRO) {
      MET mc;
      if constexpr (!MET::flat) mc.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
      flag_zone(G, i, j, k, troubled_state(nv, mc), tflags, tlist, tcount);
    }
  }
  if constexpr ((PARTS & UPD_INDUCTION) != 0) {
    if constexpr ((PARTS & UPD_HYDRO) == 0) dt = stage_dt();
#pragma unroll
    for (int nd = 0; nd < 3; ++nd) {
      const int d1 = (nd + 1) % 3, d2 = (nd + 2) % 3;
      const FS* e2 = edges + (long)d2 * G.field + c;
      const FS* e1 = edges + (long)d1 * G.field + c;
      const long s1 = G.stride(d1), s2 = G.stride(d2);
#pragma unroll
      for (int s = 0; s < 6; ++s) f[s] = e2[(s - 3) * s1];
      const double t1 = fd_deriv_o<DO>(f, 1.0 / G.dx[d1]);
#pragma unroll
      for (int s = 0; s < 6; ++s) f[s] = e1[(s - 3) * s2];
      const double t2 = fd_deriv_o<DO>(f, 1.0 / G.dx[d2]);
      const double L = -t1 + t2;
      const long o = (long)(C_BF1 + nd) * G.field + c;
      if (mode == 0)
        rk_store_rt(x, y, o, a, b, dt, L, stage);
      else
        out[o] = L;
    }
  }
}


// z-marching variant (flat metric): one thread per (i, j) column segment of
// KZ zones along x^3.  The x^3 stencils (F of the x^3 sweep, E_1, E_2) are
// kept in register windows, so each of their planes is read once per
// segment instead of six times; x^1 and x^2 stencils are read per plane.
// PARTS as in k_update (the hydro and the induction parts read disjoint
// fields, so the split costs a launch, not bytes).
constexpr int KZ = 16;

template <class MET, int ST, int DO, typename FS, int PARTS>
__global__ __launch_bounds__(256) void k_update_zm(Geom G, const double* __restrict__ prim,
                                                   double* __restrict__ x,
                                                   double* __restrict__ y,
                                                   const FS* __restrict__ flux,
                                                   const FS* __restrict__ edges,
                                                   const double* __restrict__ tab, double a,
                                                   double b, double dt_host,
                                                   const double* __restrict__ d_dt, int img,
                                                   unsigned char* __restrict__ tflags,
                                                   int* __restrict__ tlist, int* __restrict__ tcount) {
  constexpr bool HYD = (PARTS & UPD_HYDRO) != 0, IND = (PARTS & UPD_INDUCTION) != 0;
  const long t = flat_thread();
  const int nseg = (G.n[2] + KZ - 1) / KZ;
  if (t >= (long)G.n[0] * G.n[1] * nseg) return;
  const int i = (int)(t % G.n[0]);
  const long r = t / G.n[0];
  const int j = (int)(r % G.n[1]);
  const int k0 = (int)(r / G.n[1]) * KZ;
  const int k1 = min(k0 + KZ, G.n[2]);
  const double dt = dt_host > 0.0 ? dt_host : *d_dt;
  const long sx = 1, sy = G.pitch, sz = G.plane;
  const double idx0 = 1.0 / G.dx[0], idx1 = 1.0 / G.dx[1], idx2 = 1.0 / G.dx[2];
  const FS* fz = flux + 2L * 5 * G.field;       // x^3-sweep fluxes
  const FS* e1 = edges;                         // E_1 (offsets in x^2, x^3)
  const FS* e2 = edges + G.field;               // E_2 (offsets in x^3, x^1)
  const FS* e3 = edges + 2 * G.field;           // E_3 (offsets in x^1, x^2)
  // windows along x^3: w[s] holds stored index k - 3 + s
  double wf[5][6], w1[6], w2[6];
  long c = G.idx(i, j, k0);
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const long cs = c + (s - 3) * sz;
    if constexpr (HYD) {
#pragma unroll
      for (int q = 0; q < 5; ++q) wf[q][s] = fz[(long)q * G.field + cs];
    }
    if constexpr (IND) {
      w1[s] = e1[cs];
      w2[s] = e2[cs];
    }
  }
  for (int k = k0; k < k1; ++k, c += sz) {
    const long cn = c + 2 * sz;
    if constexpr (HYD) {
#pragma unroll
      for (int q = 0; q < 5; ++q) wf[q][5] = fz[(long)q * G.field + cn];
    }
    if constexpr (IND) {
      w1[5] = e1[cn];
      w2[5] = e2[cn];
    }
    double f[6], bf[3];
    if constexpr (HYD) {
      double nv[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double L = 0.0;
        const FS* fx = flux + (long)q * G.field + c;
        const FS* fy = flux + (5L + q) * G.field + c;
#pragma unroll
        for (int s = 0; s < 6; ++s) f[s] = fx[(s - 3) * sx];
        L = L - fd_deriv_o<DO>(f, idx0);
#pragma unroll
        for (int s = 0; s < 6; ++s) f[s] = fy[(s - 3) * sy];
        L = L - fd_deriv_o<DO>(f, idx1);
        L = L - fd_deriv_o<DO>(wf[q], idx2);
        nv[q] = rk_store<ST>(x, y, (long)q * G.field + c, a, b, dt, L);
      }
      if constexpr (!IND) flag_zone(G, i, j, k, troubled_state(nv, MET()), tflags, tlist, tcount);
    }
    if constexpr (IND) {
      // B^1: -D_2 E_3 + D_3 E_2
      {
#pragma unroll
        for (int s = 0; s < 6; ++s) f[s] = e3[c + (s - 3) * sy];
        const double L = -fd_deriv_o<DO>(f, idx1) + fd_deriv_o<DO>(w2, idx2);
        bf[0] = rk_store<ST>(x, y, (long)C_BF1 * G.field + c, a, b, dt, L);
      }
      // B^2: -D_3 E_1 + D_1 E_3
      {
#pragma unroll
        for (int s = 0; s < 6; ++s) f[s] = e3[c + (s - 3) * sx];
        const double L = -fd_deriv_o<DO>(w1, idx2) + fd_deriv_o<DO>(f, idx0);
        bf[1] = rk_store<ST>(x, y, (long)C_BF2 * G.field + c, a, b, dt, L);
      }
      // B^3: -D_1 E_2 + D_2 E_1
      {
        double g2[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          f[s] = e2[c + (s - 3) * sx];
          g2[s] = e1[c + (s - 3) * sy];
        }
        const double L = -fd_deriv_o<DO>(f, idx0) + fd_deriv_o<DO>(g2, idx1);
        bf[2] = rk_store<ST>(x, y, (long)C_BF3 * G.field + c, a, b, dt, L);
      }
      if (img) {
        constexpr int ff[3] = {C_BF1, C_BF2, C_BF3};
        write_images<3>(G, ST == 2 ? x : y, i, j, k, ff, bf);
      }
    }
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      if constexpr (HYD) {
#pragma unroll
        for (int q = 0; q < 5; ++q) wf[q][s] = wf[q][s + 1];
      }
      if constexpr (IND) {
        w1[s] = w1[s + 1];
        w2[s] = w2[s + 1];
      }
    }
  }
}

// ------------------------------------------------------------------ inversion
// Occupancy of the inversion: on the flat metric its registers fit 96 VGPRs
// without spills, which gives 5 wavefronts per SIMD instead of 4 (the Newton
// iteration is a dependent chain, so more wavefronts hide more latency); the
// tabulated metric needs 138 and is left to the compiler.
template <class MET>
constexpr int C2P_MIN_WAVES = MET::flat ? 5 : 1;

// With list != nullptr (learned guess) zones whose warm start has a relative
// residual above cp.defer_tol are left untouched and appended to list (their
// order is irrelevant: each is inverted on its own in the learned-guess pass);
// with cp.defer_all every zone is (one list reservation per wavefront).
template <class MET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(C2P_MIN_WAVES<MET>))) void k_c2p(Geom G, C2PParams cp, double* __restrict__ prim,
                                             double* __restrict__ cons,
                                             const double* __restrict__ tab,
                                             long long* __restrict__ partials,
                                             double* __restrict__ cfl_partials,
                                             int* __restrict__ list, int* __restrict__ list_n,
                                             double* __restrict__ list_y) {
  const long t = flat_thread();
  long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double cfl_v = 0.0;
  const bool in = t < (long)G.n[0] * G.n[1] * G.n[2];
  if (list && cp.defer_all) {
    const unsigned long long mask = __ballot(in);
    const int lane = threadIdx.x & 63;
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    int base = 0;
    if (lane == 0) base = atomicAdd(list_n, __popcll(mask));
    base = __shfl(base, 0, 64);
    if (in) list[base + rank] = (int)strip_zone_order<C2P_STRIP>(G, t);
  } else if (in) {
    const long z = strip_zone_order<C2P_STRIP>(G, t);
    const double defer = list ? cp.defer_tol : 0.0;
    double yl = -1.0;
    if (c2p_zone<MET>(G, cp, prim, cons, tab, z, -1.0, defer, cfl_partials != nullptr, st, cfl_v, -1.0,
                      &yl)) {
      const int pos = atomicAdd(list_n, 1);
      list[pos] = (int)z;
      if (list_y) list_y[pos] = yl;
    }
  }
  c2p_block_partials<true>(st, cfl_v, partials, cfl_partials, blockIdx.x, cp.run_acc);
}

// Second pass of the split inversion: the zones the first pass deferred after
// cp.split_it iterations (cp.split_it is 0 here), grid-stride over the list,
// each from the iterate it stopped at.  Slow zones, which would hold a whole
// wavefront in the first pass, run here in compact wavefronts.
template <class MET>
__global__ __launch_bounds__(256) void k_c2p_split(Geom G, C2PParams cp, double* __restrict__ prim,
                                                   double* __restrict__ cons,
                                                   const double* __restrict__ tab,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ list_n,
                                                   const double* __restrict__ list_y,
                                                   long long* __restrict__ partials,
                                                   double* __restrict__ cfl_partials) {
  long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double cfl_v = 0.0;
  const long n = *list_n;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    double cv = 0.0;
    c2p_zone<MET>(G, cp, prim, cons, tab, list[idx], -1.0, 0.0, cfl_partials != nullptr, st, cv, list_y[idx]);
    cfl_v = fmax(cfl_v, cv);
  }
  c2p_block_partials<false>(st, cfl_v, partials, cfl_partials, blockIdx.x, cp.run_acc);
}

__global__ __launch_bounds__(256) void k_reduce_stats(const long long* __restrict__ partials, int nb,
                                                      long long* __restrict__ out) {
  __shared__ long long sh[256][C2P_NSTAT];
  long long acc[C2P_NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 256) {
    const long long* p = partials + (long)b * C2P_NSTAT;
    for (int q = 0; q < C2P_NSTAT; ++q) {
      if (q == 2) acc[q] = p[q] > acc[q] ? p[q] : acc[q];
      else acc[q] += p[q];
    }
  }
  for (int q = 0; q < C2P_NSTAT; ++q) sh[threadIdx.x][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256; ++w)
      for (int q = 0; q < C2P_NSTAT; ++q) {
        if (q == 2) acc[q] = sh[w][q] > acc[q] ? sh[w][q] : acc[q];
        else acc[q] += sh[w][q];
      }
    for (int q = 0; q < C2P_NSTAT; ++q) out[q] = acc[q];
  }
}

// ------------------------------------------------------------------ prim -> cons
template <class MET>
__global__ __launch_bounds__(256) void k_prim2cons(Geom G, double* __restrict__ prim,
                                                   double* __restrict__ cons,
                                                   const double* __restrict__ tab) {
  const long t = flat_thread();
  if (t >= (long)G.n[0] * G.n[1] * G.n[2]) return;
  int i, j, k;
  zone_of(G, t, i, j, k);
  const long c = G.idx(i, j, k);
  MET m;
  if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
  double B[3];
  centred_b(G, cons, c, m, B);
  PState<double> s;
  s.rho = prim[P_RHO * G.field + c];
  s.p = prim[P_P * G.field + c];
  for (int q = 0; q < 3; ++q) { s.u[q] = prim[(P_U1 + q) * G.field + c]; s.B[q] = B[q]; }
  make_state(s, m, G.gam);
  double cc[5];
  cons_of(s, m, cc);
  for (int q = 0; q < 5; ++q) cons[(long)q * G.field + c] = cc[q];
  for (int q = 0; q < 3; ++q) prim[(P_B1 + q) * G.field + c] = B[q];
}

// ------------------------------------------------------------------ CFL
template <class MET>
__global__ __launch_bounds__(256) void k_cfl(Geom G, const double* __restrict__ prim,
                                             const double* __restrict__ tab,
                                             double* __restrict__ partials) {
  const long t = flat_thread();
  double v = 0.0;
  if (t < (long)G.n[0] * G.n[1] * G.n[2]) {
    int i, j, k;
    zone_of(G, t, i, j, k);
    const long c = G.idx(i, j, k);
    MET m;
    if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
    PState<double> s;
    s.rho = prim[P_RHO * G.field + c];
    s.p = prim[P_P * G.field + c];
    for (int q = 0; q < 3; ++q) { s.u[q] = prim[(P_U1 + q) * G.field + c]; s.B[q] = prim[(P_B1 + q) * G.field + c]; }
    make_state(s, m, G.gam);
    double tot = 0.0;
    for (int d = 0; d < 3; ++d) {
      double lp, lm;
      speeds_of(s, m, d, G.gam, lp, lm);
      tot = tot + fmax(fabs(lp), fabs(lm)) / G.dx[d];
    }
    v = tot;
  }
  __shared__ double sh[4];
  const double w = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// One workgroup of DT_THREADS reduces the partials; each thread keeps
// DT_ACC independent maxima so that DT_ACC loads are in flight at once
// (a max is exact, so the order does not matter).
constexpr int DT_THREADS = 1024, DT_ACC = 8;

__global__ __launch_bounds__(DT_THREADS) void k_dt_final(const double* __restrict__ partials, int nb,
                                                         double cfl, double* __restrict__ d_dt) {
  __shared__ double sh[DT_THREADS / 64];
  double v[DT_ACC];
#pragma unroll
  for (int u = 0; u < DT_ACC; ++u) v[u] = 0.0;
  int b = threadIdx.x;
  for (; b + (DT_ACC - 1) * DT_THREADS < nb; b += DT_ACC * DT_THREADS) {
#pragma unroll
    for (int u = 0; u < DT_ACC; ++u) v[u] = fmax(v[u], partials[b + u * DT_THREADS]);
  }
  for (; b < nb; b += DT_THREADS) v[0] = fmax(v[0], partials[b]);
#pragma unroll
  for (int u = 1; u < DT_ACC; ++u) v[0] = fmax(v[0], v[u]);
  const double w = wave_max(v[0]);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int q = 1; q < DT_THREADS / 64; ++q) r = fmax(r, sh[q]);
    d_dt[0] = cfl / r;
  }
}

// ------------------------------------------------------------------ curl of a potential
__global__ __launch_bounds__(256) void k_curl(Geom G, const double* __restrict__ a1,
                                              const double* __restrict__ a2,
                                              const double* __restrict__ a3,
                                              double* __restrict__ cons) {
  const long t = flat_thread();
  if (t >= (long)G.n[0] * G.n[1] * G.n[2]) return;
  int i, j, k;
  zone_of(G, t, i, j, k);
  const long c = G.idx(i, j, k);
  const double* A[3] = {a1, a2, a3};
  double f[6];
  for (int nd = 0; nd < 3; ++nd) {
    const int d1 = (nd + 1) % 3, d2 = (nd + 2) % 3;
    const long s1 = G.stride(d1), s2 = G.stride(d2);
    for (int s = 0; s < 6; ++s) f[s] = A[d2][c + (s - 3) * s1];
    const double t1 = fd_deriv_rt(f, 1.0 / G.dx[d1], G.dorder);
    for (int s = 0; s < 6; ++s) f[s] = A[d1][c + (s - 3) * s2];
    const double t2 = fd_deriv_rt(f, 1.0 / G.dx[d2], G.dorder);
    cons[(long)(C_BF1 + nd) * G.field + c] = t1 - t2;
  }
}

// ------------------------------------------------------------------ ghost fill
// Composite source index of a ghost element; equals filling x^1, then x^2,
// then x^3 over the full extent of the other directions.
struct GhostSrc {
  int i, j, k;
  double sign;
  bool clamp_u1;
};

__device__ __forceinline__ int wrap(int m, int n) {
  int r = m % n;
  return r < 0 ? r + n : r;
}

// Outflow source index along one direction of n: cells and tangential faces
// copy the nearest interior index; the face field normal to the direction
// keeps its evolved ghost faces -flo .. -1 and n .. n + flo - 2 and copies
// the outermost of them beyond.
__device__ __forceinline__ int outflow_src(int m, int n, bool normal, int flo) {
  if (!normal) return m < 0 ? 0 : n - 1;
  return m < 0 ? max(m, -flo) : min(m, n + flo - 2);
}

__device__ __forceinline__ GhostSrc ghost_src(const Geom& G, const BCSpec& bc, int i, int j, int k,
                                              int normal, bool flip) {
  GhostSrc s{i, j, k, 1.0, false};
  const int n1 = G.n[0], n2 = G.n[1], n3 = G.n[2];
  const int flo = -G.face_lo();
  // x^1
  if (i < 0) s.i = bc.bc[0] == 0 ? wrap(i, n1) : outflow_src(i, n1, normal == 0, flo);
  else if (i >= n1) {
    s.i = bc.bc[1] == 0 ? wrap(i, n1) : outflow_src(i, n1, normal == 0, flo);
    s.clamp_u1 = bc.bc[1] == 1;
  }
  // x^2
  bool shift = false;
  if (bc.bc[2] == 2) {
    if (normal == 1) {
      // evolved: the ghost faces -flo .. -1 and n2 .. n2 + flo - 2 (with the
      // axis faces -1 and n2 - 1); beyond, minus the face half a turn away
      if (j < -flo) { s.j = -j - 2; shift = true; }
      else if (j > n2 + flo - 2) { s.j = 2 * n2 - j - 2; shift = true; }
    } else {
      if (j < 0) { s.j = -1 - j; shift = true; }
      else if (j >= n2) { s.j = 2 * n2 - 1 - j; shift = true; }
    }
  } else {
    if (j < 0) s.j = bc.bc[2] == 0 ? wrap(j, n2) : outflow_src(j, n2, normal == 1, flo);
    else if (j >= n2) s.j = bc.bc[3] == 0 ? wrap(j, n2) : outflow_src(j, n2, normal == 1, flo);
  }
  // x^3
  if (k < 0) s.k = bc.bc[4] == 0 ? wrap(k, n3) : outflow_src(k, n3, normal == 2, flo);
  else if (k >= n3) s.k = bc.bc[5] == 0 ? wrap(k, n3) : outflow_src(k, n3, normal == 2, flo);
  if (shift) {
    s.k = wrap(s.k + n3 / 2, n3);
    if (flip) s.sign = -1.0;
  }
  return s;
}

// Enumerates exactly the ghost elements: slabs of ghost x^3 planes, then
// ghost x^2 rows of interior planes, then ghost x^1 cells of interior rows.
__device__ __forceinline__ bool ghost_index(const Geom& G, long t, int& i, int& j, int& k) {
  const long d0 = G.dims[0], d1 = G.dims[1];
  const long NA = 2L * G.ng * d1 * d0;
  const long NB = (long)G.n[2] * 2 * G.ng * d0;
  const long NC = (long)G.n[2] * G.n[1] * 2 * G.ng;
  if (t < NA) {
    const int kl = (int)(t / (d1 * d0));
    const long r = t % (d1 * d0);
    k = kl < G.ng ? kl - G.ng : G.n[2] + kl - G.ng;
    j = (int)(r / d0) - G.ng;
    i = (int)(r % d0) - G.ng;
    return true;
  }
  t -= NA;
  if (t < NB) {
    k = (int)(t / (2 * G.ng * d0));
    const long r = t % (2 * G.ng * d0);
    const int jl = (int)(r / d0);
    j = jl < G.ng ? jl - G.ng : G.n[1] + jl - G.ng;
    i = (int)(r % d0) - G.ng;
    return true;
  }
  t -= NB;
  if (t < NC) {
    k = (int)(t / ((long)G.n[1] * 2 * G.ng));
    const long r = t % ((long)G.n[1] * 2 * G.ng);
    j = (int)(r / (2 * G.ng));
    const int il = (int)(r % (2 * G.ng));
    i = il < G.ng ? il - G.ng : G.n[0] + il - G.ng;
    return true;
  }
  return false;
}

__device__ __forceinline__ long ghost_total(const Geom& G) {
  const long d0 = G.dims[0], d1 = G.dims[1];
  return 2L * G.ng * d1 * d0 + (long)G.n[2] * 2 * G.ng * d0 + (long)G.n[2] * G.n[1] * 2 * G.ng;
}

__global__ __launch_bounds__(256) void k_bc_centred(Geom G, BCSpec bc, double* __restrict__ prim,
                                                    int nfields) {
  const long t = flat_thread();
  int i, j, k;
  if (t >= ghost_total(G) || !ghost_index(G, t, i, j, k)) return;
  const long dst = G.idx(i, j, k);
  for (int f = 0; f < nfields; ++f) {
    const bool flip = (f == P_U2 || f == P_U3 || f == P_B2 || f == P_B3);
    const GhostSrc s = ghost_src(G, bc, i, j, k, -1, flip);
    double v = prim[(long)f * G.field + G.idx(s.i, s.j, s.k)] * s.sign;
    if (f == P_U1 && s.clamp_u1) v = fmax(v, 0.0);
    prim[(long)f * G.field + dst] = v;
  }
}

// Face ghost fill: every source is an owned face or an evolved ghost face
// (normal to a non-periodic boundary), which this kernel does not write.
__global__ __launch_bounds__(256) void k_bc_faces(Geom G, BCSpec bc, double* __restrict__ cons) {
  const long t = flat_thread();
  int i, j, k;
  if (t >= ghost_total(G) || !ghost_index(G, t, i, j, k)) return;
  const long dst = G.idx(i, j, k);
  for (int nd = 0; nd < 3; ++nd) {
    const GhostSrc s = ghost_src(G, bc, i, j, k, nd, nd != 0);
    if (s.i == i && s.j == j && s.k == k) continue;   // an evolved ghost face
    double* f = cons + (long)(C_BF1 + nd) * G.field;
    f[dst] = f[G.idx(s.i, s.j, s.k)] * s.sign;
  }
}

// ------------------------------------------------------------------ diagnostics
template <class MET>
__global__ __launch_bounds__(256) void k_diag(Geom G, const double* __restrict__ prim,
                                              const double* __restrict__ cons,
                                              const double* __restrict__ tab,
                                              double* __restrict__ partials) {
  const long t = flat_thread();
  double sv[DIAG_NSUM], mv[DIAG_NMAX];
  for (int q = 0; q < DIAG_NSUM; ++q) sv[q] = 0.0;
  for (int q = 0; q < DIAG_NMAX; ++q) mv[q] = -INFINITY;
  if (t < (long)G.n[0] * G.n[1] * G.n[2]) {
    int i, j, k;
    zone_of(G, t, i, j, k);
    const long c = G.idx(i, j, k);
    for (int q = 0; q < 8; ++q) sv[q] = cons[(long)q * G.field + c];
    double f[6], dv = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double* fp = cons + (long)(C_BF1 + d) * G.field + c;
      const long st = G.stride(d);
      for (int s = 0; s < 6; ++s) f[s] = fp[(s - 3) * st];
      dv = dv + fd_deriv_rt(f, 1.0 / G.dx[d], G.dorder);
    }
    MET m;
    if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
    double u[3] = {prim[P_U1 * G.field + c], prim[P_U2 * G.field + c], prim[P_U3 * G.field + c]};
    double B[3] = {prim[P_B1 * G.field + c], prim[P_B2 * G.field + c], prim[P_B3 * G.field + c]};
    double ul[3], bl[3];
    m.lower(u, ul);
    m.lower(B, bl);
    const double rho = prim[P_RHO * G.field + c], p = prim[P_P * G.field + c];
    mv[0] = fabs(dv);
    mv[1] = -rho;
    mv[2] = rho;
    mv[3] = -p;
    mv[4] = p;
    mv[5] = sqrt(1.0 + ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2]);
    mv[6] = sqrt(fmax(bl[0] * B[0] + bl[1] * B[1] + bl[2] * B[2], 0.0));
    int nf = 0;
    for (int q = 0; q < 8; ++q) nf += isfinite(prim[(long)q * G.field + c]) ? 0 : 1;
    mv[7] = (double)nf;   // summed below, not maxed
  }
  __shared__ double sh[4][DIAG_NSUM + DIAG_NMAX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < DIAG_NSUM; ++q) {
    const double s = wave_sum(sv[q]);
    if (lane == 0) sh[wv][q] = s;
  }
  for (int q = 0; q < DIAG_NMAX; ++q) {
    const double s = (q == 7) ? wave_sum(mv[q] < 0 ? 0.0 : mv[q]) : wave_max(mv[q]);
    if (lane == 0) sh[wv][DIAG_NSUM + q] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* dst = partials + (long)blockIdx.x * (DIAG_NSUM + DIAG_NMAX);
    for (int q = 0; q < DIAG_NSUM; ++q) dst[q] = ((sh[0][q] + sh[1][q]) + sh[2][q]) + sh[3][q];
    for (int q = 0; q < DIAG_NMAX; ++q) {
      const int o = DIAG_NSUM + q;
      dst[o] = (q == 7) ? ((sh[0][o] + sh[1][o]) + sh[2][o]) + sh[3][o]
                        : fmax(fmax(sh[0][o], sh[1][o]), fmax(sh[2][o], sh[3][o]));
    }
  }
}

__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partials, int nb,
                                                    double* __restrict__ out) {
  constexpr int W = DIAG_NSUM + DIAG_NMAX;
  __shared__ double sh[256][W];
  double acc[W];
  for (int q = 0; q < W; ++q) acc[q] = (q >= DIAG_NSUM && q != DIAG_NSUM + 7) ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const double* p = partials + (long)b * W;
    for (int q = 0; q < W; ++q) {
      if (q >= DIAG_NSUM && q != DIAG_NSUM + 7) acc[q] = fmax(acc[q], p[q]);
      else acc[q] += p[q];
    }
  }
  for (int q = 0; q < W; ++q) sh[threadIdx.x][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256; ++w)
      for (int q = 0; q < W; ++q) {
        if (q >= DIAG_NSUM && q != DIAG_NSUM + 7) acc[q] = fmax(acc[q], sh[w][q]);
        else acc[q] += sh[w][q];
      }
    for (int q = 0; q < W; ++q) out[q] = acc[q];
  }
}

// ------------------------------------------------------------------ launchers
unsigned zone_blocks(const Geom& G) { return nblk((long)G.n[0] * G.n[1] * G.n[2]); }

static long ghost_count(const Geom& G) {
  const long d0 = G.dims[0], d1 = G.dims[1];
  return 2L * G.ng * d1 * d0 + (long)G.n[2] * 2 * G.ng * d0 + (long)G.n[2] * G.n[1] * 2 * G.ng;
}

void launch_bc_centred(const Geom& G, const BCSpec& bc, double* prim, int nfields, hipStream_t s) {
  hipLaunchKernelGGL(k_bc_centred, dim3(nblk(ghost_count(G))), dim3(256), 0, s, G, bc, prim, nfields);
}

void launch_bc_faces(const Geom& G, const BCSpec& bc, double* cons, hipStream_t s) {
  hipLaunchKernelGGL(k_bc_faces, dim3(nblk(ghost_count(G))), dim3(256), 0, s, G, bc, cons);
}

template <int DO, typename FS, int PARTS>
static void launch_update_p(const Geom& G, bool flat, int mode, const double* prim, double* x,
                            double* y, const FS* flux, const FS* edges,
                            const double* tab, double a, double b, double dt_host,
                            const double* d_dt, double* out, int stage, hipStream_t s, int img,
                            unsigned char* tflags, int* tlist, int* tcount) {
  const unsigned nb = zone_blocks(G);
  if (flat && mode == 0) {
    const long nseg = (G.n[2] + KZ - 1) / KZ;
    const unsigned ng = nblk((long)G.n[0] * G.n[1] * nseg);
    if (stage == 1)
      hipLaunchKernelGGL((k_update_zm<FlatMet<double>, 1, DO, FS, PARTS>), dim3(ng), dim3(256), 0, s, G, prim,
                         x, y, flux, edges, tab, a, b, dt_host, d_dt, img, tflags, tlist, tcount);
    else if (stage == 2)
      hipLaunchKernelGGL((k_update_zm<FlatMet<double>, 2, DO, FS, PARTS>), dim3(ng), dim3(256), 0, s, G, prim,
                         x, y, flux, edges, tab, a, b, dt_host, d_dt, img, tflags, tlist, tcount);
    else
      hipLaunchKernelGGL((k_update_zm<FlatMet<double>, 3, DO, FS, PARTS>), dim3(ng), dim3(256), 0, s, G, prim,
                         x, y, flux, edges, tab, a, b, dt_host, d_dt, img, tflags, tlist, tcount);
  } else if (flat) {
    // the right-hand side alone (mode 1): every field
    if constexpr (PARTS == UPD_ALL)
      hipLaunchKernelGGL((k_update<FlatMet<double>, DO, FS, UPD_ALL>), dim3(nb), dim3(256), 0, s, G, mode,
                         prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out, stage, tflags, tlist, tcount);
  } else {
    hipLaunchKernelGGL((k_update<TabMet<double>, DO, FS, PARTS>), dim3(nb), dim3(256), 0, s, G, mode, prim,
                       x, y, flux, edges, tab, a, b, dt_host, d_dt, out, stage, tflags, tlist, tcount);
  }
}

template <int DO, typename FS>
static void launch_update_o(const Geom& G, bool flat, int mode, const double* prim, double* x,
                            double* y, const FS* flux, const FS* edges,
                            const double* tab, double a, double b, double dt_host,
                            const double* d_dt, double* out, int stage, hipStream_t s, int img,
                            int parts, unsigned char* tflags, int* tlist, int* tcount) {
  if (parts == UPD_HYDRO)
    launch_update_p<DO, FS, UPD_HYDRO>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out,
                                       stage, s, img, tflags, tlist, tcount);
  else if (parts == UPD_INDUCTION)
    launch_update_p<DO, FS, UPD_INDUCTION>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt,
                                           out, stage, s, img, tflags, tlist, tcount);
  else
    launch_update_p<DO, FS, UPD_ALL>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out,
                                     stage, s, img, tflags, tlist, tcount);
}

template <typename FS>
static void launch_update_s(const Geom& G, bool flat, int mode, const double* prim, double* x, double* y,
                            const FS* flux, const FS* edges, const double* tab, double a, double b,
                            double dt_host, const double* d_dt, double* out, int stage, hipStream_t s,
                            int img, int parts, unsigned char* tflags, int* tlist, int* tcount) {
  if (G.dorder == 4)
    launch_update_o<4, FS>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out, stage, s, img,
                           parts, tflags, tlist, tcount);
  else
    launch_update_o<6, FS>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out, stage, s, img,
                           parts, tflags, tlist, tcount);
}

void launch_update(const Geom& G, bool flat, bool fp32, int mode, const double* prim, double* x, double* y,
                   const double* flux, const double* edges, const double* tab, double a, double b,
                   double dt_host, const double* d_dt, double* out, int stage, hipStream_t s, int img,
                   int parts, const UpdateFallback* fb) {
  // split updates are stage updates (mode 0); the hydro part flags when fb is given
  if (mode != 0) parts = UPD_ALL;
  unsigned char* tflags = fb ? fb->flags : nullptr;
  int* tlist = fb ? fb->list : nullptr;
  int* tcount = fb ? fb->count : nullptr;
  if (fp32)
    launch_update_s<float>(G, flat, mode, prim, x, y, reinterpret_cast<const float*>(flux),
                           reinterpret_cast<const float*>(edges), tab, a, b, dt_host, d_dt, out, stage, s, img,
                           parts, tflags, tlist, tcount);
  else
    launch_update_s<double>(G, flat, mode, prim, x, y, flux, edges, tab, a, b, dt_host, d_dt, out, stage, s,
                            img, parts, tflags, tlist, tcount);
}

// ------------------------------------------------------------------ evolved ghost faces
// The face field normal to a non-periodic direction nd at the ghost faces
// that the staggered derivative of an interior cell reads: stored
// -flo .. -1 and n .. n + flo - 2 along nd (flo = 3, or 2 for the
// fourth-order derivative), interior in the other two directions.  One
// thread per face, the layer index fastest.  POT: the curl of the edge
// potentials (initial data); otherwise the RK stage of the induction
// equation with the stage's edge fields, as the update does at the owned
// faces, so the discrete div B of the cells next to the boundary keeps its
// value.
template <int DO, typename FS, bool POT>
__global__ __launch_bounds__(256) void k_ghost_normal(Geom G, int nd, double* __restrict__ x,
                                                      double* __restrict__ y, const FS* __restrict__ edges,
                                                      const double* __restrict__ a1,
                                                      const double* __restrict__ a2,
                                                      const double* __restrict__ a3, double a, double b,
                                                      double dt_host, const double* __restrict__ d_dt,
                                                      int stage) {
  const int flo = -G.face_lo(), nl = 2 * flo - 1;
  const int d1 = (nd + 1) % 3, d2 = (nd + 2) % 3;
  const long t = flat_thread();
  if (t >= (long)nl * G.n[d1] * G.n[d2]) return;
  const int l = (int)(t % nl);
  const long r = t / nl;
  int ii[3];
  ii[nd] = l < flo ? l - flo : G.n[nd] + (l - flo);
  ii[d1] = (int)(r % G.n[d1]);
  ii[d2] = (int)(r / G.n[d1]);
  const long c = G.idx(ii[0], ii[1], ii[2]);
  const long s1 = G.stride(d1), s2 = G.stride(d2);
  const long o = (long)(C_BF1 + nd) * G.field + c;
  double f[6];
  if constexpr (POT) {
    const double* A[3] = {a1, a2, a3};
    for (int s = 0; s < 6; ++s) f[s] = A[d2][c + (s - 3) * s1];
    const double t1 = fd_deriv_rt(f, 1.0 / G.dx[d1], G.dorder);
    for (int s = 0; s < 6; ++s) f[s] = A[d1][c + (s - 3) * s2];
    const double t2 = fd_deriv_rt(f, 1.0 / G.dx[d2], G.dorder);
    x[o] = t1 - t2;
  } else {
    const FS* e2 = edges + (long)d2 * G.field + c;
    const FS* e1 = edges + (long)d1 * G.field + c;
#pragma unroll
    for (int s = 0; s < 6; ++s) f[s] = e2[(s - 3) * s1];
    const double t1 = fd_deriv_o<DO>(f, 1.0 / G.dx[d1]);
#pragma unroll
    for (int s = 0; s < 6; ++s) f[s] = e1[(s - 3) * s2];
    const double t2 = fd_deriv_o<DO>(f, 1.0 / G.dx[d2]);
    const double dt = dt_host > 0.0 ? dt_host : *d_dt;
    rk_store_rt(x, y, o, a, b, dt, -t1 + t2, stage);
  }
}

static unsigned ghost_normal_blocks(const Geom& G, int nd) {
  const int flo = -G.face_lo();
  return nblk((long)(2 * flo - 1) * G.n[(nd + 1) % 3] * G.n[(nd + 2) % 3]);
}

template <typename FS>
static void launch_ghost_normal_s(const Geom& G, int nd, double* x, double* y, const FS* edges, double a,
                                  double b, double dt_host, const double* d_dt, int stage, hipStream_t s) {
  if (G.dorder == 4)
    hipLaunchKernelGGL((k_ghost_normal<4, FS, false>), dim3(ghost_normal_blocks(G, nd)), dim3(256), 0, s, G, nd,
                       x, y, edges, nullptr, nullptr, nullptr, a, b, dt_host, d_dt, stage);
  else
    hipLaunchKernelGGL((k_ghost_normal<6, FS, false>), dim3(ghost_normal_blocks(G, nd)), dim3(256), 0, s, G, nd,
                       x, y, edges, nullptr, nullptr, nullptr, a, b, dt_host, d_dt, stage);
}

void launch_ghost_normal_update(const Geom& G, const BCSpec& bc, bool fp32, double* x, double* y,
                                const double* edges, double a, double b, double dt_host, const double* d_dt,
                                int stage, hipStream_t s) {
  for (int nd = 0; nd < 3; ++nd) {
    if (bc.bc[2 * nd] == 0) continue;   // periodic: the ghosts are images of owned faces
    if (fp32)
      launch_ghost_normal_s<float>(G, nd, x, y, reinterpret_cast<const float*>(edges), a, b, dt_host, d_dt,
                                   stage, s);
    else
      launch_ghost_normal_s<double>(G, nd, x, y, edges, a, b, dt_host, d_dt, stage, s);
  }
}

void launch_ghost_normal_curl(const Geom& G, const BCSpec& bc, const double* a1, const double* a2,
                              const double* a3, double* cons, hipStream_t s) {
  for (int nd = 0; nd < 3; ++nd) {
    if (bc.bc[2 * nd] == 0) continue;
    hipLaunchKernelGGL((k_ghost_normal<6, double, true>), dim3(ghost_normal_blocks(G, nd)), dim3(256), 0, s, G,
                       nd, cons, nullptr, nullptr, a1, a2, a3, 0.0, 0.0, 0.0, nullptr, 0);
  }
}

// d_dt[0]: dt of the last step, d_dt[1]: time; src: where the device dt was read
__global__ void k_advance(double* d_dt, const double* src, double dt_host) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double dt = dt_host > 0.0 ? dt_host : src[0];
    d_dt[0] = dt;
    d_dt[1] = d_dt[1] + dt;
  }
}

void launch_advance(double* d_dt, const double* src, double dt_host, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d_dt, src, dt_host);
}

void launch_c2p(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                const double* tab, long long* partials, double* cfl_partials, int* list, int* list_n,
                double* list_y, hipStream_t s) {
  const unsigned nb = zone_blocks(G);
  if (flat)
    hipLaunchKernelGGL(k_c2p<FlatMet<double>>, dim3(nb), dim3(256), 0, s, G, cp, prim, cons, tab,
                       partials, cfl_partials, list, list_n, list_y);
  else
    hipLaunchKernelGGL(k_c2p<TabMet<double>>, dim3(nb), dim3(256), 0, s, G, cp, prim, cons, tab,
                       partials, cfl_partials, list, list_n, list_y);
}

void launch_c2p_split(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                      const double* tab, const int* list, const int* list_n, const double* list_y,
                      long long* partials, double* cfl_partials, hipStream_t s) {
  C2PParams c2 = cp;
  c2.split_it = 0;
  c2.defer_tol = 0.0;
  if (flat)
    hipLaunchKernelGGL(k_c2p_split<FlatMet<double>>, dim3(C2P_LIST_BLOCKS), dim3(256), 0, s, G, c2, prim,
                       cons, tab, list, list_n, list_y, partials, cfl_partials);
  else
    hipLaunchKernelGGL(k_c2p_split<TabMet<double>>, dim3(C2P_LIST_BLOCKS), dim3(256), 0, s, G, c2, prim,
                       cons, tab, list, list_n, list_y, partials, cfl_partials);
}

__global__ void k_zero_int(int* __restrict__ p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

void launch_zero_int(int* p, hipStream_t s) { hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, p); }

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* __restrict__ p, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) p[q] = 0ull;
}

void launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, p, n);
}

void launch_dt_final(const double* cfl_partials, int nb, double cfl, double* d_dt, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(DT_THREADS), 0, s, cfl_partials, nb, cfl, d_dt);
}

void launch_reduce_stats(const long long* partials, int nb, long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(256), 0, s, partials, nb, out);
}

void launch_prim2cons(const Geom& G, bool flat, double* prim, double* cons, const double* tab,
                      hipStream_t s) {
  const unsigned nb = zone_blocks(G);
  if (flat)
    hipLaunchKernelGGL(k_prim2cons<FlatMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, cons, tab);
  else
    hipLaunchKernelGGL(k_prim2cons<TabMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, cons, tab);
}

void launch_cfl(const Geom& G, bool flat, const double* prim, const double* tab, double cfl,
                double* partials, double* d_dt, hipStream_t s) {
  const unsigned nb = zone_blocks(G);
  if (flat)
    hipLaunchKernelGGL(k_cfl<FlatMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, tab, partials);
  else
    hipLaunchKernelGGL(k_cfl<TabMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, tab, partials);
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(DT_THREADS), 0, s, partials, (int)nb, cfl, d_dt);
}

void launch_curl(const Geom& G, const double* a1, const double* a2, const double* a3,
                 double* cons, hipStream_t s) {
  hipLaunchKernelGGL(k_curl, dim3(zone_blocks(G)), dim3(256), 0, s, G, a1, a2, a3, cons);
}

// ------------------------------------------------------------------ shell fluxes
// Over each x^1 shell i and its (j, k): the pointwise x^1-fluxes of D and tau
// of the cell-centred state, |B_face^1| and B_face^1 at the upper x^1 face,
// each times dx^2 dx^3 (flux through the sphere r = r_i in (ln r, theta,
// phi)).  Workgroup (i, chunk) sums a fixed chunk of the shell into part;
// k_shell_final adds the chunks of a shell in order (deterministic).
// out: [F_D (n1), F_tau (n1), Phi = |B|/2 (n1), Phi_signed (n1)].
constexpr int SHELL_CHUNKS = 16;

template <class MET>
__global__ __launch_bounds__(256) void k_shell(Geom G, const double* __restrict__ prim,
                                               const double* __restrict__ cons,
                                               const double* __restrict__ tab,
                                               double* __restrict__ part) {
  const int i = blockIdx.x, ch = blockIdx.y;
  const long m2 = (long)G.n[1] * G.n[2];
  const long q0 = m2 * ch / SHELL_CHUNKS, q1 = m2 * (ch + 1) / SHELL_CHUNKS;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long q = q0 + threadIdx.x; q < q1; q += 256) {
    const int j = (int)(q % G.n[1]), k = (int)(q / G.n[1]);
    const long c = G.idx(i, j, k);
    MET m;
    if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
    PState<double> st;
    st.rho = prim[P_RHO * G.field + c];
    st.p = prim[P_P * G.field + c];
    for (int a = 0; a < 3; ++a) {
      st.u[a] = prim[(P_U1 + a) * G.field + c];
      st.B[a] = prim[(P_B1 + a) * G.field + c];
    }
    make_state(st, m, G.gam);
    double f[5];
    flux_of(st, m, 0, f);
    const double bf = cons[(long)C_BF1 * G.field + c];
    acc[0] += f[0];
    acc[1] += f[4];
    acc[2] += fabs(bf);
    acc[3] += bf;
  }
  __shared__ double sh[4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int a = 0; a < 4; ++a) {
    const double w = wave_sum(acc[a]);
    if (lane == 0) sh[wv][a] = w;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int a = threadIdx.x;
    part[((long)a * G.n[0] + i) * SHELL_CHUNKS + ch] = (sh[0][a] + sh[1][a]) + (sh[2][a] + sh[3][a]);
  }
}

__global__ __launch_bounds__(256) void k_shell_final(Geom G, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= 4L * G.n[0]) return;
  double v = 0.0;
  for (int ch = 0; ch < SHELL_CHUNKS; ++ch) v += part[e * SHELL_CHUNKS + ch];
  v *= G.dx[1] * G.dx[2];
  out[e] = e / G.n[0] == 2 ? 0.5 * v : v;
}

void launch_shell(const Geom& G, bool flat, const double* prim, const double* cons, const double* tab,
                  double* part, double* out, hipStream_t s) {
  const dim3 grid(G.n[0], SHELL_CHUNKS);
  if (flat)
    hipLaunchKernelGGL(k_shell<FlatMet<double>>, grid, dim3(256), 0, s, G, prim, cons, tab, part);
  else
    hipLaunchKernelGGL(k_shell<TabMet<double>>, grid, dim3(256), 0, s, G, prim, cons, tab, part);
  hipLaunchKernelGGL(k_shell_final, dim3((unsigned)((4L * G.n[0] + 255) / 256)), dim3(256), 0, s, G, part, out);
}

long shell_part_doubles(const Geom& G) { return 4L * G.n[0] * SHELL_CHUNKS; }

// ------------------------------------------------------------------ MRI resolution
// Per zone of the stored state: the field in the fluid frame (b^t = W v.B /
// alpha, b^i = B^i / W + b^t (alpha v^i - beta^i), b^2 = B^2 / W^2 + (v.B)^2),
// the angular velocity Omega = alpha v^3 - beta^3 (u^3 / u^t), and the
// number of zones per fastest-growing MRI wavelength along x^2 and x^3,
// Q_d = 2 pi |b^d| / (|Omega| dx^d sqrt(rho h + b^2)).  Over the body zones
// (rho > rho_cut), with the weight w = rho sqrt(gamma), workgroup (i, chunk)
// sums w Q_2, w Q_3, w, the zone count and the counts with Q_2, Q_3 >= q_min
// over a fixed chunk of shell i; k_mri_final adds the chunks in order.
// out: those six sums per shell, each an n1 array.
constexpr int MRI_NSUM = 6;

template <class MET>
__global__ __launch_bounds__(256) void k_mri(Geom G, const double* __restrict__ prim,
                                             const double* __restrict__ tab, double rho_cut,
                                             double q_min, double* __restrict__ part) {
  const int i = blockIdx.x, ch = blockIdx.y;
  const long m2 = (long)G.n[1] * G.n[2];
  const long q0 = m2 * ch / SHELL_CHUNKS, q1 = m2 * (ch + 1) / SHELL_CHUNKS;
  double acc[MRI_NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  MET m;
  for (long q = q0 + threadIdx.x; q < q1; q += 256) {
    const int j = (int)(q % G.n[1]), k = (int)(q / G.n[1]);
    const long c = G.idx(i, j, k);
    if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
    PState<double> st;
    st.rho = prim[P_RHO * G.field + c];
    st.p = prim[P_P * G.field + c];
    for (int a = 0; a < 3; ++a) {
      st.u[a] = prim[(P_U1 + a) * G.field + c];
      st.B[a] = prim[(P_B1 + a) * G.field + c];
    }
    if (!(st.rho > rho_cut)) continue;
    make_state(st, m, G.gam);
    const double bt = st.W * st.vB / m.alpha();
    const double b2c = st.B[1] / st.W + bt * m.tvel(st.v[1], 1);
    const double b3c = st.B[2] / st.W + bt * m.tvel(st.v[2], 2);
    const double bsq = st.B2 / (st.W * st.W) + st.vB * st.vB;
    const double den = fabs(m.tvel(st.v[2], 2)) * sqrt(st.rhoh + bsq);
    const double qq2 = 2.0 * M_PI * fabs(b2c) / (den * G.dx[1]);
    const double qq3 = 2.0 * M_PI * fabs(b3c) / (den * G.dx[2]);
    const double w = st.rho * m.sqrtg();
    acc[0] += w * qq2;
    acc[1] += w * qq3;
    acc[2] += w;
    acc[3] += 1.0;
    acc[4] += qq2 >= q_min ? 1.0 : 0.0;
    acc[5] += qq3 >= q_min ? 1.0 : 0.0;
  }
  __shared__ double sh[4][MRI_NSUM];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int a = 0; a < MRI_NSUM; ++a) {
    const double v = wave_sum(acc[a]);
    if (lane == 0) sh[wv][a] = v;
  }
  __syncthreads();
  if (threadIdx.x < MRI_NSUM) {
    const int a = threadIdx.x;
    part[((long)a * G.n[0] + i) * SHELL_CHUNKS + ch] = (sh[0][a] + sh[1][a]) + (sh[2][a] + sh[3][a]);
  }
}

__global__ __launch_bounds__(256) void k_mri_final(Geom G, const double* __restrict__ part,
                                                   double* __restrict__ out) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)MRI_NSUM * G.n[0]) return;
  double v = 0.0;
  for (int ch = 0; ch < SHELL_CHUNKS; ++ch) v += part[e * SHELL_CHUNKS + ch];
  out[e] = v;
}

void launch_mri(const Geom& G, bool flat, const double* prim, const double* tab, double rho_cut,
                double q_min, double* part, double* out, hipStream_t s) {
  const dim3 grid(G.n[0], SHELL_CHUNKS);
  if (flat)
    hipLaunchKernelGGL(k_mri<FlatMet<double>>, grid, dim3(256), 0, s, G, prim, tab, rho_cut, q_min, part);
  else
    hipLaunchKernelGGL(k_mri<TabMet<double>>, grid, dim3(256), 0, s, G, prim, tab, rho_cut, q_min, part);
  hipLaunchKernelGGL(k_mri_final, dim3((unsigned)(((long)MRI_NSUM * G.n[0] + 255) / 256)), dim3(256), 0, s,
                     G, part, out);
}

long mri_part_doubles(const Geom& G) { return (long)MRI_NSUM * G.n[0] * SHELL_CHUNKS; }

void launch_diag(const Geom& G, bool flat, const double* prim, const double* cons,
                 const double* tab, double* partials, double* out, hipStream_t s) {
  const unsigned nb = zone_blocks(G);
  if (flat)
    hipLaunchKernelGGL(k_diag<FlatMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, cons, tab, partials);
  else
    hipLaunchKernelGGL(k_diag<TabMet<double>>, dim3(nb), dim3(256), 0, s, G, prim, cons, tab, partials);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, partials, (int)nb, out);
}

}  // namespace grmhd
