// One zone of the conservative-to-primitive inversion, wavefront reductions
// and per-block partials (device code shared by the inversion kernel and the
// learned-guess pass over deferred zones).
#pragma once
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"

namespace grmhd {

// ------------------------------------------------------------------ wavefront reductions
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ long long wave_max_ll(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ void zone_of(const Geom& G, long t, int& i, int& j, int& k) {
  i = (int)(t % G.n[0]);
  const long r = t / G.n[0];
  j = (int)(r % G.n[1]);
  k = (int)(r / G.n[1]);
}

// Periodic ghost images of interior element (i, j, k) when every direction is
// periodic and every n >= 2 ng: per direction the offset 0 and, within ng of
// a boundary, +-n.  Writes v[f] to field fields[f] of each image other than
// the element itself (at most seven).
template <int NF>
__device__ __forceinline__ void write_images(const Geom& G, double* __restrict__ base, int i, int j,
                                             int k, const int fields[NF], const double v[NF]) {
  int off[3][2], cnt[3];
  const int x[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    off[d][0] = 0;
    cnt[d] = 1;
    if (x[d] < G.ng) { off[d][1] = G.n[d]; cnt[d] = 2; }
    else if (x[d] >= G.n[d] - G.ng) { off[d][1] = -G.n[d]; cnt[d] = 2; }
  }
  for (int a = 0; a < cnt[0]; ++a)
    for (int b = 0; b < cnt[1]; ++b)
      for (int c = 0; c < cnt[2]; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        const long e = G.idx(i + off[0][a], j + off[1][b], k + off[2][c]);
#pragma unroll
        for (int f = 0; f < NF; ++f) base[(long)fields[f] * G.field + e] = v[f];
      }
}

// Centred field B^d = I_d(face field) / sqrt(gamma) at element c.
template <class MET>
__device__ __forceinline__ void centred_b(const Geom& G, const double* __restrict__ cons, long c,
                                          const MET& m, double B[3]) {
  double f[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double* fp = cons + (long)(C_BF1 + d) * G.field + c;
    const long st = G.stride(d);
#pragma unroll
    for (int s = 0; s < 6; ++s) f[s] = fp[(s - 3) * st];
    B[d] = m.undens(fd_interp_rt(f, G.dorder));
  }
}

// Inversion of interior zone t (flattened, x^1 fastest): Newton from the
// warm or cold guess per cp.guess, y_alt > 0 a second candidate start (the
// smaller residual wins; a failed learned start is rerun from the warm one),
// then floors and the W cap.  With defer_tol > 0 a zone whose warm start has a
// larger relative residual is left untouched and true is returned.  Adds the
// zone's counters to st (fail, iterations, iterations max, floor_rho,
// floor_p, W cap, learned fallback, learned chosen) and, with want_cfl, sets
// cfl_v to its sum over d of max|lambda_d| / dx_d.
// y_start > 0 replaces the warm or cold guess (a zone finished from the
// iterate at which the first pass deferred it; the warm start is the fallback
// if that fails).  With cp.split_it > 0 a zone not converged after that many
// iterations is deferred (true) with its iterate in *y_last and its
// iterations counted.
template <class MET>
__device__ __forceinline__ bool c2p_zone(const Geom& G, const C2PParams& cp, double* __restrict__ prim,
                                         double* __restrict__ cons, const double* __restrict__ tab,
                                         long t, double y_alt, double defer_tol, bool want_cfl,
                                         long long st[8], double& cfl_v, double y_start = -1.0,
                                         double* y_last = nullptr, bool learned_start = false) {
  int i, j, k;
  zone_of(G, t, i, j, k);
  const long c = G.idx(i, j, k);
  MET m;
  if constexpr (!MET::flat) m.load(tab, G.tab_plane, LOC_C, G.tidx(i, j));
  double B[3];
  centred_b(G, cons, c, m, B);
  const double dd = m.undens(cons[C_D * G.field + c]);
  const double S[3] = {m.undens(cons[C_S1 * G.field + c]), m.undens(cons[C_S2 * G.field + c]),
                       m.undens(cons[C_S3 * G.field + c])};
  const double tau = m.undens(cons[C_TAU * G.field + c]);
  double rho = prim[P_RHO * G.field + c];
  double p = prim[P_P * G.field + c];
  double u[3] = {prim[P_U1 * G.field + c], prim[P_U2 * G.field + c], prim[P_U3 * G.field + c]};
  double ywarm;
  {
    double ul[3];
    m.lower(u, ul);
    const double uu = ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2];
    const double h = 1.0 + G.gam / (G.gam - 1.0) * p / rho;
    ywarm = rho * h * (1.0 + uu);
  }
  const double y0 = y_start > 0.0 ? y_start : (cp.guess == 1 ? G.gam * (tau + dd) : ywarm);
  NewtonOut<double> r = newton<double>(dd, S, tau, B, m, G.gam, y0, cp.tol, cp.maxit, y_alt, defer_tol,
                                       cp.split_it);
  if (r.deferred) {
    st[1] += r.iters;
    if (y_last) *y_last = r.y_last;
    return true;
  }
  // learned_start: y_start is the network's guess (counted as chosen, and
  // as a fallback when it has to be rerun from the warm guess)
  if (learned_start && y_start > 0.0) st[7] += 1;
  if (y_start > 0.0 && !r.ok) {
    const int it0 = r.iters;
    r = newton<double>(dd, S, tau, B, m, G.gam, ywarm, cp.tol, cp.maxit);
    r.iters += it0;
    if (learned_start) st[6] += 1;
  }
  if (r.alt) st[7] += 1;
  if (r.alt && !r.ok) {
    const int it0 = r.iters;
    r = newton<double>(dd, S, tau, B, m, G.gam, ywarm, cp.tol, cp.maxit);
    r.iters += it0;
    st[6] += 1;
  }
  if (r.ok) {
    rho = r.rho;
    p = r.p;
    u[0] = r.u[0]; u[1] = r.u[1]; u[2] = r.u[2];
  }
  st[0] += r.ok ? 0 : 1;
  st[1] += r.iters;
  st[2] = st[2] > r.iters ? st[2] : r.iters;
  bool floored = false;
  if (cp.rho_fl_a > 0.0 || cp.p_fl_a > 0.0 || cp.w_max > 0.0) {
    const double rr = cp.coord == 1 ? exp(G.x0[0] + (i + 0.5) * G.dx[0]) : 1.0;
    if (!r.ok) {
      // failed zone -> atmosphere at rest
      rho = cp.rho_fl_a * pow(rr, cp.rho_fl_n);
      p = cp.p_fl_a * pow(rr, cp.p_fl_n);
      u[0] = u[1] = u[2] = 0.0;
      floored = true;
    }
    if (cp.rho_fl_a > 0.0) {
      const double rfl = cp.rho_fl_a * pow(rr, cp.rho_fl_n);
      if (rho < rfl) { rho = rfl; floored = true; st[3] += 1; }
    }
    if (cp.p_fl_a > 0.0) {
      const double pfl = cp.p_fl_a * pow(rr, cp.p_fl_n);
      if (p < pfl) { p = pfl; floored = true; st[4] += 1; }
    }
    if (cp.w_max > 0.0) {
      double ul[3];
      m.lower(u, ul);
      const double uu = ul[0] * u[0] + ul[1] * u[1] + ul[2] * u[2];
      const double wcur = sqrt(1.0 + uu);
      if (wcur > cp.w_max) {
        const double fac = sqrt((cp.w_max * cp.w_max - 1.0) / uu);
        u[0] *= fac; u[1] *= fac; u[2] *= fac;
        floored = true;
        st[5] += 1;
      }
    }
  }
  prim[P_RHO * G.field + c] = rho;
  prim[P_P * G.field + c] = p;
  prim[P_U1 * G.field + c] = u[0];
  prim[P_U2 * G.field + c] = u[1];
  prim[P_U3 * G.field + c] = u[2];
  prim[P_B1 * G.field + c] = B[0];
  prim[P_B2 * G.field + c] = B[1];
  prim[P_B3 * G.field + c] = B[2];
  if (cp.img) {
    constexpr int pf[8] = {P_RHO, P_U1, P_U2, P_U3, P_P, P_B1, P_B2, P_B3};
    const double pv[8] = {rho, u[0], u[1], u[2], p, B[0], B[1], B[2]};
    write_images<8>(G, prim, i, j, k, pf, pv);
  }
  if (floored || want_cfl) {
    PState<double> s;
    s.rho = rho; s.p = p;
    for (int q = 0; q < 3; ++q) { s.u[q] = u[q]; s.B[q] = B[q]; }
    make_state(s, m, G.gam);
    if (floored) {
      double cc[5];
      cons_of(s, m, cc);
      for (int q = 0; q < 5; ++q) cons[(long)q * G.field + c] = cc[q];
    }
    if (want_cfl) {
      double tot = 0.0;
      for (int d = 0; d < 3; ++d) {
        double lp, lm;
        speeds_of(s, m, d, G.gam, lp, lm);
        tot = tot + fmax(fabs(lp), fabs(lm)) / G.dx[d];
      }
      cfl_v = tot;
    }
  }
  return false;
}

// Per-block partials of the counters (C2P_NSTAT each, written at slot) and,
// with cfl_partials, of the CFL speed sum (256-thread workgroups).  PACKED
// (one zone per thread, counters 0/1 and at most 2000 iterations): the six
// 0/1 counters go in 16-bit fields of two 64-bit words and the iteration sum
// in the upper half of the second, so a wavefront reduces two words and one
// 32-bit maximum instead of eight words.
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// run_acc (nullable): the block's failed, rho-floored, p-floored and W-capped
// zones, its zones taken from the learned-guess list (nlist, per thread), and
// its learned starts and their fallbacks are also added to the accumulated
// counters (only when non-zero).
template <bool PACKED>
__device__ __forceinline__ void c2p_block_partials(const long long st[8], double cfl_v,
                                                   long long* __restrict__ partials,
                                                   double* __restrict__ cfl_partials, int slot,
                                                   unsigned long long* __restrict__ run_acc,
                                                   long long nlist = 0) {
  if (cfl_partials) {
    __shared__ double shc[4];
    const double w = wave_max(cfl_v);
    if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) cfl_partials[slot] = fmax(fmax(shc[0], shc[1]), fmax(shc[2], shc[3]));
  }
  __shared__ long long sh[4][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long rr[8];
  if constexpr (PACKED) {
    const long long w0 = st[0] | (st[3] << 16) | (st[4] << 32) | (st[5] << 48);
    const long long w1 = st[6] | (st[7] << 16) | (st[1] << 32);
    const long long s0 = wave_sum_ll(w0), s1 = wave_sum_ll(w1);
    rr[0] = s0 & 0xffff; rr[3] = (s0 >> 16) & 0xffff; rr[4] = (s0 >> 32) & 0xffff; rr[5] = (s0 >> 48) & 0xffff;
    rr[6] = s1 & 0xffff; rr[7] = (s1 >> 16) & 0xffff; rr[1] = s1 >> 32;
    rr[2] = wave_max_i((int)st[2]);
  } else {
    for (int q = 0; q < 8; ++q) rr[q] = q == 2 ? wave_max_ll(st[q]) : wave_sum_ll(st[q]);
  }
  __shared__ long long shl[4];
  const long long nl = run_acc ? wave_sum_ll(nlist) : 0;
  if (lane == 0) {
    for (int q = 0; q < 8; ++q) sh[wv][q] = rr[q];
    shl[wv] = nl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 8; ++q) o[q] = q == 2 ? (sh[w][q] > o[q] ? sh[w][q] : o[q]) : o[q] + sh[w][q];
    long long* dst = partials + (long)slot * C2P_NSTAT;
    for (int q = 0; q < 8; ++q) dst[q] = o[q];
    if (run_acc) {
      const long long v[RUN_NCOUNT] = {o[0], o[3], o[4], o[5], shl[0] + shl[1] + shl[2] + shl[3], o[7], o[6]};
      unsigned long long* a = run_acc + (long)(blockIdx.x % RUN_SLOTS) * RUN_STRIDE;
      for (int q = 0; q < RUN_NCOUNT; ++q)
        if (v[q] != 0) atomicAdd(a + q, (unsigned long long)v[q]);
    }
  }
}

}  // namespace grmhd
