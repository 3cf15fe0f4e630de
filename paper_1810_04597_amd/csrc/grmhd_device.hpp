// Device-side building blocks of the GRMHD kernels (gfx950, wave64).
//
// Method: the paper's Introduction states it (general-relativistic MHD, 3-D
// finite differences, high-order reconstruction, after ECHO).  The pieces
// here are the standard published forms of that scheme family:
//   * MP5 reconstruction (Suresh & Huynh 1997) with the point-value
//     interpolant (3, -20, 90, 60, -5)/128 and a zero limiter tolerance;
//   * 3+1 conserved variables, fluxes and fast-speed estimate (Valencia /
//     ECHO form; speeds after Gammie, McKinney & Toth 2003);
//   * HLL flux (Harten, Lax & van Leer 1983);
//   * sixth-order staggered derivative D and midpoint interpolation I.
// Every function is templated on the arithmetic type T (double, or float for
// the FP32-flux form) and on a metric policy: FlatMet (Minkowski, Cartesian;
// no metric arithmetic at all) or TabMet (tabulated alpha, beta, gamma).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grmhd {

constexpr int NG = 5;
constexpr int NPRIM = 8;   // rho, u1, u2, u3, p, B1, B2, B3
constexpr int NCONS = 8;   // D, S1, S2, S3, tau, Bf1, Bf2, Bf3
enum { P_RHO = 0, P_U1 = 1, P_U2 = 2, P_U3 = 3, P_P = 4, P_B1 = 5, P_B2 = 6, P_B3 = 7 };
enum { C_D = 0, C_S1 = 1, C_S2 = 2, C_S3 = 3, C_TAU = 4, C_BF1 = 5, C_BF2 = 6, C_BF3 = 7 };

// Metric table layout: [comp][j][i] over (n2+2ng) x (n1+2ng).
constexpr int NGEOM = 17;
enum { M_AL = 0, M_B1 = 1, M_B2 = 2, M_B3 = 3, M_G11 = 4, M_G12, M_G13, M_G22, M_G23, M_G33,
       M_U11, M_U12, M_U13, M_U22, M_U23, M_U33, M_SG };
enum { LOC_C = 0, LOC_F1 = 1, LOC_F2 = 2, LOC_E3 = 3 };
constexpr int DER_BASE = 4 * NGEOM;   // 20 centre derivatives follow
enum { D1_AL = 0, D2_AL = 1, D1_B1 = 2, D1_B2, D1_B3, D2_B1, D2_B2, D2_B3,
       D1_G11 = 8, D1_G12, D1_G13, D1_G22, D1_G23, D1_G33,
       D2_G11 = 14, D2_G12, D2_G13, D2_G22, D2_G23, D2_G33 };
constexpr int NCOMP_TAB = DER_BASE + 20;

// Grid geometry as kernels see it (passed by value).
struct Geom {
  int n[3];            // interior zones
  int dims[3];         // n + 2 NG
  long pitch, plane;   // element strides of x^2 and x^3
  long field;          // elements between fields of a group
  long off;            // offset of interior (0,0,0)
  double dx[3], x0[3];
  double gam;          // ideal-gas index
  int tab_n1;          // metric table row length (n1 + 2 NG)
  long tab_plane;      // metric table component stride
  __host__ __device__ long idx(int i, int j, int k) const {
    return off + (long)k * plane + (long)j * pitch + i;
  }
  __host__ __device__ long stride(int d) const { return d == 0 ? 1L : (d == 1 ? pitch : plane); }
  __host__ __device__ long tidx(int i, int j) const {
    return (long)(j + NG) * tab_n1 + (i + NG);
  }
};

// ------------------------------------------------------------------ MP5
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  // (sgn a + sgn b)/2 * min(|a|, |b|)
  return (a > T(0) && b > T(0)) ? fmin(a, b) : ((a < T(0) && b < T(0)) ? fmax(a, b) : T(0));
}

template <typename T>
__device__ __forceinline__ T minmod4(T w, T x, T y, T z) {
  if (w > T(0) && x > T(0) && y > T(0) && z > T(0)) return fmin(fmin(w, x), fmin(y, z));
  if (w < T(0) && x < T(0) && y < T(0) && z < T(0)) return fmax(fmax(w, x), fmax(y, z));
  return T(0);
}

// Limited left state at the face between q0 and qp1 from q_{j-2..j+2}.
template <typename T>
__device__ __forceinline__ T mp5(T qm2, T qm1, T q0, T qp1, T qp2) {
  const T ql = (T(3) * qm2 - T(20) * qm1 + T(90) * q0 + T(60) * qp1 - T(5) * qp2) * T(1.0 / 128.0);
  const T qmp = q0 + minmod(qp1 - q0, T(4) * (q0 - qm1));
  if ((ql - q0) * (ql - qmp) <= T(0)) return ql;
  const T dm1 = qm2 - T(2) * qm1 + q0;
  const T d0 = qm1 - T(2) * q0 + qp1;
  const T dp1 = q0 - T(2) * qp1 + qp2;
  const T dm4p = minmod4(T(4) * d0 - dp1, T(4) * dp1 - d0, d0, dp1);
  const T dm4m = minmod4(T(4) * d0 - dm1, T(4) * dm1 - d0, d0, dm1);
  const T qul = q0 + T(4) * (q0 - qm1);
  const T qmd = T(0.5) * (q0 + qp1) - T(0.5) * dm4p;
  const T qlc = q0 + T(0.5) * (q0 - qm1) + T(4.0 / 3.0) * dm4m;
  const T qmin = fmax(fmin(fmin(q0, qp1), qmd), fmin(fmin(q0, qul), qlc));
  const T qmax = fmin(fmax(fmax(q0, qp1), qmd), fmax(fmax(q0, qul), qlc));
  return ql + minmod(qmin - ql, qmax - ql);
}

// Left and right states at face f+1/2 from the six cells f-2 .. f+3 (c[0..5]).
template <typename T>
__device__ __forceinline__ void mp5_lr(const T c[6], T& l, T& r) {
  l = mp5(c[0], c[1], c[2], c[3], c[4]);
  r = mp5(c[5], c[4], c[3], c[2], c[1]);
}

// ------------------------------------------------------------------ FD operators
// Sixth-order staggered derivative at m from f_{m-5/2..m+5/2} = f[0..5]
// (stored indices m-3 .. m+2).
__device__ __forceinline__ double fd_deriv(const double f[6], double inv_dx) {
  return (75.0 / 64.0 * (f[3] - f[2]) - 25.0 / 384.0 * (f[4] - f[1]) +
          3.0 / 640.0 * (f[5] - f[0])) * inv_dx;
}
__device__ __forceinline__ double fd_interp(const double f[6]) {
  return (150.0 * (f[3] + f[2]) - 25.0 * (f[4] + f[1]) + 3.0 * (f[5] + f[0])) * (1.0 / 256.0);
}

// ------------------------------------------------------------------ metric policies
template <typename T>
struct FlatMet {
  static constexpr bool flat = true;
  __device__ __forceinline__ void lower(const T a[3], T o[3]) const { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }
  __device__ __forceinline__ void raise(const T a[3], T o[3]) const { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }
  __device__ __forceinline__ T guu(int) const { return T(1); }
  __device__ __forceinline__ T tvel(T v, int) const { return v; }             // alpha v - beta
  __device__ __forceinline__ T dens(T x) const { return x; }                 // sqrt(gamma) x
  __device__ __forceinline__ T undens(T x) const { return x; }
  __device__ __forceinline__ T fcomb(T x, T y, int) const { return x; }      // sqrt(g)(alpha x - beta^d y)
  __device__ __forceinline__ T alpha() const { return T(1); }
  __device__ __forceinline__ T beta(int) const { return T(0); }
  __device__ __forceinline__ T sqrtg() const { return T(1); }
  __device__ __forceinline__ T e_up(T x) const { return x; }                 // x / sqrt(gamma)
  __device__ __forceinline__ T e_lo(T x) const { return x; }                 // x * sqrt(gamma)
};

template <typename T>
struct TabMet {
  static constexpr bool flat = false;
  T al, b[3], g11, g12, g13, g22, g23, g33, u11, u12, u13, u22, u23, u33, sg;
  __device__ __forceinline__ void load(const double* __restrict__ tab, long tplane, int loc, long t) {
    const double* p = tab + (long)loc * NGEOM * tplane + t;
    al = T(p[M_AL * tplane]);
    b[0] = T(p[M_B1 * tplane]); b[1] = T(p[M_B2 * tplane]); b[2] = T(p[M_B3 * tplane]);
    g11 = T(p[M_G11 * tplane]); g12 = T(p[M_G12 * tplane]); g13 = T(p[M_G13 * tplane]);
    g22 = T(p[M_G22 * tplane]); g23 = T(p[M_G23 * tplane]); g33 = T(p[M_G33 * tplane]);
    u11 = T(p[M_U11 * tplane]); u12 = T(p[M_U12 * tplane]); u13 = T(p[M_U13 * tplane]);
    u22 = T(p[M_U22 * tplane]); u23 = T(p[M_U23 * tplane]); u33 = T(p[M_U33 * tplane]);
    sg = T(p[M_SG * tplane]);
  }
  __device__ __forceinline__ void lower(const T a[3], T o[3]) const {
    o[0] = g11 * a[0] + g12 * a[1] + g13 * a[2];
    o[1] = g12 * a[0] + g22 * a[1] + g23 * a[2];
    o[2] = g13 * a[0] + g23 * a[1] + g33 * a[2];
  }
  __device__ __forceinline__ void raise(const T a[3], T o[3]) const {
    o[0] = u11 * a[0] + u12 * a[1] + u13 * a[2];
    o[1] = u12 * a[0] + u22 * a[1] + u23 * a[2];
    o[2] = u13 * a[0] + u23 * a[1] + u33 * a[2];
  }
  __device__ __forceinline__ T guu(int d) const { return d == 0 ? u11 : (d == 1 ? u22 : u33); }
  __device__ __forceinline__ T tvel(T v, int d) const { return al * v - b[d]; }
  __device__ __forceinline__ T dens(T x) const { return sg * x; }
  __device__ __forceinline__ T undens(T x) const { return x / sg; }
  __device__ __forceinline__ T fcomb(T x, T y, int d) const { return sg * (al * x - b[d] * y); }
  __device__ __forceinline__ T alpha() const { return al; }
  __device__ __forceinline__ T beta(int d) const { return b[d]; }
  __device__ __forceinline__ T sqrtg() const { return sg; }
  __device__ __forceinline__ T e_up(T x) const { return x / sg; }
  __device__ __forceinline__ T e_lo(T x) const { return sg * x; }
};

// ------------------------------------------------------------------ pointwise physics
template <typename T>
struct PState {
  T rho, p, u[3], B[3];
  T W, v[3], vl[3], v2, Bl[3], B2, vB, E2, h, y, D, S[3], Su[3], tau;
};

// Derived quantities of a primitive state (3+1 GRMHD, ideal gas).
template <typename T, class M>
__device__ __forceinline__ void make_state(PState<T>& s, const M& m, T gam) {
  T ul[3];
  m.lower(s.u, ul);
  const T uu = ul[0] * s.u[0] + ul[1] * s.u[1] + ul[2] * s.u[2];
  s.W = sqrt(T(1) + uu);
  const T iw = T(1) / s.W;
  for (int i = 0; i < 3; ++i) { s.v[i] = s.u[i] * iw; s.vl[i] = ul[i] * iw; }
  s.v2 = uu / (T(1) + uu);
  m.lower(s.B, s.Bl);
  s.B2 = s.Bl[0] * s.B[0] + s.Bl[1] * s.B[1] + s.Bl[2] * s.B[2];
  s.vB = s.vl[0] * s.B[0] + s.vl[1] * s.B[1] + s.vl[2] * s.B[2];
  s.E2 = s.B2 * s.v2 - s.vB * s.vB;
  s.h = T(1) + gam / (gam - T(1)) * s.p / s.rho;
  s.y = s.rho * s.h * s.W * s.W;
  s.D = s.rho * s.W;
  const T yb = s.y + s.B2;
  for (int i = 0; i < 3; ++i) {
    s.S[i] = yb * s.vl[i] - s.vB * s.Bl[i];
    s.Su[i] = yb * s.v[i] - s.vB * s.B[i];
  }
  s.tau = s.y - s.p + T(0.5) * (s.B2 + s.E2) - s.D;
}

// Densitised conserved hydro variables.
template <typename T, class M>
__device__ __forceinline__ void cons_of(const PState<T>& s, const M& m, T c[5]) {
  c[0] = m.dens(s.D);
  c[1] = m.dens(s.S[0]); c[2] = m.dens(s.S[1]); c[3] = m.dens(s.S[2]);
  c[4] = m.dens(s.tau);
}

// Densitised fluxes of (D, S_1..3, tau) in direction d.
template <typename T, class M>
__device__ __forceinline__ void flux_of(const PState<T>& s, const M& m, int d, T f[5]) {
  // electric field E_i = -sqrt(g) [ijk] v^j B^k, E^i = -[ijk] v_j B_k / sqrt(g)
  T el[3], eu_d;
  el[0] = m.e_lo(-(s.v[1] * s.B[2] - s.v[2] * s.B[1]));
  el[1] = m.e_lo(-(s.v[2] * s.B[0] - s.v[0] * s.B[2]));
  el[2] = m.e_lo(-(s.v[0] * s.B[1] - s.v[1] * s.B[0]));
  const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
  eu_d = m.e_up(-(s.vl[d1] * s.Bl[d2] - s.vl[d2] * s.Bl[d1]));
  const T ptot = s.p + T(0.5) * (s.E2 + s.B2);
  f[0] = m.dens(m.tvel(s.v[d], d) * s.D);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T wdi = s.y * s.v[d] * s.vl[i] - eu_d * el[i] - s.B[d] * s.Bl[i];
    if (i == d) wdi = wdi + ptot;
    f[1 + i] = m.fcomb(wdi, s.S[i], d);
  }
  f[4] = m.fcomb(s.Su[d] - s.v[d] * s.D, s.tau, d);
}

// Fast magnetosonic speed estimate lambda^+-_d.
template <typename T, class M>
__device__ __forceinline__ void speeds_of(const PState<T>& s, const M& m, int d, T gam, T& lp, T& lm) {
  const T rhoh = s.rho * s.h;
  const T cs2 = gam * s.p / rhoh;
  const T bb = s.B2 / (s.W * s.W) + s.vB * s.vB;
  const T va2 = bb / (rhoh + bb);
  const T a2 = cs2 + va2 - cs2 * va2;
  const T vd = s.v[d];
  const T den = T(1) - s.v2 * a2;
  T rad = a2 * (T(1) - s.v2) * (m.guu(d) * den - vd * vd * (T(1) - a2));
  rad = sqrt(fmax(rad, T(0)));
  const T fac = m.alpha() / den;
  const T base = vd * (T(1) - a2);
  if (M::flat) {
    lp = fac * (base + rad);
    lm = fac * (base - rad);
  } else {
    lp = fac * (base + rad) - m.beta(d);
    lm = fac * (base - rad) - m.beta(d);
  }
}

// Threshold below which a+ + a- counts as zero.
template <typename T> __device__ __forceinline__ T tiny_speed();
template <> __device__ __forceinline__ double tiny_speed<double>() { return 1e-300; }
template <> __device__ __forceinline__ float tiny_speed<float>() { return 1e-37f; }

template <typename T>
__device__ __forceinline__ T hll(T fl, T fr, T ul, T ur, T ap, T am, T inv_s, bool tiny) {
  return tiny ? T(0.5) * (fl + fr) : (ap * fl + am * fr - ap * am * (ur - ul)) * inv_s;
}

}  // namespace grmhd
