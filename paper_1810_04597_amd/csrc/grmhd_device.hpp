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

// Device code that is also instantiated on the host by the operation-count
// harness (with a counting number type), so it is __host__ __device__.
#define GR_HD __host__ __device__ __forceinline__

namespace grmhd {

using std::sqrt;
using std::fmin;
using std::fmax;
using std::fabs;

constexpr int NG = 5;      // default ghost width (MP5 stencil + sixth-order derivative)
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
  int dims[3];         // n + 2 ng
  long pitch, plane;   // element strides of x^2 and x^3
  long field;          // elements between fields of a group
  long off;            // offset of interior (0,0,0)
  double dx[3], x0[3];
  double gam;          // ideal-gas index
  int dorder;          // order of the staggered derivative and interpolation (6 or 4)
  int ng;              // ghost layers (5, or 6 for the eight-cell MP7 stencil)
  int tab_n1;          // metric table row length (n1 + 2 ng)
  int axis2;           // x^2 is a polar-axis direction (edges on the axis are 0)
  long tab_plane;      // metric table component stride
  __host__ __device__ long idx(int i, int j, int k) const {
    return off + (long)k * plane + (long)j * pitch + i;
  }
  __host__ __device__ long stride(int d) const { return d == 0 ? 1L : (d == 1 ? pitch : plane); }
  __host__ __device__ long tidx(int i, int j) const {
    return (long)(j + ng) * tab_n1 + (i + ng);
  }
  // Faces and edges are formed at stored indices face_lo() .. n + face_lo()
  // + face_count - 1 along their offset directions: the ones the staggered
  // derivative reads at the interior, -3 .. n+1 for the sixth order and
  // -2 .. n for the fourth (whose grids may then have four ghost layers).
  __host__ __device__ int face_lo() const { return dorder == 4 ? -2 : -3; }
  __host__ __device__ int face_count(int d) const { return n[d] - 2 * face_lo() - 1; }
};

// ------------------------------------------------------------------ XCD-aware block order
// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8),
// each with its own L2.  Remapping b so that every XCD works on one contiguous
// range of the flattened index space keeps the stencil neighbours of a block
// (the rows and planes around it) in the same L2.  A bijection on [0, nb).
constexpr unsigned NXCD = 8;
#if defined(__HIPCC__)
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
#ifdef GRMHD_NO_XCD_REMAP
  (void)nb;
  return b;
#else
  const unsigned x = b % NXCD, q = b / NXCD;
  const unsigned per = nb / NXCD, rem = nb % NXCD;
  return x * per + (x < rem ? x : rem) + q;
#endif
}
__device__ __forceinline__ long flat_thread() {
  return (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}
#endif

// ------------------------------------------------------------------ MP5
// Word holding the sign bit (bit 31) of a float or double.
GR_HD int sign_word(double a) { return (int)(__builtin_bit_cast(unsigned long long, a) >> 32); }
GR_HD int sign_word(float a) { return __builtin_bit_cast(int, a); }

// minmod(a, b) = (sgn a + sgn b)/2 min(|a|, |b|): zero unless a and b have
// the same sign, else the argument nearer zero.  Written as
// max(min(a, b), 0) + min(max(a, b), 0): one of the two terms is always zero,
// so the sum is exact, and it takes four min/max and an add instead of
// compares, sign-bit logic and selects (the result can differ only in the
// sign of a zero).
template <typename T>
GR_HD T minmod(T a, T b) {
  return fmax(fmin(a, b), T(0)) + fmin(fmax(a, b), T(0));
}

// Four-argument minmod: min |.| with the common sign, zero without one; the
// same construction on the smallest and largest argument.
template <typename T>
GR_HD T minmod4(T w, T x, T y, T z) {
  const T lo = fmin(fmin(w, x), fmin(y, z)), hi = fmax(fmax(w, x), fmax(y, z));
  return fmax(lo, T(0)) + fmin(hi, T(0));
}

// Monotonicity-preserving limit (Suresh & Huynh 1997) of an unlimited value
// ql at the face between q0 and qp1, from q_{j-2..j+2}; the same limiter
// serves the fifth- and the seventh-order interpolant.
template <typename T>
GR_HD T mp_limit(T ql, T qm2, T qm1, T q0, T qp1, T qp2) {
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
  // max(min(q0, qp1, qmd), min(q0, qul, qlc)) and its mirror, with q0
  // factored out (min distributes over max): the same values, fewer operations
  const T qmin = fmin(q0, fmax(fmin(qp1, qmd), fmin(qul, qlc)));
  const T qmax = fmax(q0, fmin(fmax(qp1, qmd), fmax(qul, qlc)));
  // median(ql, qmin, qmax), written in the scheme as ql + minmod(qmin - ql,
  // qmax - ql); both bounding intervals contain q0, so qmin <= qmax and the
  // median is the clamp (equal up to the rounding of ql + (qmin - ql)).
  return fmin(fmax(ql, qmin), qmax);
}

// Limited left state at the face between q0 and qp1 from q_{j-2..j+2}.
template <typename T>
GR_HD T mp5(T qm2, T qm1, T q0, T qp1, T qp2) {
  // interpolant (3, -20, 90, 60, -5)/128 with the power-of-two scale folded
  // into the weights (the same value: scaling by 2^-7 commutes with rounding)
  const T ql = T(3.0 / 128) * qm2 - T(20.0 / 128) * qm1 + T(90.0 / 128) * q0 +
               T(60.0 / 128) * qp1 - T(5.0 / 128) * qp2;
  return mp_limit(ql, qm2, qm1, q0, qp1, qp2);
}

// MP7: the degree-6 interpolant of q_{j-3..j+3} at the face,
// (-5, 42, -175, 700, 525, -70, 7)/1024 (power-of-two scale folded into the
// weights), limited as MP5.
template <typename T>
GR_HD T mp7(T qm3, T qm2, T qm1, T q0, T qp1, T qp2, T qp3) {
  const T ql = T(-5.0 / 1024) * qm3 + T(42.0 / 1024) * qm2 - T(175.0 / 1024) * qm1 +
               T(700.0 / 1024) * q0 + T(525.0 / 1024) * qp1 - T(70.0 / 1024) * qp2 +
               T(7.0 / 1024) * qp3;
  return mp_limit(ql, qm2, qm1, q0, qp1, qp2);
}

// Left and right states at face f+1/2 from the six cells f-2 .. f+3 (c[0..5]).
template <typename T>
GR_HD void mp5_lr(const T c[6], T& l, T& r) {
  l = mp5(c[0], c[1], c[2], c[3], c[4]);
  r = mp5(c[5], c[4], c[3], c[2], c[1]);
}

// WENO5 in point-value form (Jiang & Shu 1996 smoothness indicators): the
// three quadratic interpolants at the face, combined with the weights
// d_k / (eps + beta_k)^2 normalised, d = (1, 10, 5)/16 (whose linear
// combination is the degree-4 interpolant above), eps = 1e-6.  Written with
// one division: w_k p_k summed over the common denominator.
template <typename T>
GR_HD T weno5(T qm2, T qm1, T q0, T qp1, T qp2) {
  const T p0 = T(3.0 / 8) * qm2 - T(10.0 / 8) * qm1 + T(15.0 / 8) * q0;
  const T p1 = T(-1.0 / 8) * qm1 + T(6.0 / 8) * q0 + T(3.0 / 8) * qp1;
  const T p2 = T(3.0 / 8) * q0 + T(6.0 / 8) * qp1 - T(1.0 / 8) * qp2;
  const T c0 = qm2 - T(2) * qm1 + q0, e0 = qm2 - T(4) * qm1 + T(3) * q0;
  const T c1 = qm1 - T(2) * q0 + qp1, e1 = qm1 - qp1;
  const T c2 = q0 - T(2) * qp1 + qp2, e2 = T(3) * q0 - T(4) * qp1 + qp2;
  const T s0 = T(1e-6) + T(13.0 / 12) * c0 * c0 + T(0.25) * e0 * e0;
  const T s1 = T(1e-6) + T(13.0 / 12) * c1 * c1 + T(0.25) * e1 * e1;
  const T s2 = T(1e-6) + T(13.0 / 12) * c2 * c2 + T(0.25) * e2 * e2;
  // alpha_k = d_k / s_k^2; multiply numerator and denominator by (s0 s1 s2)^2
  const T q0s = s0 * s0, q1s = s1 * s1, q2s = s2 * s2;
  const T a0 = T(1.0 / 16) * (q1s * q2s), a1 = T(10.0 / 16) * (q0s * q2s), a2 = T(5.0 / 16) * (q0s * q1s);
  return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

// PLM with the monotonized-central limiter (van Leer 1977): the cell value
// plus half the slope minmod(2 dl, 2 dr, (dl + dr)/2).
template <typename T>
GR_HD T plm_mc(T qm1, T q0, T qp1) {
  const T dl = q0 - qm1, dr = qp1 - q0;
  const T m = fmin(fmin(fabs(dl + dl), fabs(dr + dr)), fabs(T(0.5) * (dl + dr)));
  const int sl = sign_word(dl), sr = sign_word(dr);
  // same sign and neither zero (a zero difference gives m = 0 anyway)
  const T slope = (sl ^ sr) >= 0 ? (sl < 0 ? -m : m) : T(0);
  return q0 + T(0.5) * slope;
}

// Interface reconstructions: RECON_MP5 (default), RECON_WENO5, RECON_PLM,
// RECON_MP7; RECON_PCM (the cell values themselves, first order) is internal:
// the lower-order fallback's face fluxes.
constexpr int RECON_MP5 = 0, RECON_WENO5 = 1, RECON_PLM = 2, RECON_MP7 = 3, RECON_PCM = 4;

// Cells a reconstruction reads for face f+1/2: W cells f-LO .. f-LO+W-1
// (both states); cell f is c[LO], cell f+1 is c[LO+1].
template <int RC> struct Stencil { static constexpr int W = 6, LO = 2; };
template <> struct Stencil<RECON_MP7> { static constexpr int W = 8, LO = 3; };
template <> struct Stencil<RECON_PCM> { static constexpr int W = 2, LO = 0; };

template <int RC, typename T>
GR_HD void recon_lr(const T c[Stencil<RC>::W], T& l, T& r) {
  if constexpr (RC == RECON_MP7) {
    l = mp7(c[0], c[1], c[2], c[3], c[4], c[5], c[6]);
    r = mp7(c[7], c[6], c[5], c[4], c[3], c[2], c[1]);
  } else if constexpr (RC == RECON_WENO5) {
    l = weno5(c[0], c[1], c[2], c[3], c[4]);
    r = weno5(c[5], c[4], c[3], c[2], c[1]);
  } else if constexpr (RC == RECON_PLM) {
    l = plm_mc(c[1], c[2], c[3]);
    r = plm_mc(c[4], c[3], c[2]);
  } else if constexpr (RC == RECON_PCM) {
    l = c[0];
    r = c[1];
  } else {
    mp5_lr(c, l, r);
  }
}

// ------------------------------------------------------------------ FD operators
// Sixth-order staggered derivative at m from f_{m-5/2..m+5/2} = f[0..5]
// (stored indices m-3 .. m+2).
GR_HD double fd_deriv(const double f[6], double inv_dx) {
  return (75.0 / 64.0 * (f[3] - f[2]) - 25.0 / 384.0 * (f[4] - f[1]) +
          3.0 / 640.0 * (f[5] - f[0])) * inv_dx;
}
GR_HD double fd_interp(const double f[6]) {
  return (150.0 * (f[3] + f[2]) - 25.0 * (f[4] + f[1]) + 3.0 * (f[5] + f[0])) * (1.0 / 256.0);
}
// Order DO = 6 (above) or 4: the fourth-order members keep only the first
// correction, D4 = [27/24 (f_{+1/2} - f_{-1/2}) - 1/24 (f_{+3/2} - f_{-3/2})] / dx
// and I4 = [9 (f_{+1/2} + f_{-1/2}) - (f_{+3/2} + f_{-3/2})] / 16 (f[1..4]).
template <int DO>
GR_HD double fd_deriv_o(const double f[6], double inv_dx) {
  if constexpr (DO == 4)
    return (27.0 / 24.0 * (f[3] - f[2]) - 1.0 / 24.0 * (f[4] - f[1])) * inv_dx;
  else
    return fd_deriv(f, inv_dx);
}
template <int DO>
GR_HD double fd_interp_o(const double f[6]) {
  if constexpr (DO == 4)
    return (9.0 * (f[3] + f[2]) - (f[4] + f[1])) * (1.0 / 16.0);
  else
    return fd_interp(f);
}
// Run-time order (the grid's), for kernels outside the update.  Both values
// are formed and one is selected: a branch here kept the compiler from
// issuing all stencil loads of the inversion's centred field up front
// (inversion 14 % slower).
GR_HD double fd_deriv_rt(const double f[6], double inv_dx, int order) {
  const double d4 = fd_deriv_o<4>(f, inv_dx), d6 = fd_deriv(f, inv_dx);
  return order == 4 ? d4 : d6;
}
GR_HD double fd_interp_rt(const double f[6], int order) {
  const double i4 = fd_interp_o<4>(f), i6 = fd_interp(f);
  return order == 4 ? i4 : i6;
}

// ------------------------------------------------------------------ metric policies
template <typename T>
struct FlatMet {
  static constexpr bool flat = true;
  GR_HD void lower(const T a[3], T o[3]) const { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }
  GR_HD void raise(const T a[3], T o[3]) const { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }
  GR_HD T guu(int) const { return T(1); }
  GR_HD T tvel(T v, int) const { return v; }             // alpha v - beta
  GR_HD T dens(T x) const { return x; }                 // sqrt(gamma) x
  GR_HD T undens(T x) const { return x; }
  GR_HD T fcomb(T x, T y, int) const { return x; }      // sqrt(g)(alpha x - beta^d y)
  GR_HD T alpha() const { return T(1); }
  GR_HD T beta(int) const { return T(0); }
  GR_HD T sqrtg() const { return T(1); }
  GR_HD T e_up(T x) const { return x; }                 // x / sqrt(gamma)
  GR_HD T e_lo(T x) const { return x; }                 // x * sqrt(gamma)
};

template <typename T>
struct TabMet {
  static constexpr bool flat = false;
  T al, b[3], g11, g12, g13, g22, g23, g33, u11, u12, u13, u22, u23, u33, sg;
  GR_HD void load(const double* __restrict__ tab, long tplane, int loc, long t) {
    const double* p = tab + (long)loc * NGEOM * tplane + t;
    al = T(p[M_AL * tplane]);
    b[0] = T(p[M_B1 * tplane]); b[1] = T(p[M_B2 * tplane]); b[2] = T(p[M_B3 * tplane]);
    g11 = T(p[M_G11 * tplane]); g12 = T(p[M_G12 * tplane]); g13 = T(p[M_G13 * tplane]);
    g22 = T(p[M_G22 * tplane]); g23 = T(p[M_G23 * tplane]); g33 = T(p[M_G33 * tplane]);
    u11 = T(p[M_U11 * tplane]); u12 = T(p[M_U12 * tplane]); u13 = T(p[M_U13 * tplane]);
    u22 = T(p[M_U22 * tplane]); u23 = T(p[M_U23 * tplane]); u33 = T(p[M_U33 * tplane]);
    sg = T(p[M_SG * tplane]);
  }
  GR_HD void lower(const T a[3], T o[3]) const {
    o[0] = g11 * a[0] + g12 * a[1] + g13 * a[2];
    o[1] = g12 * a[0] + g22 * a[1] + g23 * a[2];
    o[2] = g13 * a[0] + g23 * a[1] + g33 * a[2];
  }
  GR_HD void raise(const T a[3], T o[3]) const {
    o[0] = u11 * a[0] + u12 * a[1] + u13 * a[2];
    o[1] = u12 * a[0] + u22 * a[1] + u23 * a[2];
    o[2] = u13 * a[0] + u23 * a[1] + u33 * a[2];
  }
  GR_HD T guu(int d) const { return d == 0 ? u11 : (d == 1 ? u22 : u33); }
  GR_HD T tvel(T v, int d) const { return al * v - b[d]; }
  GR_HD T dens(T x) const { return sg * x; }
  GR_HD T undens(T x) const { return x / sg; }
  GR_HD T fcomb(T x, T y, int d) const { return sg * (al * x - b[d] * y); }
  GR_HD T alpha() const { return al; }
  GR_HD T beta(int d) const { return b[d]; }
  GR_HD T sqrtg() const { return sg; }
  GR_HD T e_up(T x) const { return x / sg; }
  GR_HD T e_lo(T x) const { return sg * x; }
};

// ------------------------------------------------------------------ pointwise physics
template <typename T>
struct PState {
  T rho, p, u[3], B[3];
  T W, v[3], vl[3], v2, Bl[3], B2, vB, E2, rhoh, y, D, S[3], Su[3], tau;
};

// Derived quantities of a primitive state (3+1 GRMHD, ideal gas).
template <typename T, class M>
GR_HD void make_state(PState<T>& s, const M& m, T gam) {
  T ul[3];
  m.lower(s.u, ul);
  const T uu = ul[0] * s.u[0] + ul[1] * s.u[1] + ul[2] * s.u[2];
  const T w2 = T(1) + uu;   // W^2
  const T iw = rsqrt(w2);   // 1/W: one reciprocal square root, no division
  s.W = w2 * iw;
  for (int i = 0; i < 3; ++i) { s.v[i] = s.u[i] * iw; s.vl[i] = ul[i] * iw; }
  s.v2 = uu * (iw * iw);   // u^2 / W^2
  m.lower(s.B, s.Bl);
  s.B2 = s.Bl[0] * s.B[0] + s.Bl[1] * s.B[1] + s.Bl[2] * s.B[2];
  s.vB = s.vl[0] * s.B[0] + s.vl[1] * s.B[1] + s.vl[2] * s.B[2];
  s.E2 = s.B2 * s.v2 - s.vB * s.vB;
  // rho h = rho + Gamma p / (Gamma - 1): the ratio Gamma / (Gamma - 1) is the
  // same for every state of a call, so no per-state division
  s.rhoh = s.rho + gam / (gam - T(1)) * s.p;
  s.y = s.rhoh * w2;
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
GR_HD void cons_of(const PState<T>& s, const M& m, T c[5]) {
  c[0] = m.dens(s.D);
  c[1] = m.dens(s.S[0]); c[2] = m.dens(s.S[1]); c[3] = m.dens(s.S[2]);
  c[4] = m.dens(s.tau);
}

// Densitised fluxes of (D, S_1..3, tau) in direction d.
template <typename T, class M>
GR_HD void flux_of(const PState<T>& s, const M& m, int d, T f[5]) {
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
GR_HD void speeds_of(const PState<T>& s, const M& m, int d, T gam, T& lp, T& lm) {
  // a^2 = c_s^2 + v_A^2 - c_s^2 v_A^2 with c_s^2 = Gamma p / (rho h) and
  // v_A^2 = b^2 / (rho h + b^2) is exactly (Gamma p + b^2) / (rho h + b^2),
  // and 1 - a^2 = (rho h - Gamma p) / (rho h + b^2): one division for both
  const T gp = gam * s.p;
  const T bb = s.B2 * (T(1) - s.v2) + s.vB * s.vB;   // b^2 = B^2/W^2 + (v.B)^2
  const T ib = T(1) / (s.rhoh + bb);
  const T a2 = (gp + bb) * ib;
  const T one_a2 = (s.rhoh - gp) * ib;
  const T vd = s.v[d];
  const T den = T(1) - s.v2 * a2;
  T rad = a2 * (T(1) - s.v2) * (m.guu(d) * den - vd * vd * one_a2);
  rad = sqrt(fmax(rad, T(0)));
  const T fac = m.alpha() / den;
  const T base = vd * one_a2;
  if (M::flat) {
    lp = fac * (base + rad);
    lm = fac * (base - rad);
  } else {
    lp = fac * (base + rad) - m.beta(d);
    lm = fac * (base - rad) - m.beta(d);
  }
}

// Threshold below which a+ + a- counts as zero.
template <typename T> struct TinySpeed { static GR_HD double v() { return 1e-300; } };
template <> struct TinySpeed<float> { static GR_HD float v() { return 1e-37f; } };
template <typename T> GR_HD T tiny_speed() { return T(TinySpeed<T>::v()); }

template <typename T>
GR_HD T hll(T fl, T fr, T ul, T ur, T ap, T am, T inv_s, bool tiny) {
  return tiny ? T(0.5) * (fl + fr) : (ap * fl + am * fr - ap * am * (ur - ul)) * inv_s;
}

// ------------------------------------------------------------------ per-face body
constexpr double POS_FRAC = 0.1;
// qs(v, s): cell f-LO+s (s = 0 .. W-1, Stencil<RC>) of reconstructed
// variable v (rho, p, u^1, u^2, u^3, B^{d+1}, B^{d+2}), read when its
// reconstruction needs it (a caller staging the cells in LDS then holds one
// variable's cells in registers at a time instead of all 7 W).
template <int DIR, int RC = RECON_MP5, typename T, class M, class QS>
GR_HD void face_body_q(const QS& qs, T bn, bool axis, const M& m, T gam, T fh[5], T ctd[6]) {
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  constexpr int W = Stencil<RC>::W, LO = Stencil<RC>::LO;
  PState<T> sl, sr;
  auto rec = [&](int v, T& l, T& r) {
    T c[W];
#pragma unroll
    for (int s = 0; s < W; ++s) c[s] = qs(v, s);
    recon_lr<RC>(c, l, r);
  };
  // rho and p states are kept at or above POS_FRAC times the cell value on
  // their side of the face (a continuous positivity bound)
  rec(0, sl.rho, sr.rho);
  sl.rho = fmax(sl.rho, T(POS_FRAC) * qs(0, LO));
  sr.rho = fmax(sr.rho, T(POS_FRAC) * qs(0, LO + 1));
  rec(1, sl.p, sr.p);
  sl.p = fmax(sl.p, T(POS_FRAC) * qs(1, LO));
  sr.p = fmax(sr.p, T(POS_FRAC) * qs(1, LO + 1));
  rec(2, sl.u[0], sr.u[0]);
  rec(3, sl.u[1], sr.u[1]);
  rec(4, sl.u[2], sr.u[2]);
  rec(5, sl.B[T1], sr.B[T1]);
  rec(6, sl.B[T2], sr.B[T2]);
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
  for (int q5 = 0; q5 < 5; ++q5) {
    T f = hll(fl[q5], fr[q5], ul[q5], ur[q5], ap, am, inv_s, tiny);
    fh[q5] = axis ? T(0) : f;
  }
  ctd[0] = sl.v[DIR];
  ctd[1] = sr.v[DIR];
  ctd[2] = sl.v[T1];
  ctd[3] = sr.v[T1];
  ctd[4] = ap;
  ctd[5] = am;
}

// q[v][s]: the cells f-LO .. f-LO+W-1 of the reconstructed variables in the
// order rho, p, u^1, u^2, u^3, B^{d+1}, B^{d+2}; bn: normal B at the face.
template <int DIR, int RC = RECON_MP5, typename T, class M>
GR_HD void face_body(const T q[7][Stencil<RC>::W], T bn, bool axis, const M& m, T gam, T fh[5],
                     T ctd[6]) {
  face_body_q<DIR, RC>([&](int v, int s) { return q[v][s]; }, bn, axis, m, gam, fh, ctd);
}

// ------------------------------------------------------------------ per-edge body
// Edge field of family E (d = E+1, c = E+2 mod 3).  qd[v][s]: W d-faces
// along c (Stencil<RC>) of v^d_L, v^d_R, v^c_L, v^c_R, B^d; qc[s]: W
// c-faces along d of B^c; a*: speeds of the two adjacent faces of each
// family.  qds(v, s) returns qd[v][s], read when its reconstruction needs it
// (for a caller that stages qd in LDS: one variable's cells in registers at
// a time).
template <int E, int RC = RECON_MP5, typename T, class M, class QD>
GR_HD T edge_body_q(const QD& qds, const T qc[Stencil<RC>::W], T apd0, T apd1, T amd0, T amd1,
                    T apc0, T apc1, T amc0, T amc1, const M& m) {
  constexpr int D = (E + 1) % 3, C = (E + 2) % 3;
  constexpr int W = Stencil<RC>::W;
  T vd[2][2], vc[2][2], bd[2], bc[2];   // [a][b]
  auto rec = [&](int v, T& l, T& r) {
    T c[W];
#pragma unroll
    for (int s = 0; s < W; ++s) c[s] = qds(v, s);
    recon_lr<RC>(c, l, r);
  };
  rec(0, vd[0][0], vd[0][1]);
  rec(1, vd[1][0], vd[1][1]);
  rec(2, vc[0][0], vc[0][1]);
  rec(3, vc[1][0], vc[1][1]);
  rec(4, bd[0], bd[1]);
  recon_lr<RC>(qc, bc[0], bc[1]);
  const T apd = fmax(apd0, apd1), amd = fmax(amd0, amd1);
  const T apc = fmax(apc0, apc1), amc = fmax(amc0, amc1);
  const T sdd = apd + amd, scc = apc + amc;
  const bool tiny_d = sdd < tiny_speed<T>(), tiny_c = scc < tiny_speed<T>();
  const T isd = tiny_d ? T(0) : T(1) / sdd;
  const T isc = tiny_c ? T(0) : T(1) / scc;
  const T wd[2] = {tiny_d ? T(0.5) : apd * isd, tiny_d ? T(0.5) : amd * isd};
  const T wc[2] = {tiny_c ? T(0.5) : apc * isc, tiny_c ? T(0.5) : amc * isc};
  const T kd = tiny_d ? T(0) : apd * amd * isd;
  const T kc = tiny_c ? T(0) : apc * amc * isc;
  T ee = T(0);
  for (int a = 0; a < 2; ++a) {
    for (int bb = 0; bb < 2; ++bb) {
      const T vtd = m.tvel(vd[a][bb], D);
      const T vtc = m.tvel(vc[a][bb], C);
      const T eab = vtc * bd[bb] - vtd * bc[a];
      ee = ee + wd[a] * wc[bb] * eab;
    }
  }
  ee = ee + kd * (bc[1] - bc[0]) - kc * (bd[1] - bd[0]);
  return ee;
}

template <int E, int RC = RECON_MP5, typename T, class M>
GR_HD T edge_body(const T qd[5][Stencil<RC>::W], const T qc[Stencil<RC>::W], T apd0, T apd1,
                  T amd0, T amd1, T apc0, T apc1, T amc0, T amc1, const M& m) {
  return edge_body_q<E, RC>([&](int v, int s) { return qd[v][s]; }, qc, apd0, apd1, amd0, amd1, apc0,
                            apc1, amc0, amc1, m);
}

// ------------------------------------------------------------------ inversion
template <typename T>
struct NewtonOut {
  T rho, p, u[3];
  int iters;
  bool ok;
  bool alt;       // the iteration started from y_alt
  bool deferred;  // stopped early: first residual (defer_tol) or split_it iterations
  T y_last;       // the iterate when deferred by split_it
};

// Safeguarded Newton inversion in y = rho h W^2 (undensitised D, S_i, tau, B^i).
// y_alt > 0: a second candidate start; the iteration starts from whichever of
// y0 and y_alt has the smaller |residual| (one extra residual evaluation).
// defer_tol > 0: when the first residual, relative to the magnitude of its
// terms, exceeds defer_tol (or v^2 >= 1 there), stop at once with
// deferred = true and nothing else set.
// split_it > 0: a zone not converged after split_it iterations stops with
// deferred = true, iters = split_it and its current iterate in y_last (a
// later pass finishes it from there).
template <typename T, class MET>
GR_HD NewtonOut<T> newton(T dd, const T S[3], T tau, const T B[3], const MET& m, T gam,
                          T y0, double tol, int maxit, T y_alt = T(-1), double defer_tol = 0.0,
                          int split_it = 0) {
  using std::isfinite;
  NewtonOut<T> o;
  const T utot = tau + dd;
  T su[3], bl[3];
  m.raise(S, su);
  m.lower(B, bl);
  const T s2 = S[0] * su[0] + S[1] * su[1] + S[2] * su[2];
  const T b2 = bl[0] * B[0] + bl[1] * B[1] + bl[2] * B[2];
  const T sb = S[0] * B[0] + S[1] * B[1] + S[2] * B[2];
  const T sb2 = sb * sb;
  const T gf = (gam - 1.0) / gam;
  const bool valid = isfinite(dd) && isfinite(utot) && isfinite(s2) && isfinite(b2) &&
                     isfinite(sb) && dd > 0.0 && utot > 0.0;
  T a = 0.0, bb = gam * utot;
  T y = y0;
  if (!(y > a && y < bb)) y = 0.5 * (a + bb);
  o.alt = false;
  o.deferred = false;
  if (valid && y_alt > a && y_alt < bb) {
    // residual of the energy equation at a candidate start; +inf where v^2 >= 1
    auto resid = [&](T yc) {
      const T yy = yc * yc;
      const T v2 = (s2 + sb2 * (2.0 * yc + b2) / yy) / ((yc + b2) * (yc + b2));
      if (!(v2 < 1.0)) return T(INFINITY);
      const T p = gf * (yc * (1.0 - v2) - dd * sqrt(1.0 - v2));
      return fabs(yc - p + 0.5 * b2 * (1.0 + v2) - 0.5 * sb2 / yy - utot);
    };
    if (resid(y_alt) < resid(y)) {
      y = y_alt;
      o.alt = true;
    }
  }
  bool conv = false;
  int it = 0;
  const T EPS4 = T(4.0 * 2.220446049250313e-16);
  if (valid) {
    for (; it < maxit;) {
      if (split_it > 0 && it == split_it) {
        o.deferred = true;
        o.ok = false;
        o.iters = it;
        o.y_last = y;
        return o;
      }
      ++it;
      // two reciprocals and a reciprocal square root per iteration (1/y,
      // 1/(y + B^2), 1/sqrt(1 - v^2), with sqrt(1 - v^2) = (1 - v^2) / sqrt(1 - v^2));
      // the expressions are those of the residual and its derivative
      const T iy = 1.0 / y, iy2 = iy * iy;
      const T yb = y + b2, iyb = 1.0 / yb, iyb2 = iyb * iyb;
      const T num = s2 + sb2 * (2.0 * y + b2) * iy2;
      const T v2 = num * iyb2;
      const bool bad = v2 >= 1.0;
      const T omv = 1.0 - v2;
      const T isq = rsqrt(omv);
      const T sq = omv * isq;
      const T p = gf * (y * (1.0 - v2) - dd * sq);
      const T f = y - p + 0.5 * b2 * (1.0 + v2) - 0.5 * sb2 * iy2 - utot;
      const T dv2 = -2.0 * iyb * (sb2 * iy2 * iy + num * iyb2);
      const T dp = gf * ((1.0 - v2) - y * dv2 + 0.5 * dd * dv2 * isq);
      const T fp = 1.0 - dp + 0.5 * b2 * dv2 + sb2 * iy2 * iy;
      const T fabs_ = y + fabs(p) + 0.5 * b2 * (1.0 + v2) + 0.5 * sb2 * iy2 + utot;
      if (defer_tol > 0.0 && it == 1 && (bad || !(fabs(f) <= T(defer_tol) * fabs_))) {
        o.deferred = true;
        o.ok = false;
        o.iters = 0;
        return o;
      }
      if (!bad && fabs(f) <= EPS4 * fabs_) { conv = true; break; }
      const bool below = bad || (f < 0.0);
      if (below) a = y; else bb = y;
      T yn = y - f / fp;
      if (bad || !(yn >= a && yn <= bb)) yn = 0.5 * (a + bb);
      const T dy = yn - y;
      y = yn;
      if (fabs(dy) <= tol * y) { conv = true; break; }
    }
  }
  // primitives at the root: W = 1/sqrt(1 - v^2), rho = D/W, p from the
  // equation of state, v_i = (S_i + (S.B) B_i / y) / (y + B^2); two
  // reciprocals and a reciprocal square root
  const T iy = 1.0 / y, iyb = 1.0 / (y + b2);
  const T v2 = (s2 + sb2 * (2.0 * y + b2) * (iy * iy)) * (iyb * iyb);
  const T omv = 1.0 - v2;
  const T w = rsqrt(omv);
  const T sq = omv * w;                         // sqrt(1 - v^2) = 1/W
  o.p = gf * (y * omv - dd * sq);
  o.rho = dd * sq;
  T vl[3], vu[3];
  const T sby = sb * iy;
  for (int q = 0; q < 3; ++q) vl[q] = (S[q] + sby * bl[q]) * iyb;
  m.raise(vl, vu);
  for (int q = 0; q < 3; ++q) o.u[q] = w * vu[q];
  o.ok = conv && valid && (v2 < 1.0) && isfinite(o.rho) && isfinite(o.p) && isfinite(o.u[0]) &&
         isfinite(o.u[1]) && isfinite(o.u[2]);
  o.iters = it;
  return o;
}

}  // namespace grmhd
