// Operation-count harness (host).  Runs the kernels' own per-face, per-edge
// and per-zone bodies (the __host__ __device__ functions of grmhd_device.hpp)
// with a counting number type on a periodic box read from a file, and prints
// the mean number of FP64 operations per unit as JSON.  These are the
// algorithmic operation counts the benchmark's roofline uses.
//
// Input file (float64, little endian): n, then rho, u1, u2, u3, p on the n^3
// interior ([k][j][i]), then A1, A2, A3 on the (n+10)^3 ghosted edge grid.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

struct OpStats {
  long long add = 0, mul = 0, div = 0, sqrt = 0, minmax = 0, cmp = 0;
  long long flops() const { return add + mul + div + sqrt; }
};
static OpStats g_ops;

struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}
  explicit operator double() const { return v; }
  Cnt& operator+=(Cnt o) { g_ops.add++; v += o.v; return *this; }
  Cnt& operator-=(Cnt o) { g_ops.add++; v -= o.v; return *this; }
  Cnt& operator*=(Cnt o) { g_ops.mul++; v *= o.v; return *this; }
};
inline Cnt operator+(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { g_ops.mul++; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { g_ops.div++; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline bool operator<(Cnt a, Cnt b) { g_ops.cmp++; return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { g_ops.cmp++; return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { g_ops.cmp++; return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { g_ops.cmp++; return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { g_ops.cmp++; return a.v == b.v; }
inline Cnt sqrt(Cnt a) { g_ops.sqrt++; return Cnt(std::sqrt(a.v)); }
// reciprocal square root: one square root and one division in the count
inline Cnt rsqrt(Cnt a) { g_ops.sqrt++; g_ops.div++; return Cnt(1.0 / std::sqrt(a.v)); }
// plain double (states built without counting): the host has no rsqrt
inline double rsqrt(double a) { return 1.0 / std::sqrt(a); }
inline Cnt fmin(Cnt a, Cnt b) { g_ops.minmax++; return Cnt(std::fmin(a.v, b.v)); }
inline Cnt fmax(Cnt a, Cnt b) { g_ops.minmax++; return Cnt(std::fmax(a.v, b.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline bool isfinite(Cnt a) { return std::isfinite(a.v); }
// sign-bit test of the limiters: integer work, not counted
inline int sign_word(Cnt a) { return (int)(__builtin_bit_cast(unsigned long long, a.v) >> 32); }

#include "grmhd_device.hpp"

using namespace grmhd;

namespace {
int N, NT;   // interior and ghosted extent
inline long id(int i, int j, int k) { return ((long)(k + NG) * NT + (j + NG)) * NT + (i + NG); }
inline int wrap(int m) { int r = m % N; return r < 0 ? r + N : r; }
long strd(int d) { return d == 0 ? 1L : (d == 1 ? (long)NT : (long)NT * NT); }

void fill_periodic(std::vector<double>& a) {
  for (int k = -NG; k < N + NG; ++k)
    for (int j = -NG; j < N + NG; ++j)
      for (int i = -NG; i < N + NG; ++i)
        a[id(i, j, k)] = a[id(wrap(i), wrap(j), wrap(k))];
}

struct Acc {
  OpStats tot;
  long long units = 0;
  void add(const OpStats& s) {
    tot.add += s.add; tot.mul += s.mul; tot.div += s.div; tot.sqrt += s.sqrt;
    tot.minmax += s.minmax; tot.cmp += s.cmp; units++;
  }
  void print(const char* name, double bytes, bool last = false) const {
    const double u = (double)units;
    std::printf("  \"%s\": {\"flops\": %.2f, \"add\": %.2f, \"mul\": %.2f, \"div\": %.3f, "
                "\"sqrt\": %.3f, \"minmax\": %.2f, \"cmp\": %.2f, \"bytes\": %.1f, \"units\": %lld}%s\n",
                name, tot.flops() / u, tot.add / u, tot.mul / u, tot.div / u, tot.sqrt / u,
                tot.minmax / u, tot.cmp / u, bytes, units, last ? "" : ",");
  }
};
}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) { std::fprintf(stderr, "usage: opcount input.bin\n"); return 2; }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) { std::perror("open"); return 2; }
  double nd;
  if (std::fread(&nd, 8, 1, f) != 1) return 2;
  N = (int)nd;
  NT = N + 2 * NG;
  const long vol = (long)NT * NT * NT, nin = (long)N * N * N;
  std::vector<std::vector<double>> P(8, std::vector<double>(vol, 0.0));
  std::vector<double> tmp(nin);
  const int order[5] = {P_RHO, P_U1, P_U2, P_U3, P_P};
  for (int q = 0; q < 5; ++q) {
    if (std::fread(tmp.data(), 8, nin, f) != (size_t)nin) return 2;
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) P[order[q]][id(i, j, k)] = tmp[((long)k * N + j) * N + i];
  }
  std::vector<std::vector<double>> A(3, std::vector<double>(vol));
  for (int q = 0; q < 3; ++q)
    if (std::fread(A[q].data(), 8, vol, f) != (size_t)vol) return 2;
  std::fclose(f);
  const double dx = 1.0 / N, gam = 4.0 / 3.0;
  // face fields from the potential, centred B (the library's own FD operators)
  std::vector<std::vector<double>> Bf(3, std::vector<double>(vol, 0.0));
  for (int nd3 = 0; nd3 < 3; ++nd3) {
    const int d1 = (nd3 + 1) % 3, d2 = (nd3 + 2) % 3;
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
          const long c = id(i, j, k);
          double a[6], b[6];
          for (int s = 0; s < 6; ++s) {
            a[s] = A[d2][c + (s - 3) * strd(d1)];
            b[s] = A[d1][c + (s - 3) * strd(d2)];
          }
          Bf[nd3][c] = fd_deriv(a, 1.0 / dx) - fd_deriv(b, 1.0 / dx);
        }
    fill_periodic(Bf[nd3]);
  }
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
          const long c = id(i, j, k);
          double a[6];
          for (int s = 0; s < 6; ++s) a[s] = Bf[d][c + (s - 3) * strd(d)];
          P[P_B1 + d][c] = fd_interp(a);
        }
  }
  for (int q = 0; q < 8; ++q) fill_periodic(P[q]);

  const FlatMet<Cnt> m;
  Acc face_acc[3], edge_acc[3], c2p_exact, c2p_warm;
  std::vector<std::vector<double>> ctd(18, std::vector<double>(vol, 0.0));
  // faces: d-index in [-3, N+1], transverse over the ghosted range
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    const int fields[7] = {P_RHO, P_P, P_U1, P_U2, P_U3, P_B1 + t1, P_B1 + t2};
    for (int a2 = -NG; a2 < N + NG; ++a2)
      for (int a1 = -NG; a1 < N + NG; ++a1)
        for (int fi = -3; fi <= N + 1; ++fi) {
          int ii[3];
          ii[d] = fi; ii[t1] = a1; ii[t2] = a2;
          const long c = id(ii[0], ii[1], ii[2]);
          Cnt q[7][6];
          for (int v = 0; v < 7; ++v)
            for (int s = 0; s < 6; ++s) q[v][s] = Cnt(P[fields[v]][c + (s - 2) * strd(d)]);
          Cnt fh[5], cd[6];
          g_ops = OpStats();
          if (d == 0) face_body<0>(q, Cnt(Bf[0][c]), false, m, Cnt(gam), fh, cd);
          if (d == 1) face_body<1>(q, Cnt(Bf[1][c]), false, m, Cnt(gam), fh, cd);
          if (d == 2) face_body<2>(q, Cnt(Bf[2][c]), false, m, Cnt(gam), fh, cd);
          face_acc[d].add(g_ops);
          for (int q6 = 0; q6 < 6; ++q6) ctd[d * 6 + q6][c] = cd[q6].v;
        }
  }
  // edges: d, c in [-3, N+1], e interior
  for (int e = 0; e < 3; ++e) {
    const int D = (e + 1) % 3, C = (e + 2) % 3;
    for (int ae = 0; ae < N; ++ae)
      for (int ac = -3; ac <= N + 1; ++ac)
        for (int ad = -3; ad <= N + 1; ++ad) {
          int ii[3];
          ii[e] = ae; ii[D] = ad; ii[C] = ac;
          const long b = id(ii[0], ii[1], ii[2]);
          const long sc = strd(C), sd = strd(D);
          Cnt qd[5][6], qc[6];
          for (int s = 0; s < 6; ++s) {
            for (int v = 0; v < 4; ++v) qd[v][s] = Cnt(ctd[D * 6 + v][b + (s - 2) * sc]);
            qd[4][s] = Cnt(Bf[D][b + (s - 2) * sc]);
            qc[s] = Cnt(Bf[C][b + (s - 2) * sd]);
          }
          g_ops = OpStats();
          Cnt r;
          const Cnt a0(ctd[D * 6 + 4][b]), a1(ctd[D * 6 + 4][b + sc]);
          const Cnt m0(ctd[D * 6 + 5][b]), m1(ctd[D * 6 + 5][b + sc]);
          const Cnt c0(ctd[C * 6 + 4][b]), c1(ctd[C * 6 + 4][b + sd]);
          const Cnt n0(ctd[C * 6 + 5][b]), n1(ctd[C * 6 + 5][b + sd]);
          if (e == 0) r = edge_body<0>(qd, qc, a0, a1, m0, m1, c0, c1, n0, n1, m);
          if (e == 1) r = edge_body<1>(qd, qc, a0, a1, m0, m1, c0, c1, n0, n1, m);
          if (e == 2) r = edge_body<2>(qd, qc, a0, a1, m0, m1, c0, c1, n0, n1, m);
          edge_acc[e].add(g_ops);
        }
  }
  // inversion: conserved state of each zone, exact and perturbed warm guesses
  long long it_exact = 0, it_warm = 0;
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const long c = id(i, j, k);
        PState<double> s;
        s.rho = P[P_RHO][c]; s.p = P[P_P][c];
        for (int q = 0; q < 3; ++q) { s.u[q] = P[P_U1 + q][c]; s.B[q] = P[P_B1 + q][c]; }
        const FlatMet<double> md;
        make_state(s, md, gam);
        const Cnt S[3] = {Cnt(s.S[0]), Cnt(s.S[1]), Cnt(s.S[2])};
        const Cnt B[3] = {Cnt(s.B[0]), Cnt(s.B[1]), Cnt(s.B[2])};
        g_ops = OpStats();
        NewtonOut<Cnt> r1 = newton<Cnt>(Cnt(s.D), S, Cnt(s.tau), B, m, Cnt(gam), Cnt(s.y), 1e-14, 50);
        c2p_exact.add(g_ops);
        it_exact += r1.iters;
        g_ops = OpStats();
        NewtonOut<Cnt> r2 = newton<Cnt>(Cnt(s.D), S, Cnt(s.tau), B, m, Cnt(gam), Cnt(s.y * (1.0 + 1e-3)), 1e-14, 50);
        c2p_warm.add(g_ops);
        it_warm += r2.iters;
      }
  const double z = (double)N * N * N;
  const double per_iter = ((double)c2p_warm.tot.flops() - c2p_exact.tot.flops()) / (it_warm - it_exact);
  const double fixed = c2p_exact.tot.flops() / z - per_iter * (it_exact / z);
  std::printf("{\n");
  std::printf("  \"workload\": \"turbulent SRMHD box %d^3 (seed 1810), flat metric, FP64\",\n", N);
  // compulsory HBM bytes per unit of each kernel (each operand read or written once)
  face_acc[0].print("sweep_x1", 8.0 * (8 + 11));
  face_acc[1].print("sweep_x2", 8.0 * (8 + 11));
  face_acc[2].print("sweep_x3", 8.0 * (8 + 11));
  edge_acc[0].print("edge_x1", 8.0 * (10 + 1));
  edge_acc[1].print("edge_x2", 8.0 * (10 + 1));
  edge_acc[2].print("edge_x3", 8.0 * (10 + 1));
  // stage 1 (a = 0) reads no U^n; stages 2 and 3 read it: mean over the three launches of a step
  std::printf("  \"update\": {\"bytes\": %.2f, \"note\": \"reads 15 fluxes, 3 edge fields and U^(s) (8); "
              "writes U^(s+1) (8); reads U^n (8) in stages 2 and 3 only; mean over the three stages "
              "(272, 336, 336)\"},\n",
              8.0 * (15 + 3 + 8 + 8) + 8.0 * 8 * 2.0 / 3.0);
  std::printf("  \"cons2prim\": {\"flops_fixed\": %.2f, \"flops_per_iter\": %.2f, \"iters_exact_guess\": %.3f, "
              "\"iters_guess_1e-3\": %.3f, \"bytes\": %.1f},\n",
              fixed, per_iter, it_exact / z, it_warm / z, 8.0 * (8 + 5 + 8));
  std::printf("  \"bc_centred\": {\"bytes_per_ghost_cell\": %.1f}\n", 8.0 * 16);
  std::printf("}\n");
  return 0;
}
