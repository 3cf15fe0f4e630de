// Face sweeps and constrained-transport edge fields (gfx950).
//
// k_sweep<DIR>: one thread per DIR-face, faces f in [-3, n_DIR + 1] ([-2, n_DIR]
// with the fourth-order derivative; Geom::face_lo) over the whole ghosted
// transverse range, flattened with x^1 fastest so a wavefront
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
// c = E+2 mod 3), over d, c in the face range and interior x^E: upwind
// constrained transport (Londrillo & Del Zanna 2004) from MP5 along c of the
// d-face velocities and B^d, MP5 along d of B^c, and the speeds of the two
// adjacent faces of each family.
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"

namespace grmhd {

// Lane map.  MP5's limiter branch is needed by a few percent of the
// reconstructions, and those cluster in space: a wavefront that spans one
// 64-position row almost always holds one of them and runs the branch for
// all its lanes, while a compact patch of the same 64 positions more often
// holds none and skips it.  So every kernel here hands each wavefront a patch
// of PX consecutive x^1 positions times PY rows of a second axis.
constexpr int PX = 16, PY = 64 / PX;

// Direct (unstaged) kernels: a 256-thread workgroup covers PX x^1 positions
// times 4 PY positions of the middle axis at one position of the slow axis;
// wavefront w owns middle-axis rows w PY .. w PY + PY - 1 of the tile.
// x^1 alignment: a row segment of PX = 16 doubles is one 128-byte line when
// it starts at a multiple of 16 in storage.  x^1 position a of a range whose
// first element sits `shift` doubles past such a line (rows start on one:
// the pitch is a multiple of 16) goes to lane slot a + shift, so every
// segment a wavefront loads or stores covers whole lines instead of
// straddling two; the slots before the range's start stay idle.
struct TilePos {
  int a, m, s;
  bool ok;
};
__device__ __forceinline__ TilePos tile_pos(int ext0, int extm, int shift) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const unsigned nt0 = (ext0 + shift + PX - 1) / PX, ntm = (extm + 4 * PY - 1) / (4 * PY);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  TilePos p;
  p.a = (int)(b % nt0) * PX + lane % PX - shift;
  const unsigned r = b / nt0;
  p.m = (int)(r % ntm) * (4 * PY) + w * PY + lane / PX;
  p.s = (int)(r / ntm);
  p.ok = p.a >= 0 && p.a < ext0 && p.m < extm;
  return p;
}
static inline unsigned tile_blocks(long ext0, long extm, long exts, int shift) {
  return (unsigned)(((ext0 + shift + PX - 1) / PX) * ((extm + 4 * PY - 1) / (4 * PY)) * exts);
}
// Offset (doubles past a 16-double line) of x^1 index i0 in storage.
__host__ __device__ __forceinline__ int line_shift(int ng, int i0) { return (ng + i0) & 15; }
// Line-aligned lane map per edge family: it pays where the kernel's x^1
// segments are both loaded and stored from a misaligned start (family 0,
// x^1 interior); families 1 and 2 (x^1 from -3) measured faster without it,
// their idle slots costing more than the straddled lines.
constexpr bool EDGE_ALIGN[3] = {true, false, false};

// Flattened map (x^1 fastest, then the middle axis): one 64-position row
// segment per wavefront, no idle lanes at the tile edges.  The x^1 sweep on
// a tabulated metric, whose faces also load their metric from table rows,
// measured faster with it.
__device__ __forceinline__ TilePos flat_pos(int ext0, int extm, int exts) {
  const long t = flat_thread();
  TilePos p;
  p.ok = t < (long)ext0 * extm * exts;
  const long tc = p.ok ? t : 0;
  p.a = (int)(tc % ext0);
  const long r = tc / ext0;
  p.m = (int)(r % extm);
  p.s = (int)(r / extm);
  return p;
}

template <int DIR, class MET, typename T, int RC>
__global__ __launch_bounds__(256) void k_sweep(Geom G, const double* __restrict__ prim,
                                               const double* __restrict__ cons,
                                               const double* __restrict__ tab,
                                               T* __restrict__ flux,
                                               T* __restrict__ ctd) {
  int ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ext[a] = (a == DIR) ? G.face_count(a) : G.dims[a];
  // tiles: x^1 fastest; for the x^3 sweep x^3 comes next, so the six planes
  // of a stencil are read by neighbouring workgroups (L2 reuse)
  constexpr int MID = DIR == 2 ? 2 : 1, SLOW = DIR == 2 ? 1 : 2;
  const TilePos tp = MET::flat ? tile_pos(ext[0], ext[MID], line_shift(G.ng, DIR == 0 ? G.face_lo() : -G.ng))
                               : flat_pos(ext[0], ext[MID], ext[SLOW]);
  if (!tp.ok) return;
  int ii[3];
  ii[0] = tp.a;
  ii[MID] = tp.m;
  ii[SLOW] = tp.s;
#pragma unroll
  for (int a = 0; a < 3; ++a) ii[a] += (a == DIR) ? G.face_lo() : -G.ng;
  const long c = G.idx(ii[0], ii[1], ii[2]);
  const long st = G.stride(DIR);
  const T gam = T(G.gam);
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  constexpr int W = Stencil<RC>::W, LO = Stencil<RC>::LO;

  // face metric: x^1 faces -> F1, x^2 faces -> F2, x^3 faces -> centre tables
  MET m;
  if constexpr (!MET::flat) {
    constexpr int loc = DIR == 0 ? LOC_F1 : (DIR == 1 ? LOC_F2 : LOC_C);
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }

  T q[7][W];
  {
    const int fields[7] = {P_RHO, P_P, P_U1, P_U2, P_U3, P_B1 + T1, P_B1 + T2};
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const double* p = prim + (long)fields[v] * G.field + c;
#pragma unroll
      for (int s = 0; s < W; ++s) q[v][s] = T(p[(s - LO) * st]);
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
  face_body<DIR, RC>(q, bn, axis, m, gam, fh, cd);
  // non-temporal stores: the eleven per-face results are read by later
  // launches, long after they would have left the cache (sweeps 3-5 % faster
  // than with ordinary stores; the edge field's single store, the update's
  // and the inversion's measured slower that way)
#pragma unroll
  for (int q5 = 0; q5 < 5; ++q5) __builtin_nontemporal_store(fh[q5], &flux[(long)q5 * G.field + c]);
#pragma unroll
  for (int q6 = 0; q6 < 6; ++q6) __builtin_nontemporal_store(cd[q6], &ctd[(long)q6 * G.field + c]);
}

// LDS-staged sweep for DIR = 1, 2 (stencils across rows or planes, which a
// wavefront would otherwise fetch as six separate row loads per variable).
// A workgroup owns SX consecutive transverse positions (flattened, x^1
// fastest) times SF consecutive faces along DIR; it stages the SF + W - 1 cells
// of each reconstructed variable its faces need in LDS, so each cell row is
// read once per workgroup, then each wavefront runs the per-face body on one
// face row.  Workgroups of one column follow each other along DIR.
// One wavefront per face row (SX = 64); SF face rows per workgroup.
constexpr int SX = 64;
constexpr int LPAD = 0;   // extra doubles per LDS row

template <int DIR, int SF, class MET, typename T, int RC>
__global__ __launch_bounds__(SX * SF) void k_sweep_lds(Geom G, const double* __restrict__ prim,
                                                   const double* __restrict__ cons,
                                                   const double* __restrict__ tab,
                                                   T* __restrict__ flux,
                                                   T* __restrict__ ctd) {
  static_assert(DIR == 1 || DIR == 2, "x^2 and x^3 sweeps only");
  constexpr int TB = DIR == 1 ? 2 : 1;          // the transverse axis other than x^1
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  constexpr int W = Stencil<RC>::W, LO = Stencil<RC>::LO;
  constexpr int SR = SF + W - 1, NRR = (SR + SF - 1) / SF;
  __shared__ T sh[7][SR][SX + LPAD];
  // transverse positions flattened with x^1 fastest over rows of the pitch
  // (a multiple of 16, so 16-lane segments are whole 128-byte lines); the
  // pitch's padding positions past the ghosted x^1 range stay idle
  const int nA = G.dims[0], rA = (int)G.pitch;
  const long M = (long)rA * G.dims[TB];
  const int nface = G.face_count(DIR);          // faces face_lo .. face_lo + nface - 1
  const int ntf = (nface + SF - 1) / SF;
  const long bid = xcd_block(blockIdx.x, gridDim.x);
  const int ft = (int)(bid % ntf);
  const long mt = bid / ntf;
  // ty (the face row) is the wavefront index: uniform, so row offsets go to the scalar unit
  const int tx = threadIdx.x % SX, ty = __builtin_amdgcn_readfirstlane(threadIdx.x / SX);
  const long mm = mt * SX + tx;
  const unsigned mc = (unsigned)(mm < M ? mm : M - 1);
  const int xa = (int)(mc % (unsigned)rA);
  const int ok = mm < M && xa < nA;                 // a position of the ghosted range
  int ii[3];
  ii[0] = min(xa, nA - 1) - G.ng;                   // clamped: every staging load is in bounds
  ii[TB] = (int)(mc / (unsigned)rA) - G.ng;
  ii[DIR] = 0;
  const long base = G.idx(ii[0], ii[1], ii[2]);
  const long st = G.stride(DIR);
  const int f0 = G.face_lo() + ft * SF;
  // stage cells f0 - LO .. f0 + SF - LO + W - 2; wavefront ty loads rows ty + SF rr
  // (a wave-uniform condition).  Rows past the last ghost cell are clamped to
  // it: no face of the tile that exists reads them.  All loads are issued
  // before the first LDS write.
  {
    constexpr int fields[7] = {P_RHO, P_P, P_U1, P_U2, P_U3, P_B1 + T1, P_B1 + T2};
    const int cmax = G.n[DIR] + G.ng - 1;
    const double* pb = prim + base;             // per lane; the offsets below are uniform
    T stage[7][NRR];
#pragma unroll
    for (int rr = 0; rr < NRR; ++rr) {
      if (ty + SF * rr < SR) {
        const long ro = (long)min(f0 - LO + ty + SF * rr, cmax) * st;
#pragma unroll
        for (int v = 0; v < 7; ++v) stage[v][rr] = T(pb[(long)fields[v] * G.field + ro]);
      }
    }
#pragma unroll
    for (int v = 0; v < 7; ++v)
#pragma unroll
      for (int rr = 0; rr < NRR; ++rr)
        if (ty + SF * rr < SR) sh[v][ty + SF * rr][tx] = stage[v][rr];
  }
  __syncthreads();
  // compute: wavefront w takes tile positions PX w .. PX w + PX - 1 times the
  // SF face rows, a PX x PY patch
  static_assert(SF == PY && SX == (SX * SF / 64) * PX, "one PX x PY patch per wavefront");
  const int lane = threadIdx.x % 64;
  const int cx = PX * (int)(threadIdx.x / 64) + lane % PX, cy = lane / PX;
  const int f = f0 + cy;
  // lane x of every wavefront staged tile position x: take its indices
  ii[0] = __shfl(ii[0], cx);
  ii[TB] = __shfl(ii[TB], cx);
  const int okc = __shfl(ok, cx);
  if (!okc || f >= G.face_lo() + nface) return;
  ii[DIR] = f;
  const long c = G.idx(ii[0], ii[1], ii[2]);
  const T gam = T(G.gam);
  MET m;
  if constexpr (!MET::flat) {
    constexpr int loc = DIR == 1 ? LOC_F2 : LOC_C;
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
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
  face_body_q<DIR, RC>([&](int v, int s) { return sh[v][cy + s][cx]; }, bn, axis, m, gam, fh, cd);
#pragma unroll
  for (int q5 = 0; q5 < 5; ++q5) __builtin_nontemporal_store(fh[q5], &flux[(long)q5 * G.field + c]);
#pragma unroll
  for (int q6 = 0; q6 < 6; ++q6) __builtin_nontemporal_store(cd[q6], &ctd[(long)q6 * G.field + c]);
}

// Edges of families 1 and 3 (E = 0, 2: offset in x^2) on a polar axis
// (stored x^2 index -1 or n2 - 1): the covariant field there carries
// sqrt(gamma) = 0, so they are 0 (which also keeps the axis faces' field).
template <int E>
__device__ __forceinline__ bool on_axis(const Geom& G, int j) {
  if constexpr (E == 1) return false;
  else return G.axis2 && (j == -1 || j == G.n[1] - 1);
}

// Edge field of family E.  ctd_d / ctd_c: per-face data of the d and c sweeps
// (stored in the arithmetic type T, as the edge field itself).
template <int E, class MET, typename T, int RC>
__global__ __launch_bounds__(256) void k_edge(Geom G, const double* __restrict__ cons,
                                              const double* __restrict__ tab,
                                              const T* __restrict__ ctd_d,
                                              const T* __restrict__ ctd_c,
                                              T* __restrict__ edge) {
  constexpr int D = (E + 1) % 3, C = (E + 2) % 3;
  constexpr int W = Stencil<RC>::W, LO = Stencil<RC>::LO;
  int ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ext[a] = (a == E) ? G.n[a] : G.face_count(a);
  // families 1 and 2 reconstruct along x^3: tiles traverse x^3 before x^2
  constexpr int MID = E == 2 ? 1 : 2, SLOW = E == 2 ? 2 : 1;
  const TilePos tp = tile_pos(ext[0], ext[MID], EDGE_ALIGN[E] ? line_shift(G.ng, E == 0 ? 0 : G.face_lo()) : 0);
  if (!tp.ok) return;
  int ii[3];
  ii[0] = tp.a;
  ii[MID] = tp.m;
  ii[SLOW] = tp.s;
#pragma unroll
  for (int a = 0; a < 3; ++a) ii[a] += (a == E) ? 0 : G.face_lo();
  const long b = G.idx(ii[0], ii[1], ii[2]);
  const long sd = G.stride(D), sc = G.stride(C);

  T qd[5][W], qc[W];
  {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int s = 0; s < W; ++s) qd[v][s] = ctd_d[(long)v * G.field + b + (s - LO) * sc];
    const double* bds = cons + (long)(C_BF1 + D) * G.field;
#pragma unroll
    for (int s = 0; s < W; ++s) qd[4][s] = T(bds[b + (s - LO) * sc]);
    const double* bcs = cons + (long)(C_BF1 + C) * G.field;
#pragma unroll
    for (int s = 0; s < W; ++s) qc[s] = T(bcs[b + (s - LO) * sd]);
  }
  MET m;
  if constexpr (!MET::flat) {
    // x^3 edges -> E3 tables, x^1 edges (i, j+1/2, k+1/2) -> F2, x^2 edges -> F1
    constexpr int loc = E == 2 ? LOC_E3 : (E == 0 ? LOC_F2 : LOC_F1);
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }
  const T ee = edge_body<E, RC>(qd, qc, ctd_d[4 * G.field + b], ctd_d[4 * G.field + b + sc],
                            ctd_d[5 * G.field + b], ctd_d[5 * G.field + b + sc],
                            ctd_c[4 * G.field + b], ctd_c[4 * G.field + b + sd],
                            ctd_c[5 * G.field + b], ctd_c[5 * G.field + b + sd], m);
  edge[b] = on_axis<E>(G, ii[1]) ? T(0) : ee;
}

// LDS-staged edge field for families E = 0, 2, whose five d-face inputs are
// reconstructed across rows (along x^3 for E = 0, x^2 for E = 2).  Tiles of
// SX consecutive positions (flattened, x^1 fastest) times SF edges along c;
// the SF + W - 1 rows of the five inputs are staged once per workgroup.  The
// c-face B (along d) and the four speeds are read directly.
template <int E, int SF, class MET, typename T, int RC>
__global__ __launch_bounds__(SX * SF) void k_edge_lds(Geom G, const double* __restrict__ cons,
                                                      const double* __restrict__ tab,
                                                      const T* __restrict__ ctd_d,
                                                      const T* __restrict__ ctd_c,
                                                      T* __restrict__ edge) {
  static_assert(E == 0 || E == 2, "families whose d-face inputs vary across rows");
  constexpr int D = (E + 1) % 3, C = (E + 2) % 3, B = 3 - C;   // B: the non-x^1 axis that is not C
  constexpr int W = Stencil<RC>::W, LO = Stencil<RC>::LO;
  constexpr int SR = SF + W - 1, NRR = (SR + SF - 1) / SF;
  __shared__ T sh[5][SR][SX + LPAD];
  const int extA = (E == 0) ? G.n[0] : G.face_count(0), offA = (E == 0) ? 0 : G.face_lo();
  const int extB = (B == E) ? G.n[B] : G.face_count(B), offB = (B == E) ? 0 : G.face_lo();
  // positions flattened with x^1 fastest over rows of rA slots, the x^1 range
  // starting at slot shA so that 16-lane segments are whole 128-byte lines
  const int shA = EDGE_ALIGN[E] ? line_shift(G.ng, offA) : 0;
  const int rA = EDGE_ALIGN[E] ? (extA + shA + 15) / 16 * 16 : extA;
  const long M = (long)rA * extB;
  const int nc = G.face_count(C);               // edges face_lo .. face_lo + nc - 1 along c
  const int ntc = (nc + SF - 1) / SF;
  const long bid = xcd_block(blockIdx.x, gridDim.x);
  const int ct = (int)(bid % ntc);
  const long mt = bid / ntc;
  // ty (the face row) is the wavefront index: uniform, so row offsets go to the scalar unit
  const int tx = threadIdx.x % SX, ty = __builtin_amdgcn_readfirstlane(threadIdx.x / SX);
  const long mm = mt * SX + tx;
  const unsigned mc = (unsigned)(mm < M ? mm : M - 1);
  const int xa = (int)(mc % (unsigned)rA) - shA;
  const int ok = mm < M && xa >= 0 && xa < extA;
  int ii[3];
  ii[0] = min(max(xa, 0), extA - 1) + offA;      // clamped: every staging load is in bounds
  ii[B] = (int)(mc / (unsigned)rA) + offB;
  ii[C] = 0;
  const long base = G.idx(ii[0], ii[1], ii[2]);
  const long sd = G.stride(D), sc = G.stride(C);
  const int c0 = G.face_lo() + ct * SF;
  {
    const double* bds = cons + (long)(C_BF1 + D) * G.field;
    const int cmax = G.n[C] + G.ng - 1;
    T stage[5][NRR];
#pragma unroll
    for (int rr = 0; rr < NRR; ++rr) {
      if (ty + SF * rr < SR) {
        const long ro = base + (long)min(c0 - LO + ty + SF * rr, cmax) * sc;
#pragma unroll
        for (int v = 0; v < 4; ++v) stage[v][rr] = ctd_d[(long)v * G.field + ro];
        stage[4][rr] = T(bds[ro]);
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int rr = 0; rr < NRR; ++rr)
        if (ty + SF * rr < SR) sh[v][ty + SF * rr][tx] = stage[v][rr];
  }
  __syncthreads();
  // compute: wavefront w takes tile positions PX w .. PX w + PX - 1 times the
  // SF edge rows, a PX x PY patch
  static_assert(SF == PY && SX == (SX * SF / 64) * PX, "one PX x PY patch per wavefront");
  const int lane = threadIdx.x % 64;
  const int cx = PX * (int)(threadIdx.x / 64) + lane % PX, cy = lane / PX;
  const int cc = c0 + cy;
  // lane x of every wavefront staged tile position x: take its indices
  ii[0] = __shfl(ii[0], cx);
  ii[B] = __shfl(ii[B], cx);
  const int okc = __shfl(ok, cx);
  if (!okc || cc >= G.face_lo() + nc) return;
  ii[C] = cc;
  const long b = G.idx(ii[0], ii[1], ii[2]);
  T qc[W];
  {
    const double* bcs = cons + (long)(C_BF1 + C) * G.field;
#pragma unroll
    for (int s2 = 0; s2 < W; ++s2) qc[s2] = T(bcs[b + (s2 - LO) * sd]);
  }
  MET m;
  if constexpr (!MET::flat) {
    constexpr int loc = E == 2 ? LOC_E3 : LOC_F2;
    m.load(tab, G.tab_plane, loc, G.tidx(ii[0], ii[1]));
  }
  const T ee = edge_body_q<E, RC>([&](int v, int s2) { return sh[v][cy + s2][cx]; }, qc,
                                  ctd_d[4 * G.field + b], ctd_d[4 * G.field + b + sc],
                                  ctd_d[5 * G.field + b], ctd_d[5 * G.field + b + sc],
                                  ctd_c[4 * G.field + b], ctd_c[4 * G.field + b + sd],
                                  ctd_c[5 * G.field + b], ctd_c[5 * G.field + b + sd], m);
  edge[b] = on_axis<E>(G, ii[1]) ? T(0) : ee;
}

// ------------------------------------------------------------------ launchers
constexpr int SWEEP_SF = 4;   // face rows per workgroup of the staged sweeps
constexpr int EDGE_SF = 4;    // edge rows per workgroup of the staged edge fields

// The per-face results are stored in the arithmetic type T: a float field
// occupies the first half of the bytes of a double field (same element
// offsets, half the stride), so the FP32 form moves half the bytes.
template <class MET, typename T, int RC>
static void launch_sweep_t(int d, const Geom& G, const double* prim, const double* cons,
                           const double* tab, double* flux, double* ctd, hipStream_t s) {
  T* fl = reinterpret_cast<T*>(flux) + (long)d * 5 * G.field;
  T* cd = reinterpret_cast<T*>(ctd) + (long)d * 6 * G.field;
  if (d == 0) {
    const long nf = (long)G.face_count(0) * G.dims[1] * G.dims[2];
    const unsigned nb = MET::flat ? tile_blocks(G.face_count(0), G.dims[1], G.dims[2], line_shift(G.ng, G.face_lo()))
                                  : (unsigned)((nf + 255) / 256);
    hipLaunchKernelGGL((k_sweep<0, MET, T, RC>), dim3(nb), dim3(256), 0, s, G, prim, cons, tab, fl, cd);
    return;
  }
  // tiles: SX transverse positions (rows of the pitch) x SF faces
  constexpr int SF = SWEEP_SF;
  const long M = (long)G.pitch * G.dims[d == 1 ? 2 : 1];
  const long tiles = ((M + SX - 1) / SX) * ((G.face_count(d) + SF - 1) / SF);
  if (d == 1) hipLaunchKernelGGL((k_sweep_lds<1, SF, MET, T, RC>), dim3(tiles), dim3(SX * SF), 0, s, G, prim, cons, tab, fl, cd);
  if (d == 2) hipLaunchKernelGGL((k_sweep_lds<2, SF, MET, T, RC>), dim3(tiles), dim3(SX * SF), 0, s, G, prim, cons, tab, fl, cd);
}

template <class MET, typename T, int RC>
static void launch_edge_t(int e, const Geom& G, const double* cons, const double* tab,
                          const double* ctd, double* edges, hipStream_t s) {
  const int d = (e + 1) % 3, c = (e + 2) % 3;
  const T* cd = reinterpret_cast<const T*>(ctd) + (long)d * 6 * G.field;
  const T* cc = reinterpret_cast<const T*>(ctd) + (long)c * 6 * G.field;
  T* ed = reinterpret_cast<T*>(edges) + (long)e * G.field;
  if (e == 1) {
    hipLaunchKernelGGL((k_edge<1, MET, T, RC>),
                       dim3(tile_blocks(G.face_count(0), G.face_count(2), G.n[1],
                                        EDGE_ALIGN[1] ? line_shift(G.ng, G.face_lo()) : 0)),
                       dim3(256), 0, s, G, cons, tab, cd, cc, ed);
    return;
  }
  // staged families: tiles of SX positions (x^1 rows of whole lines, and the
  // remaining axis) x SF edges along c
  constexpr int SF = EDGE_SF;
  const int B = 3 - c;
  const int extA = (e == 0) ? G.n[0] : G.face_count(0);
  const int shA = EDGE_ALIGN[e] ? line_shift(G.ng, (e == 0) ? 0 : G.face_lo()) : 0;
  const long rA = EDGE_ALIGN[e] ? (extA + shA + 15) / 16 * 16 : extA;
  const long M = rA * ((B == e) ? G.n[B] : G.face_count(B));
  const long tiles = ((M + SX - 1) / SX) * ((G.face_count(c) + SF - 1) / SF);
  if (e == 0) hipLaunchKernelGGL((k_edge_lds<0, SF, MET, T, RC>), dim3(tiles), dim3(SX * SF), 0, s, G, cons, tab, cd, cc, ed);
  if (e == 2) hipLaunchKernelGGL((k_edge_lds<2, SF, MET, T, RC>), dim3(tiles), dim3(SX * SF), 0, s, G, cons, tab, cd, cc, ed);
}

template <int RC>
static void launch_sweep_r(int d, const Geom& G, bool flat, bool fp32, const double* prim,
                           const double* cons, const double* tab, double* flux, double* ctd,
                           hipStream_t s) {
  if (flat && !fp32) launch_sweep_t<FlatMet<double>, double, RC>(d, G, prim, cons, tab, flux, ctd, s);
  if (flat && fp32) launch_sweep_t<FlatMet<float>, float, RC>(d, G, prim, cons, tab, flux, ctd, s);
  if (!flat && !fp32) launch_sweep_t<TabMet<double>, double, RC>(d, G, prim, cons, tab, flux, ctd, s);
  if (!flat && fp32) launch_sweep_t<TabMet<float>, float, RC>(d, G, prim, cons, tab, flux, ctd, s);
}

template <int RC>
static void launch_edge_r(int e, const Geom& G, bool flat, bool fp32, const double* cons,
                          const double* tab, const double* ctd, double* edges, hipStream_t s) {
  if (flat && !fp32) launch_edge_t<FlatMet<double>, double, RC>(e, G, cons, tab, ctd, edges, s);
  if (flat && fp32) launch_edge_t<FlatMet<float>, float, RC>(e, G, cons, tab, ctd, edges, s);
  if (!flat && !fp32) launch_edge_t<TabMet<double>, double, RC>(e, G, cons, tab, ctd, edges, s);
  if (!flat && fp32) launch_edge_t<TabMet<float>, float, RC>(e, G, cons, tab, ctd, edges, s);
}

void launch_sweep(int d, const Geom& G, bool flat, bool fp32, int recon, const double* prim,
                  const double* cons, const double* tab, double* flux, double* ctd, hipStream_t s) {
  if (recon == RECON_MP7) launch_sweep_r<RECON_MP7>(d, G, flat, fp32, prim, cons, tab, flux, ctd, s);
  else if (recon == RECON_WENO5) launch_sweep_r<RECON_WENO5>(d, G, flat, fp32, prim, cons, tab, flux, ctd, s);
  else if (recon == RECON_PLM) launch_sweep_r<RECON_PLM>(d, G, flat, fp32, prim, cons, tab, flux, ctd, s);
  else launch_sweep_r<RECON_MP5>(d, G, flat, fp32, prim, cons, tab, flux, ctd, s);
}

void launch_edge(int e, const Geom& G, bool flat, bool fp32, int recon, const double* cons,
                 const double* tab, const double* ctd, double* edges, hipStream_t s) {
  if (recon == RECON_MP7) launch_edge_r<RECON_MP7>(e, G, flat, fp32, cons, tab, ctd, edges, s);
  else if (recon == RECON_WENO5) launch_edge_r<RECON_WENO5>(e, G, flat, fp32, cons, tab, ctd, edges, s);
  else if (recon == RECON_PLM) launch_edge_r<RECON_PLM>(e, G, flat, fp32, cons, tab, ctd, edges, s);
  else launch_edge_r<RECON_MP5>(e, G, flat, fp32, cons, tab, ctd, edges, s);
}

}  // namespace grmhd
