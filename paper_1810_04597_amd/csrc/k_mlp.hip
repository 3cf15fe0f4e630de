// Learned Newton initial guess: an MLP 8 -> 64 -> 64 -> 64 -> 5 (tanh hidden,
// linear output) on BF16 matrix cores with FP32 accumulation (gfx950).
//
// Formulation: every layer computes Z^T = W X^T with the weights as the MFMA
// A operand (M = output features), activations as the B operand (K = input
// features) and 16 samples along N.  With v_mfma_f32_16x16x16_bf16 the
// accumulator fragment of a layer (lane l: features 4*(l/16)+r, sample l%16)
// has exactly the lane layout of the next layer's B operand, so activations
// flow from layer to layer in registers.  Weight gradients (K = samples) read
// both operands transposed through a small per-wave LDS tile.
//
// Kernels: feature/target generation from primitives (the method's own
// prim -> cons map), normalisation statistics, a fused forward/backward per
// wave with register-resident gradient accumulators, a deterministic
// reduction + Adam update, forward-only inference and the per-zone guess for
// the inversion.
#include "grmhd_device.hpp"
#include "grmhd_kernels.hpp"
#include "grmhd_c2p.hpp"
#include "grmhd_mlp.hpp"

namespace grmhd {
namespace mlp {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// Four floats to bfloat16, round to nearest even (v_cvt_pk_bf16_f32; the
// same rounding as f2bf for every finite value).
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf4 pack(f4 v) {
  const b2v lo = __builtin_convertvector((f2v){v[0], v[1]}, b2v);
  const b2v hi = __builtin_convertvector((f2v){v[2], v[3]}, b2v);
  const unsigned a = __builtin_bit_cast(unsigned, lo), b = __builtin_bit_cast(unsigned, hi);
  bf4 o;
  o[0] = (short)(a & 0xffff); o[1] = (short)(a >> 16);
  o[2] = (short)(b & 0xffff); o[3] = (short)(b >> 16);
  return o;
}

__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A operand: W[row][col0 .. col0+3] of a row-major bf16 matrix with row length ld.
__device__ __forceinline__ bf4 load_a(const unsigned short* __restrict__ w, int ld, int row, int col0) {
  const uint2 v = *reinterpret_cast<const uint2*>(w + (long)row * ld + col0);
  bf4 o;
  o[0] = (short)(v.x & 0xffff); o[1] = (short)(v.x >> 16);
  o[2] = (short)(v.y & 0xffff); o[3] = (short)(v.y >> 16);
  return o;
}
// A operand of a transposed matrix: W^T[row][col0 .. +3] = W[col0 + r][row].
__device__ __forceinline__ bf4 load_at(const unsigned short* __restrict__ w, int ld, int row, int col0) {
  bf4 o;
  o[0] = (short)w[(long)(col0 + 0) * ld + row];
  o[1] = (short)w[(long)(col0 + 1) * ld + row];
  o[2] = (short)w[(long)(col0 + 2) * ld + row];
  o[3] = (short)w[(long)(col0 + 3) * ld + row];
  return o;
}

struct Acts {
  f4 h1[4], h2[4], h3[4];   // tanh outputs, C layout
  f4 out;                   // linear outputs 4*(l/16)+r of sample l%16
};

// Forward pass of one tile of 16 samples; xb: B operand of the inputs.
// tanh(x) = 1 - 2 / (exp(2x) + 1) with the hardware exp2 and reciprocal
// (absolute error ~1e-7, far below the bfloat16 rounding of the activations)
__device__ __forceinline__ float tanh_fast(float x) {
  return 1.f - __fdividef(2.f, __expf(2.f * x) + 1.f);
}

// Training and the forward entry point use the library tanhf.
__device__ __forceinline__ void forward_tile(const unsigned short* __restrict__ wb,
                                             const float* __restrict__ wf, bf4 xb, Acts& a) {
  auto act = [](float x) { return tanhf(x); };
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  bf4 hb[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(load_a(wb + OW1, 16, 16 * mt + lr, 4 * lg), xb, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = act(acc[r] + wf[OB1 + 16 * mt + 4 * lg + r]);
    a.h1[mt] = acc;
    hb[mt] = pack(acc);
  }
  bf4 hb2[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc = mfma(load_a(wb + OW2, 64, 16 * mt + lr, 16 * kt + 4 * lg), hb[kt], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = act(acc[r] + wf[OB2 + 16 * mt + 4 * lg + r]);
    a.h2[mt] = acc;
    hb2[mt] = pack(acc);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc = mfma(load_a(wb + OW3, 64, 16 * mt + lr, 16 * kt + 4 * lg), hb2[kt], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = act(acc[r] + wf[OB3 + 16 * mt + 4 * lg + r]);
    a.h3[mt] = acc;
    hb[mt] = pack(acc);
  }
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 4; ++kt)
    acc = mfma(load_a(wb + OW4, 64, lr, 16 * kt + 4 * lg), hb[kt], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] += wf[OB4 + 4 * lg + r];
  a.out = acc;
}

// Inference over four 16-sample tiles at once (the guess kernel): each
// weight fragment and bias is loaded once per wavefront and feeds the four
// tiles' independent MFMA chains; tanh_fast activations.
__device__ __forceinline__ void forward4(const unsigned short* __restrict__ wb,
                                         const float* __restrict__ wf, const bf4 xb[4], f4 out[4]) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  bf4 h[4][4];   // [tile][k tile] activations, B layout
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const bf4 w = load_a(wb + OW1, 16, 16 * mt + lr, 4 * lg);
    f4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = wf[OB1 + 16 * mt + 4 * lg + r];
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) {
      f4 acc = mfma(w, xb[tl], (f4){0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = tanh_fast(acc[r] + bias[r]);
      h[tl][mt] = pack(acc);
    }
  }
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int ow = layer == 0 ? OW2 : OW3, ob = layer == 0 ? OB2 : OB3;
    bf4 hn[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc[4];
#pragma unroll
      for (int tl = 0; tl < 4; ++tl) acc[tl] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        const bf4 w = load_a(wb + ow, 64, 16 * mt + lr, 16 * kt + 4 * lg);
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) acc[tl] = mfma(w, h[tl][kt], acc[tl]);
      }
      f4 bias;
#pragma unroll
      for (int r = 0; r < 4; ++r) bias[r] = wf[ob + 16 * mt + 4 * lg + r];
#pragma unroll
      for (int tl = 0; tl < 4; ++tl) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[tl][r] = tanh_fast(acc[tl][r] + bias[r]);
        hn[tl][mt] = pack(acc[tl]);
      }
    }
#pragma unroll
    for (int tl = 0; tl < 4; ++tl)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) h[tl][mt] = hn[tl][mt];
  }
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) out[tl] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) {
    const bf4 w = load_a(wb + OW4, 64, lr, 16 * kt + 4 * lg);
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) out[tl] = mfma(w, h[tl][kt], out[tl]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float bias = wf[OB4 + 4 * lg + r];
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) out[tl][r] += bias;
  }
}

// B operand of a tile of standardised inputs x[sample][8] (features >= 8 are 0).
__device__ __forceinline__ bf4 input_b(const float* __restrict__ feat, const float* __restrict__ norm,
                                       long s0, long n) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  bf4 xb = {0, 0, 0, 0};
  const long s = s0 + lr;
  if (lg < 2 && s < n) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * lg + r;
      xb[r] = (short)f2bf((feat[s * NFEAT_STRIDE + k] - norm[NM_FMEAN + k]) / norm[NM_FSTD + k]);
    }
  }
  return xb;
}

// ------------------------------------------------------------------ data generation
// prims (n x 8 float64, rows rho, u1, u2, u3, p, B1, B2, B3; flat frame) ->
// raw features (n x 8) and targets (n x 8, five used).
__global__ __launch_bounds__(256) void k_datagen(const double* __restrict__ prims, long n, double gam,
                                                 float* __restrict__ feat, float* __restrict__ targ,
                                                 double* __restrict__ cons_out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double* pr = prims + t * 8;
  PState<double> s;
  s.rho = pr[0];
  s.p = pr[4];
  for (int q = 0; q < 3; ++q) { s.u[q] = pr[1 + q]; s.B[q] = pr[5 + q]; }
  const FlatMet<double> m;
  make_state(s, m, gam);
  double f[8], y[5];
  mlp_features(s.D, s.S, s.tau, s.B, f);
  y[0] = log10(s.y / (s.tau + s.D));
  y[1] = log10(s.p / s.D);
  y[2] = s.u[0]; y[3] = s.u[1]; y[4] = s.u[2];
  for (int q = 0; q < 8; ++q) feat[t * NFEAT_STRIDE + q] = (float)f[q];
  for (int q = 0; q < 8; ++q) targ[t * NTARG_STRIDE + q] = q < 5 ? (float)y[q] : 0.f;
  if (cons_out) {
    double* co = cons_out + t * 8;
    co[0] = s.D; co[1] = s.S[0]; co[2] = s.S[1]; co[3] = s.S[2]; co[4] = s.tau;
    co[5] = s.B[0]; co[6] = s.B[1]; co[7] = s.B[2];
  }
}

// Batched point-wise inversion (flat frame): cons rows D, S_1..3, tau, B^1..3;
// y0 (nullable): caller's Newton guesses (cold start Gamma U when NULL).
__global__ __launch_bounds__(256) void k_points_c2p(const double* __restrict__ cons, long n, double gam,
                                                    const double* __restrict__ y0, double tol, int maxit,
                                                    double* __restrict__ prim_out,
                                                    int* __restrict__ iters_out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double* c = cons + t * 8;
  const double S[3] = {c[1], c[2], c[3]}, B[3] = {c[5], c[6], c[7]};
  const FlatMet<double> m;
  const double g = y0 ? y0[t] : gam * (c[4] + c[0]);
  const NewtonOut<double> r = newton<double>(c[0], S, c[4], B, m, gam, g, tol, maxit);
  double* po = prim_out + t * 8;
  po[0] = r.rho; po[1] = r.u[0]; po[2] = r.u[1]; po[3] = r.u[2]; po[4] = r.p;
  po[5] = B[0]; po[6] = B[1]; po[7] = B[2];
  if (iters_out) iters_out[t] = r.ok ? r.iters : -r.iters;
}

// per-block partial sums of features, squares, targets, squares (32 doubles)
__global__ __launch_bounds__(256) void k_stats(const float* __restrict__ feat, const float* __restrict__ targ,
                                               long n, double* __restrict__ part) {
  __shared__ double sh[256][32];
  double acc[32];
  for (int q = 0; q < 32; ++q) acc[q] = 0.0;
  for (long s = (long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long)gridDim.x * 256) {
    for (int q = 0; q < 8; ++q) {
      const double f = feat[s * NFEAT_STRIDE + q];
      acc[q] += f;
      acc[8 + q] += f * f;
      const double y = targ[s * NTARG_STRIDE + q];
      acc[16 + q] += y;
      acc[24 + q] += y * y;
    }
  }
  for (int q = 0; q < 32; ++q) sh[threadIdx.x][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < 32) {
    double v = 0.0;
    for (int w = 0; w < 256; ++w) v += sh[w][threadIdx.x];
    part[(long)blockIdx.x * 32 + threadIdx.x] = v;
  }
}

__global__ void k_stats_final(const double* __restrict__ part, int nb, long n, float* __restrict__ norm) {
  const int q = threadIdx.x;
  if (q >= 16) return;
  // q < 8: features, else targets (index q - 8)
  const int base = q < 8 ? 0 : 16;
  const int k = q & 7;
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < nb; ++b) {
    s1 += part[(long)b * 32 + base + k];
    s2 += part[(long)b * 32 + base + 8 + k];
  }
  const double mean = s1 / (double)n;
  double var = s2 / (double)n - mean * mean;
  double sd = var > 0.0 ? sqrt(var) : 1.0;
  if (sd < 1e-12) sd = 1.0;
  if (q < 8) { norm[NM_FMEAN + k] = (float)mean; norm[NM_FSTD + k] = (float)sd; }
  else { norm[NM_TMEAN + k] = (float)mean; norm[NM_TSTD + k] = (float)sd; }
}

// ------------------------------------------------------------------ training gradients
// One wave per block.  Each wave walks tiles of 16 samples of [0, n) and
// accumulates the gradients of the mean-squared error (normalised by
// n_norm * 5) in registers; partial gradients per wave go to part[wave][p].
__global__ __launch_bounds__(64) void k_grad(const unsigned short* __restrict__ wb,
                                             const float* __restrict__ wf,
                                             const float* __restrict__ norm,
                                             const float* __restrict__ feat,
                                             const float* __restrict__ targ, long n, double n_norm,
                                             float* __restrict__ part, double* __restrict__ part_loss) {
  __shared__ float tz[16][65];
  __shared__ float ta[16][65];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  f4 gw1[4], gw2[4][4], gw3[4][4], gw4[4];
  f4 gb1[4], gb2[4], gb3[4], gb4;
  const f4 z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gw1[i] = z4; gw4[i] = z4; gb1[i] = z4; gb2[i] = z4; gb3[i] = z4;
#pragma unroll
    for (int j = 0; j < 4; ++j) { gw2[i][j] = z4; gw3[i][j] = z4; }
  }
  gb4 = z4;
  double loss = 0.0;
  const float scale = (float)(2.0 / (n_norm * NOUT));
  const long ntiles = (n + 15) / 16;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long s0 = tile * 16;
    const bf4 xb = input_b(feat, norm, s0, n);
    Acts a;
    forward_tile(wb, wf, xb, a);
    // output error for outputs o = 4*lg + r of sample lr
    const long s = s0 + lr;
    f4 dz4 = z4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * lg + r;
      if (o < NOUT && s < n) {
        const float y = (targ[s * NTARG_STRIDE + o] - norm[NM_TMEAN + o]) / norm[NM_TSTD + o];
        const float e = a.out[r] - y;
        loss += (double)e * e;
        dz4[r] = scale * e;
      }
    }
    gb4 += dz4;
    const bf4 dz4b = pack(dz4);
    // back through layer 4: dA3 = W4^T dz4
    f4 dz3[4];
    bf4 dz3b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc = mfma(load_at(wb + OW4, 64, 16 * mt + lr, 4 * lg), dz4b, z4);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] *= 1.f - a.h3[mt][r] * a.h3[mt][r];
      dz3[mt] = acc;
      dz3b[mt] = pack(acc);
      gb3[mt] += acc;
    }
    f4 dz2[4];
    bf4 dz2b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc = z4;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma(load_at(wb + OW3, 64, 16 * mt + lr, 16 * kt + 4 * lg), dz3b[kt], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] *= 1.f - a.h2[mt][r] * a.h2[mt][r];
      dz2[mt] = acc;
      dz2b[mt] = pack(acc);
      gb2[mt] += acc;
    }
    f4 dz1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f4 acc = z4;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma(load_at(wb + OW2, 64, 16 * mt + lr, 16 * kt + 4 * lg), dz2b[kt], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] *= 1.f - a.h1[mt][r] * a.h1[mt][r];
      dz1[mt] = acc;
      gb1[mt] += acc;
    }
    // weight gradients dW = dZ A_prev^T through LDS transposes
    auto stage = [&](const f4* dz, int nz, const f4* ap, int na) {
      __syncthreads();
      for (int mt = 0; mt < nz; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) tz[lr][16 * mt + 4 * lg + r] = dz[mt][r];
      for (int mt = 0; mt < na; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) ta[lr][16 * mt + 4 * lg + r] = ap[mt][r];
      __syncthreads();
    };
    auto opa = [&](int mt) {   // A[out = 16 mt + lr][sample = 4 lg + r]
      f4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = tz[4 * lg + r][16 * mt + lr];
      return pack(v);
    };
    auto opb = [&](int nt) {   // B[sample = 4 lg + r][in = 16 nt + lr]
      f4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = ta[4 * lg + r][16 * nt + lr];
      return pack(v);
    };
    // layer 4: dW4 [16 x 64] = dz4 (16 x 16) h3^T
    stage(&dz4, 1, a.h3, 4);
    {
      const bf4 A = opa(0);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gw4[nt] = mfma(A, opb(nt), gw4[nt]);
    }
    // layer 3: dW3 = dz3 h2^T
    stage(dz3, 4, a.h2, 4);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf4 A = opa(mt);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gw3[mt][nt] = mfma(A, opb(nt), gw3[mt][nt]);
    }
    // layer 2: dW2 = dz2 h1^T
    stage(dz2, 4, a.h1, 4);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf4 A = opa(mt);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gw2[mt][nt] = mfma(A, opb(nt), gw2[mt][nt]);
    }
    // layer 1: dW1 [64 x 16] = dz1 x^T (x: standardised inputs, 16 columns)
    {
      f4 xin;
#pragma unroll
      for (int r = 0; r < 4; ++r) xin[r] = bf2f((unsigned short)xb[r]);
      stage(dz1, 4, &xin, 1);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) gw1[mt] = mfma(opa(mt), opb(0), gw1[mt]);
    }
  }
  // reduce bias partials over the 16 samples of each lane group
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        gb1[mt][r] += __shfl_xor(gb1[mt][r], o, 64);
        gb2[mt][r] += __shfl_xor(gb2[mt][r], o, 64);
        gb3[mt][r] += __shfl_xor(gb3[mt][r], o, 64);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) gb4[r] += __shfl_xor(gb4[r], o, 64);
  }
  float* P = part + (long)blockIdx.x * NPARAM;
  // weight fragments: D[row = 16 mt + 4 lg + r][col = 16 nt + lr]
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * mt + 4 * lg + r;
      P[OW1 + row * 16 + lr] = gw1[mt][r];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        P[OW2 + row * 64 + 16 * nt + lr] = gw2[mt][nt][r];
        P[OW3 + row * 64 + 16 * nt + lr] = gw3[mt][nt][r];
      }
      if (lr == 0) {
        P[OB1 + row] = gb1[mt][r];
        P[OB2 + row] = gb2[mt][r];
        P[OB3 + row] = gb3[mt][r];
      }
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * lg + r;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) P[OW4 + row * 64 + 16 * nt + lr] = gw4[nt][r];
    if (lr == 0) P[OB4 + row] = gb4[r];
  }
  // loss partial (sum of squared errors of the wave)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (lane == 0) part_loss[blockIdx.x] = loss;
}

// Sum of the per-wave partial gradients (fixed order); mode 0: write the
// gradient, mode 1: Adam step on the FP32 master weights + BF16 copy.
__global__ __launch_bounds__(256) void k_reduce_adam(const float* __restrict__ part, int nw, int mode,
                                                     float* __restrict__ grad, float* __restrict__ wf,
                                                     unsigned short* __restrict__ wb,
                                                     float* __restrict__ m1, float* __restrict__ m2,
                                                     float lr, float b1, float b2, float eps,
                                                     float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float g = 0.f;
  for (int w = 0; w < nw; ++w) g += part[(long)w * NPARAM + p];
  if (mode == 0) {
    grad[p] = g;
    return;
  }
  const float m = b1 * m1[p] + (1.f - b1) * g;
  const float v = b2 * m2[p] + (1.f - b2) * g * g;
  m1[p] = m;
  m2[p] = v;
  const float w = wf[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  wf[p] = w;
  wb[p] = f2bf(w);
}

__global__ void k_loss_final(const double* __restrict__ part_loss, int nw, double n_norm,
                             double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += part_loss[w];
  out[0] = s / (n_norm * NOUT);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ wf, unsigned short* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) wb[p] = f2bf(wf[p]);
}

// ------------------------------------------------------------------ inference
// Forward over n samples of raw features; out (n x 8 float): standardised
// network outputs (five used).  One wave per 16-sample tile, grid-stride.
__global__ __launch_bounds__(256) void k_forward(const unsigned short* __restrict__ wb,
                                                 const float* __restrict__ wf,
                                                 const float* __restrict__ norm,
                                                 const float* __restrict__ feat, long n,
                                                 float* __restrict__ out) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
  const long ntiles = (n + 15) / 16;
  for (long tile = wave; tile < ntiles; tile += nwaves) {
    const long s0 = tile * 16;
    const bf4 xb = input_b(feat, norm, s0, n);
    Acts a;
    forward_tile(wb, wf, xb, a);
    const long s = s0 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * lg + r;
      if (o < 8 && s < n) out[s * 8 + o] = a.out[r];
    }
  }
}

// Standardised network inputs of interior zone t from its conserved state
// (mlp_features in single precision with the hardware log2 / reciprocal
// square root: the inputs are rounded to bfloat16 next).  Zero when !valid.
template <class MET>
__device__ __forceinline__ void zone_features(const Geom& G, const double* __restrict__ cons,
                                              const double* __restrict__ tab,
                                              const float* __restrict__ norm, long t, bool valid,
                                              float f[8], double& utot) {
  for (int q = 0; q < 8; ++q) f[q] = 0.f;
  utot = 1.0;
  if (!valid) return;
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
  utot = tau + dd;
  double Sh[3], Bh[3];
  frame_components(m, S, B, Sh, Bh);
  const float fdd = (float)dd, fe = (float)utot;
  const float ie = __fdividef(1.f, fe), ise = __frsqrt_rn(fe);
  float fr[8];
  fr[0] = __log10f(fdd);
  fr[1] = __log10f(__fdividef((float)tau, fdd));
  for (int q = 0; q < 3; ++q) {
    fr[2 + q] = (float)Sh[q] * ie;
    fr[5 + q] = (float)Bh[q] * ise;
  }
  for (int q = 0; q < 8; ++q) {
    const float v = fr[q];
    f[q] = isfinite(v) ? (v - norm[NM_FMEAN + q]) * __fdividef(1.f, norm[NM_FSTD + q]) : 0.f;
  }
}

// Learned-guess pass over the zones the inversion deferred (their warm start
// had a large residual).  Each wavefront takes 64 list entries, evaluates the
// network for them on the matrix cores (four 16-sample tiles, features of
// lane l = sample l), and inverts each zone with the network's
// y0 = U 10^{t0} as the second candidate start.  Per-block counters and CFL
// partials go to slot blockIdx.x of partials / cfl_partials.
template <class MET>
__global__ __launch_bounds__(256) void k_c2p_list(Geom G, C2PParams cp, double* __restrict__ prim,
                                                  double* __restrict__ cons,
                                                  const double* __restrict__ tab,
                                                  const unsigned short* __restrict__ wb,
                                                  const float* __restrict__ wf,
                                                  const float* __restrict__ norm,
                                                  const int* __restrict__ list,
                                                  const int* __restrict__ list_n,
                                                  long long* __restrict__ partials,
                                                  double* __restrict__ cfl_partials) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const long n = *list_n;
  const long nwaves = (long)gridDim.x * 4;
  long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long ntaken = 0;
  double cfl_v = 0.0;
  for (long base = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; base < n; base += nwaves * 64) {
    const long idx = base + lane;
    const bool valid = idx < n;
    const long t = valid ? (long)list[idx] : 0;
    float f[8];
    double utot;
    zone_features<MET>(G, cons, tab, norm, t, valid, f, utot);
    bf4 xb[4];
#pragma unroll
    for (int tile = 0; tile < 4; ++tile) {
      const int src = 16 * tile + lr;
      f4 xv;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float lo = __shfl(f[r], src, 64);
        const float hi = __shfl(f[4 + r], src, 64);
        xv[r] = lg == 0 ? lo : (lg == 1 ? hi : 0.f);
      }
      xb[tile] = pack(xv);
    }
    f4 outs[4];
    forward4(wb, wf, xb, outs);
    // output 0 of this lane's sample: tile lane/16, row 0 of lane lane%16
    float o0 = 0.f;
#pragma unroll
    for (int tile = 0; tile < 4; ++tile) {
      const float v = __shfl(outs[tile][0], lr, 64);
      if (lg == tile) o0 = v;
    }
    if (valid) {
      const float t0 = o0 * norm[NM_TSTD + 0] + norm[NM_TMEAN + 0];
      const double y0 = utot * (double)__exp10f(t0);
      const double yg = isfinite(y0) ? y0 : -1.0;
      double cv = 0.0;
      if (cp.learned_only)
        c2p_zone<MET>(G, cp, prim, cons, tab, t, -1.0, 0.0, cfl_partials != nullptr, st, cv, yg, nullptr,
                      true);
      else
        c2p_zone<MET>(G, cp, prim, cons, tab, t, yg, 0.0, cfl_partials != nullptr, st, cv);
      cfl_v = fmax(cfl_v, cv);
      ntaken += 1;
    }
  }
  c2p_block_partials<false>(st, cfl_v, partials, cfl_partials, blockIdx.x, cp.run_acc, ntaken);
}

}  // namespace mlp

// ------------------------------------------------------------------ launchers
void mlp_launch_datagen(const double* prims, long n, double gam, float* feat, float* targ,
                        double* cons_out, double* part, float* norm, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(mlp::k_datagen, dim3(nb), dim3(256), 0, s, prims, n, gam, feat, targ, cons_out);
  if (norm) {
    const int nbs = 256;
    hipLaunchKernelGGL(mlp::k_stats, dim3(nbs), dim3(256), 0, s, feat, targ, n, part);
    hipLaunchKernelGGL(mlp::k_stats_final, dim3(1), dim3(64), 0, s, part, nbs, n, norm);
  }
}

void launch_points_c2p(const double* cons, long n, double gam, const double* y0, double tol, int maxit,
                       double* prim_out, int* iters_out, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(mlp::k_points_c2p, dim3(nb), dim3(256), 0, s, cons, n, gam, y0, tol, maxit,
                     prim_out, iters_out);
}

void mlp_launch_grad(const MlpState& M, const float* feat, const float* targ, long n, int nwaves,
                     hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_grad, dim3(nwaves), dim3(64), 0, s, M.wb, M.wf, M.norm, feat, targ, n,
                     (double)n, M.part, M.part_loss);
  hipLaunchKernelGGL(mlp::k_loss_final, dim3(1), dim3(64), 0, s, M.part_loss, nwaves, (double)n, M.loss);
}

void mlp_launch_reduce(const MlpState& M, int nwaves, int mode, float* grad, float lr, int step,
                       hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp::k_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, M.part, nwaves,
                     mode, grad, M.wf, M.wb, M.m1, M.m2, lr, b1, b2, eps, c1, c2);
}

void mlp_launch_to_bf16(const MlpState& M, hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_to_bf16, dim3((NPARAM + 255) / 256), dim3(256), 0, s, M.wf, M.wb);
}

void mlp_launch_forward(const MlpState& M, const float* feat, long n, float* out, hipStream_t s) {
  const long ntiles = (n + 15) / 16;
  long nb = (ntiles + 3) / 4;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(mlp::k_forward, dim3((unsigned)nb), dim3(256), 0, s, M.wb, M.wf, M.norm, feat, n, out);
}

void mlp_launch_c2p_list(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                         const double* tab, const MlpState& M, const int* list, const int* list_n,
                         long long* partials, double* cfl_partials, hipStream_t s) {
  if (flat)
    hipLaunchKernelGGL(mlp::k_c2p_list<FlatMet<double>>, dim3(C2P_LIST_BLOCKS), dim3(256), 0, s, G, cp,
                       prim, cons, tab, M.wb, M.wf, M.norm, list, list_n, partials, cfl_partials);
  else
    hipLaunchKernelGGL(mlp::k_c2p_list<TabMet<double>>, dim3(C2P_LIST_BLOCKS), dim3(256), 0, s, G, cp,
                       prim, cons, tab, M.wb, M.wf, M.norm, list, list_n, partials, cfl_partials);
}

}  // namespace grmhd
