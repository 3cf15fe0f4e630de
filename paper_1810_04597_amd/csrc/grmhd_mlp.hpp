// Learned Newton guess: parameter layout, features and launchers (internal).
//
// Parameter block (float32 master and bfloat16 copy share the layout):
//   W1 [64][16] (inputs padded 8 -> 16 with zeros), b1 [64],
//   W2 [64][64], b2 [64], W3 [64][64], b3 [64],
//   W4 [16][64] (outputs padded 5 -> 16 with zeros), b4 [16].
// Normalisation block (32 floats): feature mean[8], std[8], target mean[8],
// std[8] (five targets used).
#pragma once
#include <hip/hip_runtime.h>
#include "grmhd_device.hpp"

namespace grmhd {
namespace mlp {
constexpr int NIN = 8, NH = 64, NOUT = 5;
constexpr int OW1 = 0;
constexpr int OB1 = OW1 + 64 * 16;
constexpr int OW2 = OB1 + 64;
constexpr int OB2 = OW2 + 64 * 64;
constexpr int OW3 = OB2 + 64;
constexpr int OB3 = OW3 + 64 * 64;
constexpr int OW4 = OB3 + 64;
constexpr int OB4 = OW4 + 16 * 64;
constexpr int NPARAM = OB4 + 16;       // 10448
constexpr int NNORM = 32;
constexpr int NM_FMEAN = 0, NM_FSTD = 8, NM_TMEAN = 16, NM_TSTD = 24;
constexpr int NFEAT_STRIDE = 8, NTARG_STRIDE = 8;
}  // namespace mlp
using mlp::NPARAM;

// Orthonormal-frame components (Cholesky gamma = L L^T): S_hat = L^-1 S,
// B_hat = L^T B.  Identity in flat space.
template <class MET>
GR_HD void frame_components(const MET& m, const double S[3], const double B[3], double Sh[3],
                            double Bh[3]) {
  if constexpr (MET::flat) {
    for (int q = 0; q < 3; ++q) { Sh[q] = S[q]; Bh[q] = B[q]; }
  } else {
    const double l11 = sqrt(m.g11);
    const double l21 = m.g12 / l11, l31 = m.g13 / l11;
    const double l22 = sqrt(m.g22 - l21 * l21);
    const double l32 = (m.g23 - l31 * l21) / l22;
    const double l33 = sqrt(m.g33 - l31 * l31 - l32 * l32);
    Sh[0] = S[0] / l11;
    Sh[1] = (S[1] - l21 * Sh[0]) / l22;
    Sh[2] = (S[2] - l31 * Sh[0] - l32 * Sh[1]) / l33;
    Bh[0] = l11 * B[0] + l21 * B[1] + l31 * B[2];
    Bh[1] = l22 * B[1] + l32 * B[2];
    Bh[2] = l33 * B[2];
  }
}

// Raw network inputs from undensitised D, orthonormal S_hat, tau, B_hat:
// [log10 D, log10(tau/D), S_hat/(tau+D), B_hat/sqrt(tau+D)].
GR_HD void mlp_features(double dd, const double S[3], double tau, const double B[3], double f[8]) {
  const double e = dd + tau;
  f[0] = log10(dd);
  f[1] = log10(tau / dd);
  for (int q = 0; q < 3; ++q) f[2 + q] = S[q] / e;
  const double se = sqrt(e);
  for (int q = 0; q < 3; ++q) f[5 + q] = B[q] / se;
}

struct MlpState {
  unsigned short* wb = nullptr;   // bf16 weights
  float* wf = nullptr;            // fp32 master weights
  float* norm = nullptr;          // normalisation block
  float* m1 = nullptr;            // Adam first moment
  float* m2 = nullptr;            // Adam second moment
  float* part = nullptr;          // per-wave partial gradients [nwaves][NPARAM]
  double* part_loss = nullptr;    // per-wave partial losses
  double* loss = nullptr;         // reduced loss
  double* dpart = nullptr;        // statistics partials
  int nwaves = 0;
  int step = 0;
  bool weights_set = false;
};

void mlp_launch_datagen(const double* prims, long n, double gam, float* feat, float* targ,
                        double* cons_out, double* part, float* norm, hipStream_t s);
void launch_points_c2p(const double* cons, long n, double gam, const double* y0, double tol, int maxit,
                       double* prim_out, int* iters_out, hipStream_t s);
void mlp_launch_grad(const MlpState& M, const float* feat, const float* targ, long n, int nwaves,
                     hipStream_t s);
void mlp_launch_reduce(const MlpState& M, int nwaves, int mode, float* grad, float lr, int step,
                       hipStream_t s);
void mlp_launch_to_bf16(const MlpState& M, hipStream_t s);
void mlp_launch_forward(const MlpState& M, const float* feat, long n, float* out, hipStream_t s);
// Learned-guess pass over the zones the inversion deferred (list / list_n):
// network guess and inversion; per-block counters and CFL partials (nullable)
// at [0, C2P_LIST_BLOCKS) of partials / cfl_partials.
void mlp_launch_c2p_list(const Geom& G, bool flat, const C2PParams& cp, double* prim, double* cons,
                         const double* tab, const MlpState& M, const int* list, const int* list_n,
                         long long* partials, double* cfl_partials, hipStream_t s);

}  // namespace grmhd
