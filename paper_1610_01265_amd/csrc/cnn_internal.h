// Internal declarations of the CNN part of libsts (learned initial guess of
// the backward-Euler solve): the network state behind sts_cnn and the host
// launchers of k_cnn.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {

constexpr int kCnnC = 16;                        // channels of every padded layer
constexpr int kCnnTaps = 27;                     // 3 x 3 x 3 kernel
constexpr int kCnnWPerLayer = kCnnC * kCnnC * kCnnTaps;  // padded W[co][ci][tap]
constexpr int kCnnPPerLayer = kCnnWPerLayer + kCnnC;     // + bias[co]
constexpr int kCnnFrag = 14 * 64 * 8;            // bf16 MFMA A fragments per layer

struct CnnLaunch {
  hipStream_t stream;
  int n0, n1, n2;
  int rev;  // debug: reversed workgroup order of the plane-marching kernels
};

// kind: 0 ReLU -> bf16 [cells][16]; 1 channel 0 -> FP32 [cells];
// 2 masked (mask > 0) -> bf16 [cells][16]; 3 -> FP32 [cells][16];
// 5 channels 0..3 -> FP32 [cells][4]
void launch_cnn_conv(const CnnLaunch &L, int kind, const void *in, const void *wfrag,
                     const float *bias, const void *mask, void *out_bf, float *outf);
int cnn_wgrad_parts();
// weight and bias gradients of one layer into g (padded master layout, 6928 values)
void launch_cnn_wgrad(const CnnLaunch &L, const void *act, const void *dout, float *part,
                      float *g);
void launch_cnn_pack_input(const CnnLaunch &L, const double *rhs, const double *T, double rs,
                           double tsh, double tsc, void *x);
int cnn_loss_parts();
void launch_cnn_loss(const CnnLaunch &L, const float *pred, const double *xs, const double *T,
                     double inv_sd, void *g, double *part);
void launch_cnn_guess(const CnnLaunch &L, const double *T, const float *pred, double sd,
                      double *x0);
void launch_cnn_adam(const CnnLaunch &L, int n, float *p, float *m, float *v, const float *g,
                     const float *mask, float lr, int step, float b1, float b2, float eps);
void launch_cnn_make_frags(const CnnLaunch &L, const float *W, void *ffwd, void *fbwd);
int cnn_moment_parts();
void launch_cnn_moments(const CnnLaunch &L, const double *x, const double *y, double sc,
                        double *part, double *out2);
void launch_cnn_sum_parts(const CnnLaunch &L, const double *part, int n, double *out);

}  // namespace sts

struct sts_cnn {
  sts_ctx *ctx = nullptr;
  int layers = 0;
  int nout = 1;                // output channels: 1 (initial guess) or 4 (factor network)
  long long ncell = 0;
  long long nparam = 0;        // unpadded parameter count (host weight vector)
  float *d_P = nullptr;        // padded FP32 master parameters, layers * kCnnPPerLayer
  float *d_M = nullptr, *d_V = nullptr;  // Adam moments
  float *d_G = nullptr;        // gradients (same layout)
  float *d_mask = nullptr;     // 1 where the padded network has a parameter
  void *d_frag = nullptr;      // bf16 fragments: layer l forward at 2l, transposed at 2l+1
  void *d_act = nullptr;       // bf16 [layers][cells][16]: network input, hidden activations
  void *d_g = nullptr;         // bf16 [2][cells][16]: back-propagated gradients
  float *d_pred = nullptr;     // FP32 [cells][nout] network output
  double *d_F = nullptr;       // FP64 [cells] F(T_prev) for cnn_guess
  float *d_wpart = nullptr;    // weight-gradient partials
  double *d_part = nullptr;    // loss / moment partials
  double *d_out = nullptr;     // two device scalars read by the host
  double rhs_scale = 1.0, t_shift = 0.0, t_scale = 1.0, delta_scale = 1.0;
  int step = 0;                // Adam steps taken
  float adam_b1 = 0.9f, adam_b2 = 0.999f, adam_eps = 1e-8f;  // Adam constants

  sts::CnnLaunch launch() const;
  void *act(int l) const { return (char *)d_act + (size_t)l * ncell * sts::kCnnC * 2; }
  void *g(int q) const { return (char *)d_g + (size_t)q * ncell * sts::kCnnC * 2; }
  void *frag(int l, int transposed) const {
    return (char *)d_frag + (size_t)(2 * l + transposed) * sts::kCnnFrag * 2;
  }
};
