// Host side of the CNN entry points of include/sts.h (learned initial guess
// of the backward-Euler solve): state, argument checks, weight-vector
// layout conversion and the launch sequences of inference and training.
#include <cmath>
#include <string>
#include <vector>

#include "cnn_internal.h"

using namespace sts;

sts::CnnLaunch sts_cnn::launch() const {
  return CnnLaunch{ctx->stream, ctx->n0, ctx->n1, ctx->n2,
                   (ctx->debug & STS_DEBUG_WG_REVERSE) ? 1 : 0};
}

namespace {

#define NFAIL(code, msg)      \
  do {                        \
    net->ctx->err = (msg);    \
    return (code);            \
  } while (0)

#define NHIPCHK(expr)                                                             \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      net->ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return STS_EHIP;                                                            \
    }                                                                             \
  } while (0)

#define NLAUNCHCHK() NHIPCHK(hipGetLastError())

int in_ch(const sts_cnn *net, int l) { return l == 0 ? 2 : kCnnC; }
int out_ch(const sts_cnn *net, int l) { return l == net->layers - 1 ? net->nout : kCnnC; }

long long count_params(const sts_cnn *net) {
  long long n = 0;
  for (int l = 0; l < net->layers; ++l) n += (long long)out_ch(net, l) * (in_ch(net, l) * kCnnTaps + 1);
  return n;
}

sts_status nalloc(sts_cnn *net, void **p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    net->ctx->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return STS_ENOMEM;
  }
  return STS_OK;
}

template <class T>
void nfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void refresh_frags(sts_cnn *net) {
  const CnnLaunch L = net->launch();
  for (int l = 0; l < net->layers; ++l)
    launch_cnn_make_frags(L, net->d_P + (size_t)l * kCnnPPerLayer, net->frag(l, 0), net->frag(l, 1));
}

const float *bias(const sts_cnn *net, int l) { return net->d_P + (size_t)l * kCnnPPerLayer + kCnnWPerLayer; }

void adam(sts_cnn *net, const float *G, float lr);

// forward from the packed input act(0) through every layer into d_pred
// (one channel: kind 1; the factor network's four channels: kind 5)
void forward_packed(sts_cnn *net) {
  const CnnLaunch L = net->launch();
  for (int l = 0; l + 1 < net->layers; ++l)
    launch_cnn_conv(L, 0, net->act(l), net->frag(l, 0), bias(net, l), nullptr, net->act(l + 1),
                    nullptr);
  const int l = net->layers - 1;
  launch_cnn_conv(L, net->nout == 1 ? 1 : 5, net->act(l), net->frag(l, 0), bias(net, l), nullptr,
                  nullptr, net->d_pred);
}

// network input into act(0), forward through every layer into d_pred
void forward(sts_cnn *net, const double *F_prev, double dt, const double *T_prev) {
  launch_cnn_pack_input(net->launch(), F_prev, T_prev, dt * net->rhs_scale, net->t_shift,
                        net->t_scale, net->act(0));
  forward_packed(net);
}

// gradient of the loss with respect to the network output in g(0):
// back-propagation into grad (padded layout, layers x kCnnPPerLayer)
void backward(sts_cnn *net, float *grad) {
  const CnnLaunch L = net->launch();
  int q = 0;  // g(q): gradient with respect to the output of layer l
  for (int l = net->layers - 1; l >= 0; --l) {
    float *G = grad + (size_t)l * kCnnPPerLayer;
    launch_cnn_wgrad(L, net->act(l), net->g(q), net->d_wpart, G);
    if (l > 0) {
      launch_cnn_conv(L, 2, net->g(q), net->frag(l, 1), nullptr, net->act(l), net->g(1 - q),
                      nullptr);
      q = 1 - q;
    }
  }
}

void backward_adam(sts_cnn *net, float lr) {
  backward(net, net->d_G);
  adam(net, net->d_G, lr);
}

bool finite_nonzero(double x) { return std::isfinite(x) && x != 0.0; }

// one Adam step of the master parameters with gradient G (padded layout),
// then the bf16 fragments of the updated weights
void adam(sts_cnn *net, const float *G, float lr) {
  net->step += 1;
  launch_cnn_adam(net->launch(), net->layers * kCnnPPerLayer, net->d_P, net->d_M, net->d_V, G,
                  net->d_mask, lr, net->step, net->adam_b1, net->adam_b2, net->adam_eps);
  refresh_frags(net);
}

}  // namespace

extern "C" {

static sts_status create_net(sts_cnn **out, sts_ctx *ctx, int layers, int channels, int nout) {
  if (!out || !ctx) return STS_EINVAL;
  *out = nullptr;
  if (layers < 2 || layers > 8) {
    ctx->err = "cnn_create: layers must be in [2, 8]";
    return STS_EINVAL;
  }
  if (channels != kCnnC) {
    ctx->err = "cnn_create: only 16 hidden channels are supported";
    return STS_EINVAL;
  }
  sts_cnn *net = new sts_cnn;
  net->ctx = ctx;
  net->layers = layers;
  net->nout = nout;
  net->ncell = ctx->ncell;
  net->nparam = count_params(net);
  const size_t np = (size_t)layers * kCnnPPerLayer, nc = (size_t)ctx->ncell;
  sts_status st = STS_OK;
  auto A = [&](void **p, size_t bytes) {
    if (st == STS_OK) st = nalloc(net, p, bytes);
  };
  A((void **)&net->d_P, np * 4);
  A((void **)&net->d_M, np * 4);
  A((void **)&net->d_V, np * 4);
  A((void **)&net->d_G, np * 4);
  A((void **)&net->d_mask, np * 4);
  A(&net->d_frag, (size_t)2 * layers * kCnnFrag * 2);
  A(&net->d_act, (size_t)layers * nc * kCnnC * 2);
  A(&net->d_g, (size_t)2 * nc * kCnnC * 2);
  A((void **)&net->d_pred, nc * 4 * nout);
  A((void **)&net->d_F, nc * 8);
  A((void **)&net->d_wpart, (size_t)cnn_wgrad_parts() * (kCnnTaps + 1) * 256 * 4);
  const int npart = std::max(cnn_loss_parts(), 2 * cnn_moment_parts());
  A((void **)&net->d_part, (size_t)npart * 8);
  A((void **)&net->d_out, 16);
  if (st != STS_OK) {
    cnn_destroy(net);
    return st;
  }
  std::vector<float> mask(np, 0.0f);
  for (int l = 0; l < layers; ++l) {
    float *m = mask.data() + (size_t)l * kCnnPPerLayer;
    for (int co = 0; co < out_ch(net, l); ++co) {
      for (int ci = 0; ci < in_ch(net, l); ++ci)
        for (int t = 0; t < kCnnTaps; ++t) m[(co * kCnnC + ci) * kCnnTaps + t] = 1.0f;
      m[kCnnWPerLayer + co] = 1.0f;
    }
  }
  hipStream_t s = ctx->stream;
  if (hipMemcpyAsync(net->d_mask, mask.data(), np * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(net->d_P, 0, np * 4, s) != hipSuccess ||
      hipMemsetAsync(net->d_M, 0, np * 4, s) != hipSuccess ||
      hipMemsetAsync(net->d_V, 0, np * 4, s) != hipSuccess ||
      hipMemsetAsync(net->d_act, 0, (size_t)layers * nc * kCnnC * 2, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    ctx->err = "cnn_create: initialisation failed";
    cnn_destroy(net);
    return STS_EHIP;
  }
  refresh_frags(net);
  if (hipGetLastError() != hipSuccess) {
    ctx->err = "cnn_create: fragment kernel launch failed";
    cnn_destroy(net);
    return STS_EHIP;
  }
  *out = net;
  return STS_OK;
}

sts_status cnn_create(sts_cnn **out, sts_ctx *ctx, int layers, int channels) {
  return create_net(out, ctx, layers, channels, 1);
}

sts_status cnn_create_pc(sts_cnn **out, sts_ctx *ctx, int layers, int channels) {
  return create_net(out, ctx, layers, channels, 4);
}

sts_status cnn_destroy(sts_cnn *net) {
  if (!net) return STS_EINVAL;
  if (net->ctx && net->ctx->stream) (void)hipStreamSynchronize(net->ctx->stream);
  nfree(net->d_P);
  nfree(net->d_M);
  nfree(net->d_V);
  nfree(net->d_G);
  nfree(net->d_mask);
  nfree(net->d_frag);
  nfree(net->d_act);
  nfree(net->d_g);
  nfree(net->d_pred);
  nfree(net->d_F);
  nfree(net->d_wpart);
  nfree(net->d_part);
  nfree(net->d_out);
  delete net;
  return STS_OK;
}

long long cnn_num_params(const sts_cnn *net) { return net ? net->nparam : 0; }

sts_status cnn_set_weights(sts_cnn *net, const float *w, long long n) {
  if (!net) return STS_EINVAL;
  if (!w || n != net->nparam) NFAIL(STS_EINVAL, "cnn_set_weights: need cnn_num_params values");
  for (long long q = 0; q < n; ++q)
    if (!std::isfinite(w[q])) NFAIL(STS_EINVAL, "cnn_set_weights: non-finite weight");
  const size_t np = (size_t)net->layers * kCnnPPerLayer;
  std::vector<float> P(np, 0.0f);
  const float *src = w;
  for (int l = 0; l < net->layers; ++l) {
    float *dst = P.data() + (size_t)l * kCnnPPerLayer;
    const int co_n = out_ch(net, l), ci_n = in_ch(net, l);
    for (int co = 0; co < co_n; ++co)
      for (int ci = 0; ci < ci_n; ++ci)
        for (int t = 0; t < kCnnTaps; ++t) dst[(co * kCnnC + ci) * kCnnTaps + t] = *src++;
    for (int co = 0; co < co_n; ++co) dst[kCnnWPerLayer + co] = *src++;
  }
  hipStream_t s = net->ctx->stream;
  NHIPCHK(hipMemcpyAsync(net->d_P, P.data(), np * 4, hipMemcpyHostToDevice, s));
  NHIPCHK(hipMemsetAsync(net->d_M, 0, np * 4, s));
  NHIPCHK(hipMemsetAsync(net->d_V, 0, np * 4, s));
  refresh_frags(net);
  NLAUNCHCHK();
  NHIPCHK(hipStreamSynchronize(s));
  net->step = 0;
  return STS_OK;
}

sts_status cnn_get_weights(sts_cnn *net, float *w, long long n) {
  if (!net) return STS_EINVAL;
  if (!w || n != net->nparam) NFAIL(STS_EINVAL, "cnn_get_weights: need cnn_num_params values");
  const size_t np = (size_t)net->layers * kCnnPPerLayer;
  std::vector<float> P(np);
  NHIPCHK(hipMemcpyAsync(P.data(), net->d_P, np * 4, hipMemcpyDeviceToHost, net->ctx->stream));
  NHIPCHK(hipStreamSynchronize(net->ctx->stream));
  float *dst = w;
  for (int l = 0; l < net->layers; ++l) {
    const float *src = P.data() + (size_t)l * kCnnPPerLayer;
    const int co_n = out_ch(net, l), ci_n = in_ch(net, l);
    for (int co = 0; co < co_n; ++co)
      for (int ci = 0; ci < ci_n; ++ci)
        for (int t = 0; t < kCnnTaps; ++t) *dst++ = src[(co * kCnnC + ci) * kCnnTaps + t];
    for (int co = 0; co < co_n; ++co) *dst++ = src[kCnnWPerLayer + co];
  }
  return STS_OK;
}

long long cnn_state_size(const sts_cnn *net) {
  return net ? 3LL * net->layers * kCnnPPerLayer : 0;
}

sts_status cnn_get_state(sts_cnn *net, float *buf, long long n, double meta[8]) {
  if (!net) return STS_EINVAL;
  const long long np = (long long)net->layers * kCnnPPerLayer;
  if (!buf || !meta || n != 3 * np) NFAIL(STS_EINVAL, "cnn_get_state: need cnn_state_size values");
  hipStream_t s = net->ctx->stream;
  NHIPCHK(hipMemcpyAsync(buf, net->d_P, np * 4, hipMemcpyDeviceToHost, s));
  NHIPCHK(hipMemcpyAsync(buf + np, net->d_M, np * 4, hipMemcpyDeviceToHost, s));
  NHIPCHK(hipMemcpyAsync(buf + 2 * np, net->d_V, np * 4, hipMemcpyDeviceToHost, s));
  NHIPCHK(hipStreamSynchronize(s));
  const double m[8] = {(double)net->step, net->rhs_scale, net->t_shift, net->t_scale,
                       net->delta_scale, net->adam_b1, net->adam_b2, net->adam_eps};
  for (int q = 0; q < 8; ++q) meta[q] = m[q];
  return STS_OK;
}

sts_status cnn_set_state(sts_cnn *net, const float *buf, long long n, const double meta[8]) {
  if (!net) return STS_EINVAL;
  const long long np = (long long)net->layers * kCnnPPerLayer;
  if (!buf || !meta || n != 3 * np) NFAIL(STS_EINVAL, "cnn_set_state: need cnn_state_size values");
  for (long long q = 0; q < n; ++q)
    if (!std::isfinite(buf[q])) NFAIL(STS_EINVAL, "cnn_set_state: non-finite value");
  for (long long q = 2 * np; q < n; ++q)
    if (buf[q] < 0.0f) NFAIL(STS_EINVAL, "cnn_set_state: negative second moment");
  if (!(meta[0] >= 0.0 && meta[0] < 2147483647.0 && meta[0] == (double)(long long)meta[0]))
    NFAIL(STS_EINVAL, "cnn_set_state: bad step count");
  if (!finite_nonzero(meta[1]) || !std::isfinite(meta[2]) || !finite_nonzero(meta[3]) ||
      !finite_nonzero(meta[4]))
    NFAIL(STS_EINVAL, "cnn_set_state: scalings must be finite and nonzero");
  if (!(meta[5] >= 0.0 && meta[5] < 1.0) || !(meta[6] >= 0.0 && meta[6] < 1.0) ||
      !(meta[7] > 0.0) || !std::isfinite(meta[7]))
    NFAIL(STS_EINVAL, "cnn_set_state: bad Adam constants");
  // the padding entries, which hold no parameter, stay zero
  std::vector<float> mask(np);
  hipStream_t s = net->ctx->stream;
  NHIPCHK(hipMemcpyAsync(mask.data(), net->d_mask, np * 4, hipMemcpyDeviceToHost, s));
  NHIPCHK(hipStreamSynchronize(s));
  for (long long q = 0; q < np; ++q)
    if (mask[q] == 0.0f && (buf[q] != 0.0f || buf[np + q] != 0.0f || buf[2 * np + q] != 0.0f))
      NFAIL(STS_EINVAL, "cnn_set_state: nonzero value at a padding entry");
  NHIPCHK(hipMemcpyAsync(net->d_P, buf, np * 4, hipMemcpyHostToDevice, s));
  NHIPCHK(hipMemcpyAsync(net->d_M, buf + np, np * 4, hipMemcpyHostToDevice, s));
  NHIPCHK(hipMemcpyAsync(net->d_V, buf + 2 * np, np * 4, hipMemcpyHostToDevice, s));
  refresh_frags(net);
  NLAUNCHCHK();
  NHIPCHK(hipStreamSynchronize(s));
  net->step = (int)meta[0];
  net->rhs_scale = meta[1];
  net->t_shift = meta[2];
  net->t_scale = meta[3];
  net->delta_scale = meta[4];
  net->adam_b1 = (float)meta[5];
  net->adam_b2 = (float)meta[6];
  net->adam_eps = (float)meta[7];
  return STS_OK;
}

sts_status cnn_set_norm(sts_cnn *net, double rhs_scale, double T_shift, double T_scale,
                        double delta_scale) {
  if (!net) return STS_EINVAL;
  if (!finite_nonzero(rhs_scale) || !std::isfinite(T_shift) || !finite_nonzero(T_scale) ||
      !finite_nonzero(delta_scale))
    NFAIL(STS_EINVAL, "cnn_set_norm: scalings must be finite and nonzero");
  net->rhs_scale = rhs_scale;
  net->t_shift = T_shift;
  net->t_scale = T_scale;
  net->delta_scale = delta_scale;
  return STS_OK;
}

sts_status cnn_moments(sts_cnn *net, const double *x, const double *y, double scale,
                       double out[2]) {
  if (!net) return STS_EINVAL;
  if (!x || !out || !std::isfinite(scale)) NFAIL(STS_EINVAL, "cnn_moments: bad argument");
  launch_cnn_moments(net->launch(), x, y, scale, net->d_part, net->d_out);
  NLAUNCHCHK();
  double h[2];
  NHIPCHK(hipMemcpyAsync(h, net->d_out, 16, hipMemcpyDeviceToHost, net->ctx->stream));
  NHIPCHK(hipStreamSynchronize(net->ctx->stream));
  const double n = (double)net->ncell;
  out[0] = h[0] / n;
  out[1] = std::sqrt(h[1] / n);
  return STS_OK;
}

sts_status cnn_pack_input(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                          void *x16) {
  if (!net) return STS_EINVAL;
  if (!F_prev || !T_prev || !x16) NFAIL(STS_EINVAL, "cnn_pack_input: null array");
  if (!std::isfinite(dt)) NFAIL(STS_EINVAL, "cnn_pack_input: dt must be finite");
  launch_cnn_pack_input(net->launch(), F_prev, T_prev, dt * net->rhs_scale, net->t_shift,
                        net->t_scale, x16);
  NLAUNCHCHK();
  return STS_OK;
}

sts_status cnn_conv(sts_cnn *net, int layer, int kind, const void *in16, const void *mask16,
                    void *out) {
  if (!net) return STS_EINVAL;
  if (layer < 0 || layer >= net->layers) NFAIL(STS_EINVAL, "cnn_conv: layer out of range");
  if (!in16 || !out || in16 == out) NFAIL(STS_EINVAL, "cnn_conv: null or aliased arrays");
  const CnnLaunch L = net->launch();
  const float *b = bias(net, layer);
  switch (kind) {
    case 0:
      launch_cnn_conv(L, 0, in16, net->frag(layer, 0), b, nullptr, out, nullptr);
      break;
    case 1:
      launch_cnn_conv(L, 1, in16, net->frag(layer, 0), b, nullptr, nullptr, (float *)out);
      break;
    case 2:
      launch_cnn_conv(L, 2, in16, net->frag(layer, 1), nullptr, mask16, out, nullptr);
      break;
    case 3:
      launch_cnn_conv(L, 3, in16, net->frag(layer, 0), b, nullptr, nullptr, (float *)out);
      break;
    case 4:
      launch_cnn_conv(L, 3, in16, net->frag(layer, 1), nullptr, nullptr, nullptr, (float *)out);
      break;
    case 5:
      launch_cnn_conv(L, 5, in16, net->frag(layer, 0), b, nullptr, nullptr, (float *)out);
      break;
    default:
      NFAIL(STS_EINVAL, "cnn_conv: kind must be 0..5");
  }
  NLAUNCHCHK();
  return STS_OK;
}

sts_status cnn_weight_grad(sts_cnn *net, int layer, const void *act16, const void *dout16,
                           float *grad) {
  if (!net) return STS_EINVAL;
  if (layer < 0 || layer >= net->layers) NFAIL(STS_EINVAL, "cnn_weight_grad: layer out of range");
  if (!act16 || !dout16 || !grad) NFAIL(STS_EINVAL, "cnn_weight_grad: null array");
  const CnnLaunch L = net->launch();
  launch_cnn_wgrad(L, act16, dout16, net->d_wpart, grad);
  NLAUNCHCHK();
  return STS_OK;
}

sts_status cnn_forward(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                       double *x0) {
  if (!net) return STS_EINVAL;
  if (net->nout != 1) NFAIL(STS_EINVAL, "cnn_forward: not an initial-guess network");
  if (!F_prev || !T_prev || !x0) NFAIL(STS_EINVAL, "cnn_forward: null array");
  if (!std::isfinite(dt)) NFAIL(STS_EINVAL, "cnn_forward: dt must be finite");
  forward(net, F_prev, dt, T_prev);
  launch_cnn_guess(net->launch(), T_prev, net->d_pred, net->delta_scale, x0);
  NLAUNCHCHK();
  return STS_OK;
}

sts_status cnn_train_step(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                          const double *x_star, float lr, double *loss) {
  if (!net) return STS_EINVAL;
  if (net->nout != 1) NFAIL(STS_EINVAL, "cnn_train_step: not an initial-guess network");
  if (!F_prev || !T_prev || !x_star) NFAIL(STS_EINVAL, "cnn_train_step: null array");
  if (!std::isfinite(dt)) NFAIL(STS_EINVAL, "cnn_train_step: dt must be finite");
  if (!(lr > 0.0f) || !std::isfinite(lr)) NFAIL(STS_EINVAL, "cnn_train_step: lr must be > 0");
  const CnnLaunch L = net->launch();
  forward(net, F_prev, dt, T_prev);
  launch_cnn_loss(L, net->d_pred, x_star, T_prev, 1.0 / net->delta_scale, net->g(0), net->d_part);
  if (loss) launch_cnn_sum_parts(L, net->d_part, cnn_loss_parts(), net->d_out);
  backward_adam(net, lr);
  NLAUNCHCHK();
  if (loss) {
    double h;
    NHIPCHK(hipMemcpyAsync(&h, net->d_out, 8, hipMemcpyDeviceToHost, net->ctx->stream));
    NHIPCHK(hipStreamSynchronize(net->ctx->stream));
    *loss = h / (double)net->ncell;
  }
  return STS_OK;
}

sts_status cnn_set_adam(sts_cnn *net, double beta1, double beta2, double eps) {
  if (!net) return STS_EINVAL;
  if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    NFAIL(STS_EINVAL, "cnn_set_adam: beta1 and beta2 must lie in [0, 1)");
  if (!(eps > 0.0) || !std::isfinite(eps)) NFAIL(STS_EINVAL, "cnn_set_adam: eps must be > 0");
  net->adam_b1 = (float)beta1;
  net->adam_b2 = (float)beta2;
  net->adam_eps = (float)eps;
  return STS_OK;
}

sts_status cnn_adam_step(sts_cnn *net, const float *grad, float lr) {
  if (!net) return STS_EINVAL;
  if (!grad) NFAIL(STS_EINVAL, "cnn_adam_step: null gradient");
  if (!(lr > 0.0f) || !std::isfinite(lr)) NFAIL(STS_EINVAL, "cnn_adam_step: lr must be > 0");
  adam(net, grad, lr);
  NLAUNCHCHK();
  return STS_OK;
}

sts_status cnn_guess(sts_cnn *net, const double *T_prev, double dt, double *x0, int *used_net,
                     double relres[2]) {
  if (!net) return STS_EINVAL;
  sts_ctx *ctx = net->ctx;
  if (net->nout != 1) NFAIL(STS_EINVAL, "cnn_guess: not an initial-guess network");
  if (!T_prev || !x0 || T_prev == x0) NFAIL(STS_EINVAL, "cnn_guess: null or aliased arrays");
  if (!(dt > 0.0) || !std::isfinite(dt)) NFAIL(STS_EINVAL, "cnn_guess: dt must be finite, > 0");
  sts_status st = apply_F(ctx, T_prev, net->d_F, 1);
  if (st) return st;
  forward(net, net->d_F, dt, T_prev);
  launch_cnn_guess(net->launch(), T_prev, net->d_pred, net->delta_scale, x0);
  NLAUNCHCHK();
  double r_net = 0.0, r_prev = 0.0;
  if ((st = sts_be_residual(ctx, T_prev, x0, dt, &r_net))) return st;
  if ((st = sts_be_residual(ctx, T_prev, T_prev, dt, &r_prev))) return st;
  const bool keep = std::isfinite(r_net) && r_net <= r_prev;
  if (!keep)
    NHIPCHK(hipMemcpyAsync(x0, T_prev, (size_t)net->ncell * 8, hipMemcpyDeviceToDevice,
                           ctx->stream));
  NHIPCHK(hipStreamSynchronize(ctx->stream));
  if (used_net) *used_net = keep ? 1 : 0;
  if (relres) {
    relres[0] = r_net;
    relres[1] = r_prev;
  }
  return STS_OK;
}

// ---- the factor network: M^-1 = G G^T for STS_PC_FACTOR -----------------

// input features of the factor network at dt into act(0)
static sts_status pc_features(sts_cnn *net, const double *T, double dt) {
  sts_ctx *ctx = net->ctx;
  double dte;
  sts_status st = sts_dt_euler(ctx, &dte);
  if (st) return st;
  const double lscale = 1.0 / std::log1p(dt / dte);
  launch_pc_pack(ctx, dt, lscale, T, net->t_shift, net->t_scale, net->act(0));
  return STS_OK;
}

static sts_status pc_checks(sts_cnn *net, const char *name, const double *T, double dt) {
  sts_ctx *ctx = net->ctx;
  if (net->nout != 4) NFAIL(STS_EINVAL, std::string(name) + ": not a factor network");
  if (ctx->op == OP_NONE) NFAIL(STS_EINVAL, "no operator set");
  if (ctx->prec != 0) NFAIL(STS_EINVAL, std::string(name) + ": FP64 operators only");
  if (!T) NFAIL(STS_EINVAL, std::string(name) + ": null T");
  if (!(dt > 0.0) || !std::isfinite(dt))
    NFAIL(STS_EINVAL, std::string(name) + ": dt must be finite, > 0");
  return STS_OK;
}

sts_status cnn_pc_set_norm(sts_cnn *net, double T_shift, double T_scale) {
  if (!net) return STS_EINVAL;
  if (!std::isfinite(T_shift) || !finite_nonzero(T_scale))
    NFAIL(STS_EINVAL, "cnn_pc_set_norm: scalings must be finite, T_scale nonzero");
  net->t_shift = T_shift;
  net->t_scale = T_scale;
  return STS_OK;
}

sts_status cnn_pc_factor(sts_cnn *net, const double *T, double dt, int *used_net) {
  if (!net) return STS_EINVAL;
  sts_status st = pc_checks(net, "cnn_pc_factor", T, dt);
  if (st) return st;
  if ((st = pc_features(net, T, dt))) return st;
  forward_packed(net);
  NLAUNCHCHK();
  st = build_pc_factor(net->ctx, dt, net->d_pred);
  bool used = st == STS_OK;
  if (st == STS_BREAKDOWN) st = build_pc_factor(net->ctx, dt, nullptr);  // point Jacobi
  if (st) return st;
  if (used_net) *used_net = used ? 1 : 0;
  return STS_OK;
}

// features, forward, factor, objective sweeps with the output gradient in
// g(0), back-propagation into grad; the loss partial sum into d_out[0]
static sts_status pc_gradient(sts_cnn *net, const char *name, const double *T, double dt,
                              const double *z, float *grad, bool want_loss) {
  sts_status st = pc_checks(net, name, T, dt);
  if (st) return st;
  if (!z) NFAIL(STS_EINVAL, std::string(name) + ": null z");
  sts_ctx *ctx = net->ctx;
  if ((st = pc_features(net, T, dt))) return st;
  forward_packed(net);
  NLAUNCHCHK();
  if ((st = build_pc_factor(ctx, dt, net->d_pred))) return st;
  if ((st = pc_objective_sweeps(ctx, dt, z, nullptr, net->g(0)))) return st;
  if (want_loss) launch_cnn_sum_parts(net->launch(), ctx->d_red, pc_parts(ctx), net->d_out);
  backward(net, grad);
  NLAUNCHCHK();
  return STS_OK;
}

static sts_status read_loss(sts_cnn *net, double *loss) {
  double h;
  NHIPCHK(hipMemcpyAsync(&h, net->d_out, 8, hipMemcpyDeviceToHost, net->ctx->stream));
  NHIPCHK(hipStreamSynchronize(net->ctx->stream));
  *loss = h / (double)net->ncell;
  return STS_OK;
}

sts_status cnn_pc_grad(sts_cnn *net, const double *T, double dt, const double *z, float *grad,
                       double *loss) {
  if (!net) return STS_EINVAL;
  if (!grad) NFAIL(STS_EINVAL, "cnn_pc_grad: null gradient array");
  sts_status st = pc_gradient(net, "cnn_pc_grad", T, dt, z, grad, loss != nullptr);
  if (st) return st;
  return loss ? read_loss(net, loss) : STS_OK;
}

sts_status cnn_pc_train_step(sts_cnn *net, const double *T, double dt, const double *z, float lr,
                             double *loss) {
  if (!net) return STS_EINVAL;
  if (!(lr > 0.0f) || !std::isfinite(lr)) NFAIL(STS_EINVAL, "cnn_pc_train_step: lr must be > 0");
  sts_status st = pc_gradient(net, "cnn_pc_train_step", T, dt, z, net->d_G, loss != nullptr);
  if (st) return st;
  adam(net, net->d_G, lr);
  NLAUNCHCHK();
  return loss ? read_loss(net, loss) : STS_OK;
}

}  // extern "C"
