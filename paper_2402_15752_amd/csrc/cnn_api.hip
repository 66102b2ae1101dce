// C-ABI of the closure network: workspace layout, parameter initialisation,
// forward, backward (loss and every gradient) and the Adam step.  All
// arithmetic runs in the kernels of cnn.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/cplb.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace pflb;

namespace {

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {16, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 16};
constexpr int kLossParts = 256;   // FP64 loss partials

int num_params() {
  int n = 0;
  for (int l = 0; l < kLayers; ++l) n += kCout[l] * kCin[l] * 9 + kCout[l];
  return n;
}

int w_offset(int l) {  // start of W of layer l in the parameter vector
  int n = 0;
  for (int k = 0; k < l; ++k) n += kCout[k] * kCin[k] * 9 + kCout[k];
  return n;
}

struct CnnLayout {
  size_t theta, m, v, grad, wg[kLayers], wf[kLayers], scale, x0, z[kLayers], a[kLayers],
      dz[kLayers], wpart, bpart, lpart, loss, bal, total;
};

CnnLayout cnn_layout(long long P, int W, int nsamples) {
  CnnLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, kAlign);
    return o;
  };
  const size_t n = (size_t)num_params();
  L.theta = take(n * 4);
  L.m = take(n * 4);
  L.v = take(n * 4);
  L.grad = take(n * 4);
  for (int l = 0; l < kLayers; ++l) {
    L.wg[l] = take((size_t)kCout[l] * 9 * kCin[l] * 2);
    L.wf[l] = take((size_t)kCin[l] * 9 * kCout[l] * 2);
  }
  L.scale = take(16 * 4);
  L.x0 = take((size_t)P * 16 * 2);
  for (int l = 0; l < kLayers; ++l) {
    L.z[l] = take((size_t)P * kCout[l] * 4);
    L.a[l] = take((size_t)P * kCout[l] * 2);
    L.dz[l] = take((size_t)P * kCout[l] * 2);
  }
  const long long nparts = cnn_wgrad_parts(W, P / W);
  L.wpart = take((size_t)nparts * 32 * 9 * 32 * 4);
  L.bpart = take((size_t)nparts * 32 * 4);
  L.lpart = take(kLossParts * 8);
  L.loss = take(8);
  L.bal = take((size_t)cnn_balance_parts(nsamples) * 8);
  L.total = off;
  return L;
}

// splitmix64 and Box-Muller: a portable, seeded normal generator
struct Rng {
  unsigned long long s;
  unsigned long long next() {
    unsigned long long z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

}  // namespace

struct cplb_cnn {
  int nsamples, H, W;
  long long P;
  hipStream_t stream;
  char* ws;
  CnnLayout L;
  long long used_P;  // pixels of the last forward
  int adam_t;
  float out_scale[2];  // output scale of the c1 and c2 corrections
  char err[512];
  template <class X>
  X* at(size_t off) const {
    return (X*)(ws + off);
  }
};

namespace {

__attribute__((format(printf, 3, 4))) int set_err(cplb_cnn_t* c, int code, const char* fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

int hip_check(cplb_cnn_t* c, hipError_t e, const char* where) {
  if (e == hipSuccess) return CPLB_OK;
  return set_err(c, CPLB_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int refresh_weights(cplb_cnn_t* c) {
  for (int l = 0; l < kLayers; ++l) {
    const int rc = hip_check(c, cnn_weights(c->at<float>(c->L.theta) + w_offset(l), kCin[l], kCout[l],
                                            c->at<unsigned short>(c->L.wg[l]),
                                            c->at<unsigned short>(c->L.wf[l]), c->stream),
                             "weight copies");
    if (rc) return rc;
  }
  return CPLB_OK;
}

}  // namespace

extern "C" {

int cplb_cnn_num_params(void) { return num_params(); }

int cplb_cnn_workspace_bytes(int nsamples, int H, int W, size_t* bytes) {
  if (!bytes || nsamples < 1 || H < 1 || W < 1) return CPLB_EINVAL;
  if ((double)nsamples * H * W > 2.0e8) return CPLB_EINVAL;
  *bytes = cnn_layout((long long)nsamples * H * W, W, nsamples).total;
  return CPLB_OK;
}

int cplb_cnn_create(int nsamples, int H, int W, void* dev_workspace, size_t bytes,
                    void* hip_stream, cplb_cnn_t** out) {
  if (!out) return CPLB_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = cplb_cnn_workspace_bytes(nsamples, H, W, &need);
  if (rc) return rc;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign)) return CPLB_EINVAL;
  if (bytes < need) return CPLB_ENOMEM;
  cplb_cnn_t* c = new (std::nothrow) cplb_cnn_t();
  if (!c) return CPLB_ENOMEM;
  c->nsamples = nsamples;
  c->H = H;
  c->W = W;
  c->P = (long long)nsamples * H * W;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)dev_workspace;
  c->L = cnn_layout(c->P, W, nsamples);
  c->used_P = 0;
  c->adam_t = 0;
  c->out_scale[0] = c->out_scale[1] = 1.f;
  c->err[0] = 0;
  const float one[16] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  rc = hip_check(c, hipMemcpyAsync(c->at<float>(c->L.scale), one, sizeof(one),
                                   hipMemcpyHostToDevice, c->stream), "scale upload");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "create synchronise");
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return CPLB_OK;
}

void cplb_cnn_destroy(cplb_cnn_t* c) { delete c; }

int cplb_cnn_set_params(cplb_cnn_t* c, const float* host_theta) {
  if (!c || !host_theta) return CPLB_EINVAL;
  const size_t nb = (size_t)num_params() * 4;
  int rc = hip_check(c, hipMemcpyAsync(c->at<float>(c->L.theta), host_theta, nb,
                                       hipMemcpyHostToDevice, c->stream), "parameter upload");
  if (rc) return rc;
  // Adam state restarts with new parameters (zeroed by a host copy of zeros)
  std::vector<float> zero(num_params(), 0.f);
  rc = hip_check(c, hipMemcpyAsync(c->at<float>(c->L.m), zero.data(), nb, hipMemcpyHostToDevice,
                                   c->stream), "adam state");
  if (!rc) rc = hip_check(c, hipMemcpyAsync(c->at<float>(c->L.v), zero.data(), nb,
                                            hipMemcpyHostToDevice, c->stream), "adam state");
  if (!rc) rc = refresh_weights(c);
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "parameter synchronise");
  c->adam_t = 0;
  return rc;
}

int cplb_cnn_init_params(cplb_cnn_t* c, uint64_t seed) {
  if (!c) return CPLB_EINVAL;
  std::vector<float> theta(num_params(), 0.f);
  Rng r{seed};
  for (int l = 0; l < kLayers; ++l) {
    const double std = std::sqrt(2.0 / (9.0 * kCin[l])) * (l == kLayers - 1 ? 0.1 : 1.0);
    float* w = theta.data() + w_offset(l);
    for (int i = 0; i < kCout[l] * kCin[l] * 9; ++i) w[i] = (float)(std * r.normal());
  }
  return cplb_cnn_set_params(c, theta.data());
}

int cplb_cnn_get_params(cplb_cnn_t* c, float* host_theta) {
  if (!c || !host_theta) return CPLB_EINVAL;
  int rc = hip_check(c, hipMemcpyAsync(host_theta, c->at<float>(c->L.theta),
                                       (size_t)num_params() * 4, hipMemcpyDeviceToHost, c->stream),
                     "parameter download");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "parameter synchronise");
  return rc;
}

int cplb_cnn_get_grads(cplb_cnn_t* c, float* host_grad) {
  if (!c || !host_grad) return CPLB_EINVAL;
  int rc = hip_check(c, hipMemcpyAsync(host_grad, c->at<float>(c->L.grad), (size_t)num_params() * 4,
                                       hipMemcpyDeviceToHost, c->stream), "gradient download");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "gradient synchronise");
  return rc;
}

int cplb_cnn_set_input_scale(cplb_cnn_t* c, const float scale[16]) {
  if (!c || !scale) return CPLB_EINVAL;
  int rc = hip_check(c, hipMemcpyAsync(c->at<float>(c->L.scale), scale, 16 * sizeof(float),
                                       hipMemcpyHostToDevice, c->stream), "scale upload");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "scale synchronise");
  return rc;
}

int cplb_cnn_forward(cplb_cnn_t* c, int nsamples, const float* dev_planes, int cin, float* dev_out) {
  if (!c) return CPLB_EINVAL;
  if (nsamples < 1 || nsamples > c->nsamples)
    return set_err(c, CPLB_EINVAL, "nsamples %d outside 1..%d", nsamples, c->nsamples);
  if (cin < 1 || cin > 16) return set_err(c, CPLB_EINVAL, "input planes %d outside 1..16", cin);
  if (!dev_planes) return set_err(c, CPLB_EINVAL, "null input planes");
  const long long hw = (long long)c->H * c->W, P = nsamples * hw;
  const int rows = nsamples * c->H;
  int rc = hip_check(c, cnn_pack(dev_planes, cin, c->at<float>(c->L.scale), hw, P,
                                 c->at<unsigned short>(c->L.x0), c->stream), "input packing");
  if (rc) return rc;
  const unsigned short* x = c->at<unsigned short>(c->L.x0);
  for (int l = 0; l < kLayers; ++l) {
    const float* bias = c->at<float>(c->L.theta) + w_offset(l) + kCout[l] * kCin[l] * 9;
    rc = hip_check(c, cnn_conv(l, kConvForward, x, c->at<unsigned short>(c->L.wg[l]), bias,
                               c->at<float>(c->L.z[l]), c->at<unsigned short>(c->L.a[l]), nullptr,
                               c->H, c->W, rows, 1.f, 1.f, c->stream), "forward convolution");
    if (rc) return rc;
    x = c->at<unsigned short>(c->L.a[l]);
  }
  c->used_P = P;
  if (dev_out) {
    rc = hip_check(c, cnn_output(c->at<float>(c->L.z[kLayers - 1]), P, hw, c->out_scale[0],
                                 c->out_scale[1], dev_out, c->stream), "output copy");
    if (!rc)
      rc = hip_check(c, cnn_balance(dev_out, nsamples, hw, c->at<double>(c->L.bal), c->stream),
                     "output balance");
  }
  return rc;
}

int cplb_cnn_infer(cplb_cnn_t* c, int nsamples, const float* dev_planes, int cin, float* dev_out) {
  if (!c) return CPLB_EINVAL;
  if (nsamples < 1 || nsamples > c->nsamples)
    return set_err(c, CPLB_EINVAL, "nsamples %d outside 1..%d", nsamples, c->nsamples);
  if (cin < 1 || cin > 16) return set_err(c, CPLB_EINVAL, "input planes %d outside 1..16", cin);
  if (!dev_planes || !dev_out) return set_err(c, CPLB_EINVAL, "null input planes or output");
  const long long hw = (long long)c->H * c->W, P = nsamples * hw;
  const int rows = nsamples * c->H;
  int rc = hip_check(c, cnn_pack(dev_planes, cin, c->at<float>(c->L.scale), hw, P,
                                 c->at<unsigned short>(c->L.x0), c->stream), "input packing");
  if (rc) return rc;
  // activations ping-pong between a[0] and a[1]; no FP32 pre-activations
  const unsigned short* x = c->at<unsigned short>(c->L.x0);
  for (int l = 0; l < kLayers && rc == CPLB_OK; ++l) {
    const float* bias = c->at<float>(c->L.theta) + w_offset(l) + kCout[l] * kCin[l] * 9;
    unsigned short* a = c->at<unsigned short>(c->L.a[l % 2]);
    const bool last = l == kLayers - 1;
    rc = hip_check(c, cnn_conv(l, last ? kConvInferOut : kConvInfer, x,
                               c->at<unsigned short>(c->L.wg[l]), bias, last ? dev_out : nullptr,
                               a, nullptr, c->H, c->W, rows, c->out_scale[0], c->out_scale[1],
                               c->stream),
                   "inference convolution");
    x = a;
  }
  if (!rc)
    rc = hip_check(c, cnn_balance(dev_out, nsamples, hw, c->at<double>(c->L.bal), c->stream),
                   "output balance");
  c->used_P = 0;  // the training buffers of the last forward are gone
  return rc;
}

int cplb_cnn_set_stream(cplb_cnn_t* c, void* hip_stream) {
  if (!c) return CPLB_EINVAL;
  c->stream = (hipStream_t)hip_stream;
  return CPLB_OK;
}

int cplb_cnn_backward(cplb_cnn_t* c, const float* dev_target, double* loss) {
  if (!c) return CPLB_EINVAL;
  if (!dev_target) return set_err(c, CPLB_EINVAL, "null target");
  if (c->used_P == 0) return set_err(c, CPLB_EINVAL, "backward needs a forward first");
  const long long P = c->used_P;
  const int rows = (int)(P / c->W);
  double* dloss = c->at<double>(c->L.loss);
  int rc = hip_check(c, cnn_loss(c->at<float>(c->L.z[kLayers - 1]), dev_target, P,
                                 (long long)c->H * c->W, c->at<unsigned short>(c->L.dz[kLayers - 1]),
                                 c->at<double>(c->L.lpart), kLossParts, dloss, c->stream),
                     "loss");
  if (rc) return rc;
  float* grad = c->at<float>(c->L.grad);
  for (int l = kLayers - 1; l >= 0 && rc == CPLB_OK; --l) {
    const unsigned short* xin = l == 0 ? c->at<unsigned short>(c->L.x0) : c->at<unsigned short>(c->L.a[l - 1]);
    const int wo = w_offset(l);
    rc = hip_check(c, cnn_wgrad(l, xin, c->at<unsigned short>(c->L.dz[l]), c->at<float>(c->L.wpart),
                                c->at<float>(c->L.bpart), c->H, c->W, rows, grad + wo,
                                grad + wo + kCout[l] * kCin[l] * 9, c->stream),
                   "weight gradient");
    if (rc || l == 0) break;
    rc = hip_check(c, cnn_conv(l, kConvAdjoint, c->at<unsigned short>(c->L.dz[l]),
                               c->at<unsigned short>(c->L.wf[l]), nullptr, nullptr,
                               c->at<unsigned short>(c->L.dz[l - 1]), c->at<float>(c->L.z[l - 1]),
                               c->H, c->W, rows, 1.f, 1.f, c->stream), "input gradient");
  }
  if (rc) return rc;
  if (loss) {
    rc = hip_check(c, hipMemcpyAsync(loss, dloss, sizeof(double), hipMemcpyDeviceToHost, c->stream),
                   "loss copy");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "loss synchronise");
  }
  return rc;
}

int cplb_cnn_adam(cplb_cnn_t* c, float lr, float beta1, float beta2, float eps) {
  if (!c) return CPLB_EINVAL;
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return set_err(c, CPLB_EINVAL, "invalid Adam hyper-parameters");
  c->adam_t++;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, c->adam_t));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, c->adam_t));
  int rc = hip_check(c, cnn_adam(c->at<float>(c->L.theta), c->at<float>(c->L.m), c->at<float>(c->L.v),
                                 c->at<float>(c->L.grad), num_params(), lr, beta1, beta2, eps, bc1,
                                 bc2, c->stream), "adam");
  if (!rc) rc = refresh_weights(c);
  return rc;
}

int cplb_cnn_set_output_scale(cplb_cnn_t* c, float scale1, float scale2) {
  if (!c || !std::isfinite(scale1) || !std::isfinite(scale2)) return CPLB_EINVAL;
  c->out_scale[0] = scale1;
  c->out_scale[1] = scale2;
  return CPLB_OK;
}

int cplb_cnn_restrict(void* hip_stream, const float* dev_fine, int nsamples, int H, int W, int f,
                      float* dev_coarse) {
  if (!dev_fine || !dev_coarse || nsamples < 1 || H < 1 || W < 1 || f < 1) return CPLB_EINVAL;
  return cnn_restrict(dev_fine, nsamples, H, W, f, dev_coarse, (hipStream_t)hip_stream) ==
                 hipSuccess
             ? CPLB_OK
             : CPLB_EHIP;
}

const char* cplb_cnn_last_error(const cplb_cnn_t* c) { return c ? c->err : "null network"; }

}  // extern "C"
