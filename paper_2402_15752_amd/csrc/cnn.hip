// Closure network: forward, backward and Adam on the GPU, with BF16 MFMA
// (v_mfma_f32_16x16x16_bf16, FP32 accumulate) for every convolution.
//
// Network (fixed): four 3x3 correlations 16 -> 32 -> 32 -> 32 -> 16 with
// leaky-ReLU (slope 0.1) after the first three; the output is channel 0 of
// the last layer.  Padding: periodic along x, zero outside the sample along
// y (samples are stacked along y).
//
// Layouts.  Activations are NHWC, pixel p = (sample * H + y) * W + x.  The
// FP32 master parameters follow W[co][ci][ky][kx], b[co] per layer.  For
// the MFMA the weights are kept in BF16 as Wg[co][k], k = tap * C_in + ci
// (tap = 3 ky + kx), so that the four K-consecutive values a lane needs are
// one 8-byte load; the adjoint (input gradient) uses the flipped transpose
// Wf[ci][tap' * C_out + co] = W[co][ci][8 - tap'], which turns the adjoint
// of the padded correlation into a forward correlation with the same
// padding.
//
// MFMA 16x16x16 operand layout (lane l, g = l / 16, j = 0..3):
//   A[m][k]: lane holds A[l % 16][4 g + j];  B[k][n]: B[4 g + j][l % 16];
//   D[m][n]: lane holds D[4 g + j][l % 16].
#include <hip/hip_runtime.h>

#include "../../include/cplb.h"
#include "kernels.hpp"

namespace pflb {

namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr float kSlope = 0.1f;

// FP32 -> BF16 with round to nearest, ties to even (finite inputs)
__device__ inline unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline short4v load4(const unsigned short* p) {
  return __builtin_bit_cast(short4v, *(const unsigned long long*)p);
}

__device__ inline float4v mfma(short4v a, short4v b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

enum { kFwdAct = 0, kFwdLinear = 1, kBwd = 2, kInfAct = 3, kInfOut = 4 };

// Tile of the convolution kernels: kConvRows rows x kConvCols pixels, one
// row per wave (4 waves), kConvCols / 16 groups of 16 pixels per wave.
constexpr int kConvRows = 4;
constexpr int kConvCols = 32;

// Each block stages its input rows (with a one-pixel halo, periodic in x)
// and the layer's BF16 weights in LDS once, then every wave runs its row x
// all COUT channels with both MFMA operands read from LDS.  Pixel and weight
// rows are padded by 8 bytes so that the 16 lanes of a 64-bit LDS read hit
// distinct banks.  The accumulation order (tap, channel group, MFMA) is that
// of a direct loop over the taps.
// kFwdAct / kFwdLinear: Z = conv(X) + b (FP32), A = act(Z) (BF16).
// kInfAct: A = lrelu(conv(X) + b) only (inference: no FP32 copy).
// kInfOut: out[p] = scale * (conv(X) + b)[channel 0], written to Z.
// kBwd: X is dZ of the layer above, W its flipped transpose; the result is
// dA of the layer below, written as dZ = dA * lrelu'(Zprev) in BF16.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const unsigned short* __restrict__ X,
                                                   const unsigned short* __restrict__ Wg,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ Z,
                                                   unsigned short* __restrict__ A,
                                                   const float* __restrict__ Zprev, int H, int W,
                                                   int rows, float scale) {
  constexpr int NT = COUT / 16, K = 9 * CIN, G = kConvCols / 16;
  constexpr int PS = CIN + 4;            // LDS pixel stride (BF16 values)
  constexpr int KS = K + 4;              // LDS weight-row stride
  constexpr int LC = kConvCols + 2, LR = kConvRows + 2;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels in multiples of 16");
  __shared__ __align__(16) unsigned short sx[LR * LC * PS];
  __shared__ __align__(16) unsigned short sw[COUT * KS];
  typedef unsigned long long u64;

  const int tiles_x = (W + kConvCols - 1) / kConvCols;
  const int x0 = (blockIdx.x % tiles_x) * kConvCols;
  const int R0 = (blockIdx.x / tiles_x) * kConvRows;
  // stage the input rows R0-1 .. R0+kConvRows and columns x0-1 .. x0+kConvCols
  // (wrapped in x; columns past x = W and rows outside the batch are zero;
  // the zero padding in y between samples is applied per tap below)
  for (int e = threadIdx.x; e < LR * LC * (CIN / 4); e += 256) {
    const int c4 = e % (CIN / 4), pix = e / (CIN / 4);
    const int lr = pix / LC, lc = pix % LC;
    const int Rg = R0 + lr - 1;
    int xs = x0 + lc - 1;
    u64 v = 0;
    if (Rg >= 0 && Rg < rows && xs <= W) {
      xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
      v = *(const u64*)(X + ((long long)Rg * W + xs) * CIN + c4 * 4);
    }
    *(u64*)(sx + (lr * LC + lc) * PS + c4 * 4) = v;
  }
  for (int e = threadIdx.x; e < COUT * (K / 4); e += 256) {
    const int k4 = e % (K / 4), co = e / (K / 4);
    *(u64*)(sw + co * KS + k4 * 4) = *(const u64*)(Wg + (long long)co * K + k4 * 4);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = R0 + wave;  // global row (sample * H + y) of this wave
  if (R >= rows) return;
  const int m = lane & 15, g = lane >> 4;
  const int y = R % H;
  float4v acc[G][NT];
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[q][t] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    if (y + dy < 0 || y + dy >= H) continue;  // zero padding in y (uniform per wave)
    const unsigned short* xrow = sx + (wave + 1 + dy) * LC * PS;
#pragma unroll
    for (int cg = 0; cg < CIN / 16; ++cg) {
      const int k = tap * CIN + cg * 16 + 4 * g;
      short4v b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = __builtin_bit_cast(short4v, *(const u64*)(sw + (t * 16 + m) * KS + k));
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int col = q * 16 + m + dx + 1;  // LDS column of this lane's A row
        const short4v a =
            __builtin_bit_cast(short4v, *(const u64*)(xrow + col * PS + cg * 16 + 4 * g));
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = mfma(a, b[t], acc[q][t]);
      }
    }
  }
  // D[pixel 4 g + j][channel l % 16]
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int xq = x0 + q * 16;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + m;
      if (MODE == kInfOut && co != 0) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int xp = xq + 4 * g + j;
        if (xp >= W) continue;
        const long long p = (long long)R * W + xp;
        float v = acc[q][t][j];
        if (MODE == kBwd) {
          const float zp = Zprev[p * COUT + co];
          v *= zp > 0.f ? 1.f : kSlope;
          A[p * COUT + co] = to_bf16(v);
        } else if (MODE == kInfOut) {
          Z[p] = scale * (v + bias[0]);
        } else {
          v += bias[co];
          if (MODE != kInfAct) Z[p * COUT + co] = v;
          A[p * COUT + co] = to_bf16(MODE == kFwdLinear ? v : (v > 0.f ? v : kSlope * v));
        }
      }
    }
  }
}

// Weight and bias gradients, per chunk of pixels:
//   partial[chunk][co][k] = sum_p dZ[p][co] * X(p shifted by tap(k))[ci(k)],
//   bpart[chunk][co]      = sum_p dZ[p][co].
// One wave per 16-wide tile of k = tap * CIN + ci and chunk, all output
// channels at once (the shifted-X operand is loaded once for every co tile);
// the pixel sum is the MFMA's K dimension.  Each lane walks its four pixels
// p = pb + 4 g + j with 32-bit row / column counters instead of dividing.
// The k tile 0 also sums its dZ operand for the bias.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(const unsigned short* __restrict__ X,
                                                    const unsigned short* __restrict__ dZ,
                                                    float* __restrict__ partial,
                                                    float* __restrict__ bpart, int H, int W,
                                                    int P, int chunk) {
  constexpr int K = 9 * CIN, MT = COUT / 16, NTL = K / 16;
  const int lane = threadIdx.x & 63;
  const int nt = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (nt >= NTL) return;
  const int c = blockIdx.y;
  const int m = lane & 15, g = lane >> 4;
  const int kk = nt * 16 + m;  // B column of this lane
  const int tap = kk / CIN, ci = kk % CIN;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int p0 = c * chunk;
  const int p1 = p0 + chunk < P ? p0 + chunk : P;
  // row R (sample * H + y), column x and y of the lane's pixel p0 + 4 g + j
  int R[4], xc[4], yc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = p0 + 4 * g + j;
    R[j] = p / W;
    xc[j] = p - R[j] * W;
    yc[j] = R[j] % H;
  }
  float4v acc[MT];
  float bsum[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    acc[t] = float4v{0.f, 0.f, 0.f, 0.f};
    bsum[t] = 0.f;
  }
  for (int pb = p0; pb < p1; pb += 16) {
    short4v a[MT], b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = pb + 4 * g + j;
      const bool valid = p < p1;
      unsigned short bv = 0;
      if (valid && yc[j] + dy >= 0 && yc[j] + dy < H) {
        int xs = xc[j] + dx;
        xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
        bv = X[((long long)(R[j] + dy) * W + xs) * CIN + ci];
      }
      b[j] = (short)bv;
#pragma unroll
      for (int t = 0; t < MT; ++t)
        a[t][j] = (short)(valid ? dZ[(long long)p * COUT + t * 16 + m] : (unsigned short)0);
      // advance to pixel p + 16
      xc[j] += 16;
      while (xc[j] >= W) {
        xc[j] -= W;
        ++R[j];
        if (++yc[j] == H) yc[j] = 0;
      }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      acc[t] = mfma(a[t], b, acc[t]);
      if (nt == 0)
        bsum[t] += (from_bf16((unsigned short)a[t][0]) + from_bf16((unsigned short)a[t][1])) +
                   (from_bf16((unsigned short)a[t][2]) + from_bf16((unsigned short)a[t][3]));
    }
  }
  // D[co row 4 g + j][k column l % 16]
  float* out = partial + (long long)c * COUT * K;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(t * 16 + 4 * g + j) * K + nt * 16 + m] = acc[t][j];
  if (nt == 0) {
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      float v = bsum[t];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (g == 0) bpart[c * COUT + t * 16 + m] = v;
    }
  }
}

// grad W[co][ci][ky][kx] = sum over chunks of partial[chunk][co][tap * CIN + ci];
// grad b[co] = sum over chunks of bpart[chunk][co]
__global__ void wgrad_reduce(const float* __restrict__ partial, const float* __restrict__ bpart,
                             int nchunks, int cin, int cout, float* __restrict__ gradW,
                             float* __restrict__ gradb) {
  const int K = 9 * cin;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // oracle layout index
  if (i < cout * K) {
    const int co = i / K, r = i % K, ci = r / 9, tap = r % 9;
    const long long src = (long long)co * K + tap * cin + ci;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partial[(long long)c * cout * K + src];
    gradW[i] = s;
  } else if (i < cout * K + cout) {
    const int co = i - cout * K;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += bpart[c * cout + co];
    gradb[co] = s;
  }
}

// FP32 planes [sample][c][y][x] (c < cin) -> X0[p][16] in BF16, scaled
__global__ void pack_kernel(const float* __restrict__ planes, int cin, const float* __restrict__ scale,
                            long long hw, long long P, unsigned short* __restrict__ X0) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= P * 16) return;
  const long long p = i / 16;
  const int c = (int)(i % 16);
  const long long s = p / hw, q = p % hw;
  X0[i] = c < cin ? to_bf16(scale[c] * planes[(s * cin + c) * hw + q]) : (unsigned short)0;
}

// out[p] = scale * Z4[p][0]
__global__ void output_kernel(const float* __restrict__ Z4, long long P, float scale,
                              float* __restrict__ out) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p < P) out[p] = scale * Z4[p * 16];
}

__global__ void restrict_kernel(const float* __restrict__ fine, int nsamples, int H, int W, int f,
                                float* __restrict__ coarse) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long n = (long long)nsamples * H * W;
  if (i >= n) return;
  const long long s = i / ((long long)H * W);
  const int r = (int)(i % ((long long)H * W));
  const int y = r / W, x = r % W;
  const long long Wf = (long long)W * f;
  const float* base = fine + s * (long long)H * f * Wf;
  float acc = 0.f;
  for (int j = 0; j < f; ++j)
    for (int k = 0; k < f; ++k) acc += base[(long long)(f * y + j) * Wf + f * x + k];
  coarse[i] = acc / (float)(f * f);
}

// loss partials (FP64) and dZ4 = d(mean (z - t)^2) / dz4 in BF16 (channel 0)
__global__ void loss_kernel(const float* __restrict__ Z4, const float* __restrict__ target,
                            long long P, unsigned short* __restrict__ dZ4,
                            double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += stride) {
    const float r = Z4[p * 16] - target[p];
    s += (double)r * (double)r;
    dZ4[p * 16] = to_bf16(2.0f * r / (float)P);
#pragma unroll
    for (int c = 1; c < 16; ++c) dZ4[p * 16 + c] = 0;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials(const double* __restrict__ partial, int n, long long P,
                             double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)P;
}

// Adam on the FP32 master parameters (bias-corrected step size c1 / (sqrt(v^) + eps))
__global__ void adam_kernel(float* __restrict__ theta, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ grad, int n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 GEMM copies of one layer: Wg[co][tap * cin + ci] and the flipped
// transpose Wf[ci][tap' * cout + co] = W[co][ci][8 - tap']
__global__ void weights_kernel(const float* __restrict__ W, int cin, int cout,
                               unsigned short* __restrict__ Wg, unsigned short* __restrict__ Wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // oracle layout
  if (i >= cout * cin * 9) return;
  const int co = i / (cin * 9), r = i % (cin * 9), ci = r / 9, tap = r % 9;
  const unsigned short h = to_bf16(W[i]);
  Wg[(long long)co * 9 * cin + tap * cin + ci] = h;
  Wf[(long long)ci * 9 * cout + (8 - tap) * cout + co] = h;
}

}  // namespace

// ------------------------------------------------------------------ launch

hipError_t cnn_conv(int layer, int mode, const unsigned short* X, const unsigned short* Wg,
                    const float* bias, float* Z, unsigned short* A, const float* Zprev, int H,
                    int W, int rows, float scale, hipStream_t s) {
  const long long blocks =
      (long long)((W + kConvCols - 1) / kConvCols) * ((rows + kConvRows - 1) / kConvRows);
  const dim3 grid((unsigned)blocks), blk(256);
#define PFLB_CONV(CI, CO, MO) \
  hipLaunchKernelGGL((conv_kernel<CI, CO, MO>), grid, blk, 0, s, X, Wg, bias, Z, A, Zprev, H, W, rows, scale)
  // forward: layer l maps C_in(l) -> C_out(l); backward (the adjoint of
  // layer l) maps C_out(l) -> C_in(l)
  switch (mode) {
    case kFwdAct:
    case kFwdLinear:
      switch (layer) {
        case 0: PFLB_CONV(16, 32, kFwdAct); break;
        case 1: case 2: PFLB_CONV(32, 32, kFwdAct); break;
        default: PFLB_CONV(32, 16, kFwdLinear);
      }
      break;
    case kInfAct:
    case kInfOut:
      switch (layer) {
        case 0: PFLB_CONV(16, 32, kInfAct); break;
        case 1: case 2: PFLB_CONV(32, 32, kInfAct); break;
        default: PFLB_CONV(32, 16, kInfOut);
      }
      break;
    default:
      switch (layer) {
        case 1: case 2: PFLB_CONV(32, 32, kBwd); break;
        case 3: PFLB_CONV(16, 32, kBwd); break;
        default: return hipErrorInvalidValue;  // the input layer needs no input gradient
      }
  }
#undef PFLB_CONV
  return hipGetLastError();
}

hipError_t cnn_wgrad(int layer, const unsigned short* X, const unsigned short* dZ, float* partial,
                     float* bpart, int nchunks, int chunk, int H, int W, long long P, float* gradW,
                     float* gradb, hipStream_t s) {
  const int cin = layer == 0 ? 16 : 32, cout = layer == 3 ? 16 : 32;
  const int ntiles = 9 * cin / 16;
  const dim3 grid((ntiles + 3) / 4, nchunks), blk(256);
  const int Pi = (int)P;
  switch (layer) {
    case 0: hipLaunchKernelGGL((wgrad_kernel<16, 32>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, Pi, chunk); break;
    case 1: case 2: hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, Pi, chunk); break;
    default: hipLaunchKernelGGL((wgrad_kernel<32, 16>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, Pi, chunk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = cout * cin * 9 + cout;
  hipLaunchKernelGGL(wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, partial, bpart, nchunks,
                     cin, cout, gradW, gradb);
  return hipGetLastError();
}

hipError_t cnn_pack(const float* planes, int cin, const float* scale, long long hw, long long P,
                    unsigned short* X0, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((P * 16 + 255) / 256)), dim3(256), 0, s, planes,
                     cin, scale, hw, P, X0);
  return hipGetLastError();
}

hipError_t cnn_output(const float* Z4, long long P, float scale, float* out, hipStream_t s) {
  hipLaunchKernelGGL(output_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, Z4, P,
                     scale, out);
  return hipGetLastError();
}

hipError_t cnn_restrict(const float* fine, int nsamples, int H, int W, int f, float* coarse,
                        hipStream_t s) {
  const long long n = (long long)nsamples * H * W;
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fine,
                     nsamples, H, W, f, coarse);
  return hipGetLastError();
}

hipError_t cnn_loss(const float* Z4, const float* target, long long P, unsigned short* dZ4,
                    double* partial, int nparts, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(nparts), dim3(256), 0, s, Z4, target, P, dZ4, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, partial, nparts, P, loss);
  return hipGetLastError();
}

hipError_t cnn_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float b1,
                    float b2, float eps, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta, m, v, grad, n, lr,
                     b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t cnn_weights(const float* W, int cin, int cout, unsigned short* Wg, unsigned short* Wf,
                       hipStream_t s) {
  const int n = cout * cin * 9;
  hipLaunchKernelGGL(weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, W, cin, cout, Wg, Wf);
  return hipGetLastError();
}

}  // namespace pflb
