// Closure network: forward, backward and Adam on the GPU, with BF16 MFMA
// and FP32 accumulation: v_mfma_f32_16x16x32_bf16 for the convolutions
// (forward, adjoint, inference), v_mfma_f32_16x16x16_bf16 for the weight
// gradients.
//
// Network (fixed): four 3x3 correlations 16 -> 32 -> 32 -> 32 -> 16 with
// leaky-ReLU (slope 0.1) after the first three; the outputs are channels 0
// and 1 of the last layer (the corrections of c1 and c2).  Padding: periodic along x, zero outside the sample along
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
// MFMA operand layouts (lane l, g = l / 16):
//   16x16x16: A[m][k]: lane holds A[l % 16][4 g + j], B[k][n]: B[4 g + j][l % 16]
//             (j = 0..3);
//   16x16x32: A[m][k]: lane holds A[l % 16][8 g + j], B[k][n]: B[8 g + j][l % 16]
//             (j = 0..7);
//   both:     D[m][n]: lane holds D[4 g + j][l % 16] (j = 0..3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "../../include/cplb.h"
#include "kernels.hpp"

namespace pflb {

namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr float kSlope = 0.1f;
constexpr int kOut = 2;  // output channels: the corrections of c1 and c2

// FP32 -> BF16 with round to nearest, ties to even (finite inputs)
__device__ inline unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline float4v mfma(short4v a, short4v b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's double-rate shape: A[m][k] lane l holds A[l % 16][8 g + j],
// B[k][n] lane l holds B[8 g + j][l % 16] (g = l / 16, j = 0..7); D as above
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ inline float4v mfma32(bf16x8 a, bf16x8 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline bf16x8 lds8(const unsigned short* p) {
  return __builtin_bit_cast(bf16x8, *(const uint4*)p);
}

enum { kFwdAct = 0, kFwdLinear = 1, kBwd = 2, kInfAct = 3, kInfOut = 4 };

// Tiles of the convolution kernels: rows of kConvCols pixels, one row per
// wave, kConvCols / 16 groups of 16 pixels per wave.  A forward, adjoint or
// inference convolution takes kConvRowsF rows per work-group (the layer's
// weights are staged once per 256 pixels: 5-7 % faster than 4 rows at the
// closure's batch sizes, same results bit for bit); the weight gradient
// takes kConvRows rows per tile.
constexpr int kConvRows = 4;
constexpr int kConvCols = 32;
constexpr int kConvRowsF = 8;
// work-groups (one partial each) of the weight gradient: at most
// kWgradParts, each taking at least kWgradTiles pixel tiles, so that the
// partials its reduction reads stay small at any batch size
constexpr int kWgradTiles = 2;
constexpr int kWgradParts = 1024;

// LDS staging of the convolution tiles.  Each thread issues all of its
// global loads before its LDS stores (fixed trip counts, unrolled), so a
// tile's loads are in flight together instead of one round trip per slot.
//
// stage_rows: rows R0-1 .. R0+kConvRows and columns x0-1 .. x0+kConvCols of
// an NHWC BF16 tensor of C channels (pixel stride PS in LDS), wrapped in x;
// columns past x = W and rows outside [0, rows) are zero.
// (in two halves: load_rows into registers, store_rows into LDS, so a
// persistent work-group can fetch its next tile while it computes one)
template <int C, int ROWS, int NTH>
constexpr int rows_per_thread() {
  return ((kConvCols + 2) * (ROWS + 2) * (C / 4) + NTH - 1) / NTH;
}

template <int C, int ROWS, int NTH>
__device__ inline void load_rows(const unsigned short* __restrict__ X,
                                 unsigned long long (&v)[rows_per_thread<C, ROWS, NTH>()], int R0,
                                 int x0, int W, int rows) {
  typedef unsigned long long u64;
  constexpr int LC = kConvCols + 2, LR = ROWS + 2, N = LR * LC * (C / 4);
  constexpr int IT = rows_per_thread<C, ROWS, NTH>();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    const int c4 = e % (C / 4), pix = e / (C / 4);
    const int lr = pix / LC, lc = pix % LC;
    const int Rg = R0 + lr - 1;
    int xs = x0 + lc - 1;
    v[it] = 0;
    if (e < N && Rg >= 0 && Rg < rows && xs <= W) {
      xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
      v[it] = *(const u64*)(X + ((long long)Rg * W + xs) * C + c4 * 4);
    }
  }
}

template <int C, int PS, int ROWS, int NTH>
__device__ inline void store_rows(unsigned short* sx,
                                  const unsigned long long (&v)[rows_per_thread<C, ROWS, NTH>()]) {
  typedef unsigned long long u64;
  constexpr int LC = kConvCols + 2, LR = ROWS + 2, N = LR * LC * (C / 4);
  constexpr int IT = rows_per_thread<C, ROWS, NTH>();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    if (e < N) *(u64*)(sx + (e / (C / 4)) * PS + (e % (C / 4)) * 4) = v[it];
  }
}

template <int C, int PS, int ROWS = kConvRows, int NTH = 256>
__device__ inline void stage_rows(const unsigned short* __restrict__ X, unsigned short* sx, int R0,
                                  int x0, int W, int rows) {
  unsigned long long v[rows_per_thread<C, ROWS, NTH>()];
  load_rows<C, ROWS, NTH>(X, v, R0, x0, W, rows);
  store_rows<C, PS, ROWS, NTH>(sx, v);
}

// stage_matrix: NR rows of NC BF16 values (NC % 4 == 0, row i starts at
// src + i * src_stride) into LDS rows of stride LS; rows with valid(i) false
// are zero.
template <int NR, int NC, int LS, int NTH = 256, class Valid, class Src>
__device__ inline void stage_matrix(Src src_row, unsigned short* dst, Valid valid) {
  typedef unsigned long long u64;
  constexpr int N = NR * (NC / 4), IT = (N + NTH - 1) / NTH;
  u64 v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    const int i = e / (NC / 4), c4 = e % (NC / 4);
    v[it] = 0;
    if (e < N && valid(i)) v[it] = *(const u64*)(src_row(i) + c4 * 4);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    if (e < N) *(u64*)(dst + (e / (NC / 4)) * LS + (e % (NC / 4)) * 4) = v[it];
  }
}


// Each block stages its input rows (with a one-pixel halo, periodic in x)
// and the layer's BF16 weights in LDS once, then every wave runs its row x
// all COUT channels with both MFMA operands read from LDS, 32 values of the
// K = 9 CIN reduction (k = tap CIN + ci) per 16x16x32 MFMA: one tap of 32
// channels, or two taps of 16 channels (K padded with zero weights to a
// multiple of 32).  Pixel and weight rows are padded by 16 bytes so that the
// 16 lanes of a 128-bit LDS read hit distinct banks.
// kFwdAct / kFwdLinear: Z = conv(X) + b (FP32), A = act(Z) (BF16).
// kInfAct: A = lrelu(conv(X) + b) only (inference: no FP32 copy).
// kInfOut: out[sample][c][q] = scale_c * (conv(X) + b)[channel c] for the
// kOut output channels, written to Z ([sample][kOut][H W] planes).
// kBwd: X is dZ of the layer above, W its flipped transpose; the result is
// dA of the layer below, written as dZ = dA * lrelu'(Zprev) in BF16.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(64 * kConvRowsF) void conv_kernel(const unsigned short* __restrict__ X,
                                                   const unsigned short* __restrict__ Wg,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ Z,
                                                   unsigned short* __restrict__ A,
                                                   const float* __restrict__ Zprev, int H, int W,
                                                   int rows, float scale0, float scale1) {
  constexpr int NT = COUT / 16, K = 9 * CIN, G = kConvCols / 16;
  constexpr int NK = (K + 31) / 32;      // K steps of 32
  constexpr int PS = CIN + 8;            // LDS pixel stride (BF16 values)
  constexpr int KS = 32 * NK + 8;        // LDS weight-row stride
  constexpr int LC = kConvCols + 2, LR = kConvRowsF + 2;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels in multiples of 16");
  __shared__ __align__(16) unsigned short sx[LR * LC * PS];
  __shared__ __align__(16) unsigned short sw[COUT * KS];
  typedef unsigned long long u64;

  const int tiles_x = (W + kConvCols - 1) / kConvCols;
  const int ntiles = tiles_x * ((rows + kConvRowsF - 1) / kConvRowsF);
  constexpr int NTH = 64 * kConvRowsF;
  // the layer's weights, once per work-group
  stage_matrix<COUT, K, KS, NTH>([&](int co) { return Wg + (long long)co * K; }, sw,
                                 [](int) { return true; });
  if constexpr (32 * NK > K) {
    // zero weights of the padded K range
    for (int e = threadIdx.x; e < COUT * (32 * NK - K); e += NTH)
      sw[(e / (32 * NK - K)) * KS + K + e % (32 * NK - K)] = 0;
  }
  // Persistent work-group: tiles blockIdx.x, blockIdx.x + gridDim.x, ...
  // The input rows R0-1 .. R0+kConvRowsF and columns x0-1 .. x0+kConvCols of
  // the next tile (the zero padding in y between samples is applied per tap
  // below) are loaded into registers while the current tile is computed.
  u64 nxt[rows_per_thread<CIN, kConvRowsF, NTH>()];
  int tile = blockIdx.x;
  if (tile < ntiles)
    load_rows<CIN, kConvRowsF, NTH>(X, nxt, (tile / tiles_x) * kConvRowsF, (tile % tiles_x) * kConvCols,
                                    W, rows);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  for (; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tiles_x) * kConvCols;
    const int R0 = (tile / tiles_x) * kConvRowsF;
    __syncthreads();  // every wave is done with the previous tile's rows
    store_rows<CIN, PS, kConvRowsF, NTH>(sx, nxt);
    __syncthreads();  // the rows (and, the first time, the weights) are in place
    const int next = tile + gridDim.x;
    if (next < ntiles)
      load_rows<CIN, kConvRowsF, NTH>(X, nxt, (next / tiles_x) * kConvRowsF,
                                      (next % tiles_x) * kConvCols, W, rows);
    const int R = R0 + wave;  // global row (sample * H + y) of this wave
    if (R >= rows) continue;
    const int y = R % H;
    float4v acc[G][NT];
#pragma unroll
    for (int q = 0; q < G; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[q][t] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      // this lane's 8 values of the K step: tap and first channel
      const int k = 32 * ks + 8 * g;
      const int tap = k / CIN, ci = k % CIN;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      // zero padding in y, and the zero-weight K padding past the ninth tap
      const bool live = tap < 9 && y + dy >= 0 && y + dy < H;
      const unsigned short* xrow = sx + (wave + 1 + (tap < 9 ? dy : 0)) * LC * PS;
      bf16x8 b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = lds8(sw + (t * 16 + m) * KS + k);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int col = q * 16 + m + (tap < 9 ? dx : 0) + 1;  // LDS column of this lane's A row
        bf16x8 a = lds8(xrow + col * PS + ci);
        if (!live) a = bf16x8{};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = mfma32(a, b[t], acc[q][t]);
      }
    }
    // D[pixel 4 g + j][channel l % 16]
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int xq = x0 + q * 16;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + m;
        if (MODE == kInfOut && co >= kOut) continue;
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
            const long long q = (long long)(R % H) * W + xp, hw = (long long)H * W;
            Z[((long long)(R / H) * kOut + co) * hw + q] = (co == 0 ? scale0 : scale1) * (v + bias[co]);
          } else {
            v += bias[co];
            if (MODE != kInfAct) Z[p * COUT + co] = v;
            A[p * COUT + co] = to_bf16(MODE == kFwdLinear ? v : (v > 0.f ? v : kSlope * v));
          }
        }
      }
    }
  }
}

// Weight and bias gradients, per work-group of the pixel tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...
// (kConvRows x kConvCols pixels each, the convolution's tiles):
//   partial[g][co][k] = sum_p dZ[p][co] * X(p shifted by tap(k))[ci(k)],
//   bpart[g][co]      = sum_p dZ[p][co],
// with k = tap * CIN + ci.  Per tile the group stages its input rows with a
// one-pixel halo (periodic in x, as the convolution) and its dZ rows in LDS;
// then wave w accumulates the k tiles w, w + 4, ... for all output channels,
// 16 pixels (one MFMA K step, within one row) at a time: the A operand is
// dZ transposed, the B operand the shifted input.  A K step whose row has
// tap's neighbour row outside its sample is skipped (zero padding in y).
// Pixels past the lattice have dZ = 0 in LDS.  The accumulators stay in
// registers across the group's tiles.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(const unsigned short* __restrict__ X,
                                                    const unsigned short* __restrict__ dZ,
                                                    float* __restrict__ partial,
                                                    float* __restrict__ bpart, int H, int W,
                                                    int rows) {
  constexpr int K = 9 * CIN, MT = COUT / 16, NTL = K / 16, KPW = (NTL + 3) / 4;
  constexpr int PS = CIN + 4, DS = COUT + 4;  // LDS pixel strides (BF16 values)
  constexpr int LC = kConvCols + 2, LR = kConvRows + 2, TP = kConvRows * kConvCols;
  constexpr int NG = 256 / COUT, GP = TP / NG;  // bias: pixel groups, pixels per group
  static_assert(CIN % 16 == 0 && COUT % 16 == 0 && 256 % COUT == 0, "channel counts");
  __shared__ __align__(16) unsigned short sx[LR * LC * PS];
  __shared__ __align__(16) unsigned short sdz[TP * DS];
  __shared__ float sb[256];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int tiles_x = (W + kConvCols - 1) / kConvCols;
  const int ntiles = tiles_x * ((rows + kConvRows - 1) / kConvRows);
  float4v acc[KPW][MT];
#pragma unroll
  for (int i = 0; i < KPW; ++i)
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[i][t] = float4v{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  const int bco = threadIdx.x % COUT, bgrp = threadIdx.x / COUT;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tiles_x) * kConvCols;
    const int R0 = (tile / tiles_x) * kConvRows;
    // input rows R0-1 .. R0+kConvRows, columns x0-1 .. x0+kConvCols, and dZ
    // of the tile's pixels (local pixel r * kConvCols + c)
    stage_rows<CIN, PS>(X, sx, R0, x0, W, rows);
    stage_matrix<TP, COUT, DS>(
        [&](int pix) {
          return dZ + ((long long)(R0 + pix / kConvCols) * W + x0 + pix % kConvCols) * COUT;
        },
        sdz, [&](int pix) { return R0 + pix / kConvCols < rows && x0 + pix % kConvCols < W; });
    __syncthreads();
#pragma unroll 4
    for (int p = bgrp * GP; p < (bgrp + 1) * GP; ++p) bacc += from_bf16(sdz[p * DS + bco]);
#pragma unroll 1
    for (int st = 0; st < TP / 16; ++st) {
      const int r = st / (kConvCols / 16), cb = (st % (kConvCols / 16)) * 16;
      if (R0 + r >= rows) break;  // uniform; later steps are past the batch too
      const int y = (R0 + r) % H;
      const unsigned short* dzp = sdz + (r * kConvCols + cb + 4 * g) * DS;
      short4v a[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) a[t][j] = (short)dzp[j * DS + t * 16 + m];
#pragma unroll
      for (int i = 0; i < KPW; ++i) {
        const int kt = wave + 4 * i;
        if (kt >= NTL) break;
        const int tap = kt * 16 / CIN, ci = kt * 16 % CIN + m;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        if (y + dy < 0 || y + dy >= H) continue;  // uniform
        const unsigned short* xp = sx + ((r + 1 + dy) * LC + cb + 4 * g + dx + 1) * PS + ci;
        short4v b;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (short)xp[j * PS];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[i][t] = mfma(a[t], b, acc[i][t]);
      }
    }
    __syncthreads();
  }
  // D[co row 4 g + j][k column m] of k tile wave + 4 i
  float* out = partial + (long long)blockIdx.x * COUT * K;
#pragma unroll
  for (int i = 0; i < KPW; ++i) {
    const int kt = wave + 4 * i;
    if (kt >= NTL) break;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) out[(t * 16 + 4 * g + j) * K + kt * 16 + m] = acc[i][t][j];
  }
  sb[threadIdx.x] = bacc;
  __syncthreads();
  if (threadIdx.x < COUT) {
    float v = 0.f;
    for (int k = 0; k < NG; ++k) v += sb[k * COUT + threadIdx.x];
    bpart[blockIdx.x * COUT + threadIdx.x] = v;
  }
}

// grad W[co][ci][ky][kx] = sum over parts of partial[part][co][tap * CIN + ci];
// grad b[co] = sum over parts of bpart[part][co].  A work-group takes 64
// consecutive partial columns (read coalesced); wave w of its kRedWaves
// sums the parts w, w + kRedWaves, ... in order and the wave sums are added
// in wave order.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(64 * kRedWaves) void wgrad_reduce(const float* __restrict__ partial,
                                                    const float* __restrict__ bpart, int nparts,
                                                    int cin, int cout, float* __restrict__ gradW,
                                                    float* __restrict__ gradb) {
  __shared__ float red[kRedWaves][64];
  const int K = 9 * cin, nW = cout * K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;  // partial column: co * K + tap * cin + ci
  float s = 0.f;
  if (col < nW) {
#pragma unroll 8
    for (int c = wave; c < nparts; c += kRedWaves) s += partial[(long long)c * nW + col];
  } else if (col < nW + cout) {
    for (int c = wave; c < nparts; c += kRedWaves) s += bpart[c * cout + (col - nW)];
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && col < nW + cout) {
    float v = red[0][lane];
#pragma unroll
    for (int w = 1; w < kRedWaves; ++w) v += red[w][lane];
    if (col < nW) {
      const int co = col / K, r = col % K, tap = r / cin, ci = r % cin;
      gradW[(co * cin + ci) * 9 + tap] = v;
    } else {
      gradb[col - nW] = v;
    }
  }
}

// FP32 planes [sample][c][y][x] (c < cin) -> X0[p][16] in BF16, scaled: one
// pixel per thread (coalesced plane reads, two 16-byte stores)
__global__ void pack_kernel(const float* __restrict__ planes, int cin, const float* __restrict__ scale,
                            long long hw, long long P, unsigned short* __restrict__ X0) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const long long s = p / hw, q = p % hw;
  unsigned short v[16];
#pragma unroll
  for (int c = 0; c < 16; ++c)
    v[c] = c < cin ? to_bf16(scale[c] * planes[(s * cin + c) * hw + q]) : (unsigned short)0;
  uint4* dst = (uint4*)(X0 + p * 16);
  dst[0] = __builtin_bit_cast(uint4, *(const unsigned short(*)[8])v);
  dst[1] = __builtin_bit_cast(uint4, *(const unsigned short(*)[8])(v + 8));
}

// out[sample][c][q] = scale_c * Z4[p][c], p = sample * hw + q, c < kOut
__global__ void output_kernel(const float* __restrict__ Z4, long long P, long long hw,
                              float scale0, float scale1, float* __restrict__ out) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const long long smp = p / hw, q = p % hw;
  out[(smp * kOut + 0) * hw + q] = scale0 * Z4[p * 16 + 0];
  out[(smp * kOut + 1) * hw + q] = scale1 * Z4[p * 16 + 1];
}

// Balance per sample: subtract half the sample's mean of out[c=0] +
// out[c=1] from both planes, so that the corrections of c1 and c2 add
// nothing to the sample's total scalar.  Two passes over kBalanceParts
// chunks of every sample (grid chunks x samples): FP64 chunk sums, then each
// chunk adds its sample's kBalanceParts sums in a fixed order (the same mean
// for every chunk) and subtracts.
constexpr int kBalanceParts = 64;

__global__ __launch_bounds__(256) void balance_sums(const float* __restrict__ out, long long hw,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  const float* o = out + (long long)blockIdx.y * kOut * hw;
  const long long q0 = hw * blockIdx.x / kBalanceParts, q1 = hw * (blockIdx.x + 1) / kBalanceParts;
  double s = 0.0;
  for (long long q = q0 + threadIdx.x; q < q1; q += 256) s += (double)o[q] + (double)o[hw + q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kBalanceParts + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void balance_apply(float* __restrict__ out, long long hw,
                                                     const double* __restrict__ part) {
  float* o = out + (long long)blockIdx.y * kOut * hw;
  double s = 0.0;
  for (int k = 0; k < kBalanceParts; ++k) s += part[blockIdx.y * kBalanceParts + k];
  const float m = (float)(s / (2.0 * (double)hw));
  const long long q0 = hw * blockIdx.x / kBalanceParts, q1 = hw * (blockIdx.x + 1) / kBalanceParts;
  for (long long q = q0 + threadIdx.x; q < q1; q += 256) {
    o[q] -= m;
    o[hw + q] -= m;
  }
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

// loss partials (FP64) and dZ4 = d(mean (z - t)^2) / dz4 in BF16, the mean
// over the kOut output channels of every pixel; target [sample][c][hw]
__global__ void loss_kernel(const float* __restrict__ Z4, const float* __restrict__ target,
                            long long P, long long hw, unsigned short* __restrict__ dZ4,
                            double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const float inv = 1.0f / (float)P;  // 2 / (kOut P)
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += stride) {
    const long long smp = p / hw, q = p % hw;
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
      const float r = Z4[p * 16 + c] - target[(smp * kOut + c) * hw + q];
      s += (double)r * (double)r;
      dZ4[p * 16 + c] = to_bf16(r * inv);
    }
#pragma unroll
    for (int c = kOut; c < 16; ++c) dZ4[p * 16 + c] = 0;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials(const double* __restrict__ partial, int n, long long count,
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
  if (threadIdx.x == 0) out[0] = red[0] / (double)count;
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

namespace {

// work-groups of conv_kernel<CI, CO, MO> the device holds at once (the
// persistent grid), from its compiled resource usage; cached per kernel
template <int CI, int CO, int MO>
long long conv_resident() {
  static std::atomic<long long> cache{0};
  long long n = cache.load(std::memory_order_relaxed);
  if (n > 0) return n;
  int per_cu = 0, cus = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(conv_kernel<CI, CO, MO>), 64 * kConvRowsF, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  n = (long long)per_cu * cus;
  cache.store(n, std::memory_order_relaxed);
  return n;
}

}  // namespace

hipError_t cnn_conv(int layer, int mode, const unsigned short* X, const unsigned short* Wg,
                    const float* bias, float* Z, unsigned short* A, const float* Zprev, int H,
                    int W, int rows, float scale0, float scale1, hipStream_t s) {
  const long long ntiles =
      (long long)((W + kConvCols - 1) / kConvCols) * ((rows + kConvRowsF - 1) / kConvRowsF);
  const dim3 blk(64 * kConvRowsF);
  // a persistent grid: at most the work-groups the device holds at once
#define PFLB_CONV(CI, CO, MO)                                                                     \
  hipLaunchKernelGGL((conv_kernel<CI, CO, MO>),                                                    \
                     dim3((unsigned)std::min(ntiles, conv_resident<CI, CO, MO>())), blk, 0, s, X, Wg, \
                     bias, Z, A, Zprev, H, W, rows, scale0, scale1)
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

int cnn_wgrad_parts(int W, long long rows) {
  const long long tiles =
      (long long)((W + kConvCols - 1) / kConvCols) * ((rows + kConvRows - 1) / kConvRows);
  const long long parts = (tiles + kWgradTiles - 1) / kWgradTiles;
  return (int)(parts < kWgradParts ? parts : kWgradParts);
}

hipError_t cnn_wgrad(int layer, const unsigned short* X, const unsigned short* dZ, float* partial,
                     float* bpart, int H, int W, int rows, float* gradW, float* gradb,
                     hipStream_t s) {
  const int cin = layer == 0 ? 16 : 32, cout = layer == 3 ? 16 : 32;
  const int nparts = cnn_wgrad_parts(W, rows);
  const dim3 grid(nparts), blk(256);
  switch (layer) {
    case 0: hipLaunchKernelGGL((wgrad_kernel<16, 32>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, rows); break;
    case 1: case 2: hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, rows); break;
    default: hipLaunchKernelGGL((wgrad_kernel<32, 16>), grid, blk, 0, s, X, dZ, partial, bpart, H, W, rows);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = cout * cin * 9 + cout;
  hipLaunchKernelGGL(wgrad_reduce, dim3((n + 63) / 64), dim3(64 * kRedWaves), 0, s, partial, bpart, nparts,
                     cin, cout, gradW, gradb);
  return hipGetLastError();
}

hipError_t cnn_pack(const float* planes, int cin, const float* scale, long long hw, long long P,
                    unsigned short* X0, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, planes,
                     cin, scale, hw, P, X0);
  return hipGetLastError();
}

hipError_t cnn_output(const float* Z4, long long P, long long hw, float scale0, float scale1,
                      float* out, hipStream_t s) {
  hipLaunchKernelGGL(output_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, Z4, P, hw,
                     scale0, scale1, out);
  return hipGetLastError();
}

int cnn_balance_parts(int nsamples) { return nsamples * kBalanceParts; }

hipError_t cnn_balance(float* out, int nsamples, long long hw, double* part, hipStream_t s) {
  hipLaunchKernelGGL(balance_sums, dim3(kBalanceParts, nsamples), dim3(256), 0, s, out, hw, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(balance_apply, dim3(kBalanceParts, nsamples), dim3(256), 0, s, out, hw, part);
  return hipGetLastError();
}

hipError_t cnn_restrict(const float* fine, int nsamples, int H, int W, int f, float* coarse,
                        hipStream_t s) {
  const long long n = (long long)nsamples * H * W;
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fine,
                     nsamples, H, W, f, coarse);
  return hipGetLastError();
}

hipError_t cnn_loss(const float* Z4, const float* target, long long P, long long hw,
                    unsigned short* dZ4, double* partial, int nparts, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(nparts), dim3(256), 0, s, Z4, target, P, hw, dZ4, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, partial, nparts, kOut * P, loss);
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
