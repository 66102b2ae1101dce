// 2-D fused step on D2Q9 (f, g, h1, h2 all D2Q9).
//
// One launch = one time step.  A work-group owns a TX x TY tile of nodes, one
// node per thread:
//   1. every global load the thread needs is issued first: f, h1, h2 of its
//      node (27 values, coalesced along x), its g populations and history,
//      and f, h1, h2 of at most one node of the halo ring around the tile
//      (re-read from L2: the neighbouring tile ran on the same XCD);
//   2. the deviations of phi and psi = c1 + Keq c2 of the tile and its halo
//      go to LDS;
//   3. after one barrier each thread takes the 9-point gradient / Laplacian
//      stencils from LDS, collides all four sets and pushes the
//      post-collision values to x + c_i of the other lattice (periodic wrap
//      or half-way bounce-back).
// Work-group ids are remapped so that the tiles one XCD runs form a
// contiguous band of rows: halo rows are then shared through that XCD's L2.
//
// Variants (tile shape, non-temporal population traffic) are template
// parameters; the host picks one per lattice (cplb_tune times them all).
#include "step2d_tile.hpp"

namespace pflb {

namespace {

using L = D2Q9;
using Lay = Layout<D2Q9, D2Q9>;

// The lattice constants are read through a constant-address-space pointer
// (scalar loads of the device copy) rather than passed by value: the kernel
// arguments stay a few dozen bytes.
template <class S, class T, int TX, int TY, int NTM, int MODE, class Off, int MODEL>
__global__ __launch_bounds__(TX* TY) void step2d_kernel(const S* __restrict__ src,
                                                        S* __restrict__ dst,
                                                        const T* __restrict__ hin,
                                                        T* __restrict__ hout,
                                                        T* __restrict__ fields, KPtr<T> Pg,
                                                        Geo2<Off> G) {
  // XCD-aware tile order: work-groups are dealt round-robin to the 8 XCDs
  // (group b runs on XCD b % 8), so XCD k gets the contiguous tile run
  // [k*per, (k+1)*per) and tiles that share halo rows share an L2.  Groups
  // past the last tile exit before any barrier.
  const int per = (G.ntiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= G.ntiles) return;
  step2d_tile<S, T, TX, TY, NTM, MODE, Off, MODEL>(src, dst, hin, hout, fields, params(Pg), G,
                                                   tile);
}

template <class S, class T, int TX, int TY, int NTM, int MODE, class Off, int MODEL>
hipError_t launch_variant(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                          const KParams<T>* Pdev, const float* closure, hipStream_t stream) {
  Geo2<Off> G;
  G.nx = P.nx;
  G.ny = P.ny;
  G.px = P.px;
  G.wall_x = P.wall[0];
  G.wall_y = P.wall[1];
  G.tiles_x = (P.nx + TX - 1) / TX;
  G.ntiles = G.tiles_x * ((P.ny + TY - 1) / TY);
  G.sS = Off(P.stride * (long long)sizeof(S));
  G.sT = Off(P.stride * (long long)sizeof(T));
  G.closure = closure;
  const int nblocks = ((G.ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL((step2d_kernel<S, T, TX, TY, NTM, MODE, Off, MODEL>), dim3(nblocks), dim3(TX * TY),
                     0, stream, src, dst, hin, hout, fields, (KPtr<T>)Pdev, G);
  return hipGetLastError();
}

}  // namespace

// variant table: tile TX x TY and non-temporal population traffic
const char* step2d_variant_name(int v) {
  static const char* names[kVariants2D] = {"64x4",    "32x8",    "32x4",    "128x4",
                                          "64x4 nt", "32x8 nt", "32x4 nt", "128x4 nt",
                                          "128x4 nt-st", "128x4 nt-own", "256x4", "256x4 nt-st"};
  return v >= 0 && v < kVariants2D ? names[v] : "?";
}

namespace {

// the variant switch of one scalar-model variant (kModel*)
template <class S, class T, int MODEL>
hipError_t launch_model(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                        const KParams<T>* Pdev, int mode, int variant, const float* closure,
                        hipStream_t stream) {
  constexpr int M = kModeStep;
  using U = uint32_t;
  if (!fits_u32(L::Q, P.stride, sizeof(S), sizeof(T), kNumFields)) {
    // very large grids: 64-bit offsets, one tile shape
    if (mode == kModeMacros)
      return launch_variant<S, T, 64, 4, 0, kModeMacros, uint64_t, MODEL>(src, dst, hin, hout, fields,
                                                                           P, Pdev, closure, stream);
    return launch_variant<S, T, 128, 4, 0, M, uint64_t, MODEL>(src, dst, hin, hout, fields, P,
                                                                Pdev, closure, stream);
  }
  if (mode == kModeMacros)
    return launch_variant<S, T, 64, 4, 0, kModeMacros, U, MODEL>(src, dst, hin, hout, fields, P,
                                                                  Pdev, closure, stream);
  switch (variant) {
    case 1: return launch_variant<S, T, 32, 8, 0, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 2: return launch_variant<S, T, 32, 4, 0, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 3: return launch_variant<S, T, 128, 4, 0, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 4: return launch_variant<S, T, 64, 4, 7, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 5: return launch_variant<S, T, 32, 8, 7, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 6: return launch_variant<S, T, 32, 4, 7, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 7: return launch_variant<S, T, 128, 4, 7, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 8: return launch_variant<S, T, 128, 4, 2, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 9: return launch_variant<S, T, 128, 4, 3, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 10: return launch_variant<S, T, 256, 4, 0, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    case 11: return launch_variant<S, T, 256, 4, 2, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
    default: return launch_variant<S, T, 64, 4, 0, M, U, MODEL>(src, dst, hin, hout, fields, P, Pdev, closure, stream);
  }
}

}  // namespace

template <class S, class T>
hipError_t launch_step2d(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                         const KParams<T>* Pdev, int mode, int variant, const float* closure,
                         hipStream_t stream) {
  if (P.one_scalar)
    return launch_model<S, T, kModelOne>(src, dst, hin, hout, fields, P, Pdev, mode, variant, nullptr,
                                         stream);
  if (P.local_grad)
    return launch_model<S, T, kModelTwoLocal>(src, dst, hin, hout, fields, P, Pdev, mode, variant,
                                              closure, stream);
  if (P.dirichlet)
    return launch_model<S, T, kModelTwoDirichlet>(src, dst, hin, hout, fields, P, Pdev, mode, variant,
                                                  closure, stream);
  return launch_model<S, T, kModelTwo>(src, dst, hin, hout, fields, P, Pdev, mode, variant, closure,
                                       stream);
}

template hipError_t launch_step2d<double, double>(const double*, double*, const double*, double*, double*,
                                                  const KParams<double>&, const KParams<double>*,
                                                  int, int, const float*, hipStream_t);
template hipError_t launch_step2d<float, float>(const float*, float*, const float*, float*, float*,
                                                const KParams<float>&, const KParams<float>*,
                                                int, int, const float*, hipStream_t);
template hipError_t launch_step2d<__half, float>(const __half*, __half*, const float*, float*, float*,
                                                 const KParams<float>&, const KParams<float>*,
                                                int, int, const float*, hipStream_t);
template hipError_t launch_step2d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         const float*, float*, float*,
                                                         const KParams<float>&,
                                                         const KParams<float>*, int, int,
                                                         const float*, hipStream_t);

}  // namespace pflb
