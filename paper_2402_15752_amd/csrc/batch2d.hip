// Batched 2-D step: many independent D2Q9 lattices of different sizes and
// parameters advanced by one launch per size class.
//
// The work list of a launch is the concatenation of the tile lists of the
// class's cases.  A work-group takes global tile g (dealt XCD-aware, as in
// the single-lattice kernel), finds its case by a binary search over the
// class's tile prefix (scalar loads: every lane of the group agrees), reads
// that case's geometry and lattice constants from device tables, and runs
// the same tile body as the single-lattice kernel -- so each case of a
// batch is bit-identical to the same case run alone.
#include "step2d_tile.hpp"

namespace pflb {

namespace {

template <class X>
using CPtr = const __attribute__((address_space(4))) X*;

template <class S, class T, int TX, int TY, int NTM, int MODE>
__global__ __launch_bounds__(TX* TY) void batch2d_kernel(CPtr<BatchCase> cases, CPtr<int> ids,
                                                         CPtr<int> prefix, int ncls,
                                                         CPtr<int> map, int total, KPtr<T> kps,
                                                         int parity) {
  const int per = (total + 7) / 8;
  const int g = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (g >= total) return;
  int c, tile;
  if (map) {
    // (case, tile of the case): one pair of scalar loads
    c = map[2 * g];
    tile = map[2 * g + 1];
  } else {
    // last k with prefix[k] <= g
    int lo = 0, hi = ncls;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (prefix[mid] <= g) lo = mid;
      else hi = mid;
    }
    c = ids[lo];
    tile = g - prefix[lo];
  }
  CPtr<BatchCase> D = cases + c;
  Geo2<uint32_t> G;
  G.nx = D->nx;
  G.ny = D->ny;
  G.px = D->px;
  G.wall_x = D->wall_x;
  G.wall_y = D->wall_y;
  G.tiles_x = (G.nx + TX - 1) / TX;
  G.ntiles = G.tiles_x * ((G.ny + TY - 1) / TY);
  G.sS = D->sS;
  G.sT = D->sT;
  G.closure = D->closure;
  const S* src = (const S*)D->lat[parity];
  S* dst = (S*)D->lat[parity ^ 1];
  const KParams<T>& P = *(const KParams<T>*)(kps + c);
  step2d_tile<S, T, TX, TY, NTM, MODE, uint32_t>(src, dst, (const T*)D->hist[parity],
                                                 (T*)D->hist[parity ^ 1], (T*)D->fields, P, G,
                                                 tile);
}

template <class S, class T, int TX, int TY, int NTM, int MODE>
hipError_t launch_b(const BatchCase* cases, const int* ids, const int* prefix, int ncls,
                    const int* map, int total, const KParams<T>* kps, int parity,
                    hipStream_t stream) {
  const int nblocks = ((total + 7) / 8) * 8;
  hipLaunchKernelGGL((batch2d_kernel<S, T, TX, TY, NTM, MODE>), dim3(nblocks), dim3(TX * TY), 0,
                     stream, (CPtr<BatchCase>)cases, (CPtr<int>)ids, (CPtr<int>)prefix, ncls,
                     (CPtr<int>)map, total, (KPtr<T>)kps, parity);
  return hipGetLastError();
}

}  // namespace

// tile shapes of the 2-D variants (the same table as the single-lattice step)
int step2d_tiles(int nx, int ny, int variant) {
  static const int tx[kVariants2D] = {64, 32, 32, 128, 64, 32, 32, 128, 128, 128, 256, 256};
  static const int ty[kVariants2D] = {4, 8, 4, 4, 4, 8, 4, 4, 4, 4, 4, 4};
  if (variant < 0 || variant >= kVariants2D) variant = 0;
  return ((nx + tx[variant] - 1) / tx[variant]) * ((ny + ty[variant] - 1) / ty[variant]);
}

template <class S, class T>
hipError_t launch_batch2d(const BatchCase* cases, const int* ids, const int* prefix, int ncls,
                          const int* map, int total, const KParams<T>* kps, int parity, int mode,
                          int variant, hipStream_t stream) {
  if (total <= 0) return hipSuccess;
  constexpr int M = kModeStep;
  if (mode == kModeMacros)
    return launch_b<S, T, 64, 4, 0, kModeMacros>(cases, ids, prefix, ncls, map, total, kps,
                                                     parity, stream);
  switch (variant) {
    case 1: return launch_b<S, T, 32, 8, 0, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 2: return launch_b<S, T, 32, 4, 0, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 3: return launch_b<S, T, 128, 4, 0, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 4: return launch_b<S, T, 64, 4, 7, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 5: return launch_b<S, T, 32, 8, 7, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 6: return launch_b<S, T, 32, 4, 7, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 7: return launch_b<S, T, 128, 4, 7, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 8: return launch_b<S, T, 128, 4, 2, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 9: return launch_b<S, T, 128, 4, 3, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 10: return launch_b<S, T, 256, 4, 0, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    case 11: return launch_b<S, T, 256, 4, 2, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
    default: return launch_b<S, T, 64, 4, 0, M>(cases, ids, prefix, ncls, map, total, kps, parity, stream);
  }
}

namespace {

struct GatherIds {
  int id[9];
};

template <class T>
__global__ void gather_kernel(CPtr<BatchCase> cases, GatherIds ids, int nplanes,
                              float* __restrict__ dst) {
  const int c = blockIdx.y, f = blockIdx.z;
  CPtr<BatchCase> D = cases + c;
  const long long n = (long long)D->nx * D->ny;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T* src = (const T*)((const char*)D->fields + (size_t)ids.id[f] * D->sT);
  dst[D->out_off * nplanes + f * n + i] = (float)src[pitched(i, D->nx, D->px)];
}

// Fields that need only the node's own moments (phi, c1, c2, psi): f, h1,
// h2 of each node, the recovery of Sec. III C, straight into the gathered
// planes -- no stencils, no flow macros, no field buffer.  The values are
// those the macros mode writes (the same moments() arithmetic).
template <class S, class T>
__global__ void gather_moments_kernel(CPtr<BatchCase> cases, KPtr<T> kps, int parity,
                                      GatherIds ids, int nf, int nplanes,
                                      float* __restrict__ dst) {
  using L = D2Q9;
  using Lay = Layout<D2Q9, D2Q9>;
  const int c = blockIdx.y;
  CPtr<BatchCase> D = cases + c;
  const int n = D->nx * D->ny;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const KParams<T>& P = *(const KParams<T>*)(kps + c);
  const S* lat = (const S*)D->lat[parity];
  const uint32_t sS = D->sS;
  const uint32_t node = uint32_t(pitched(i, D->nx, D->px)) * uint32_t(sizeof(S));
  T f[9], h1[9], h2[9];
  load_q<L, false, false>(at(lat, uint32_t(Lay::F0) * sS), sS, node, f);
  load_q<L, false, false>(at(lat, uint32_t(Lay::H10) * sS), sS, node, h1);
  load_q<L, false, false>(at(lat, uint32_t(Lay::H20) * sS), sS, node, h2);
  // references of the stored populations: the history planes phi, c1, c2
  const T* hist = (const T*)D->hist[parity];
  const uint32_t nodeT = node * uint32_t(sizeof(T) / sizeof(S));
  const T rphi = *at(hist, 2u * D->sT + nodeT);
  const T rc1 = *at(hist, 3u * D->sT + nodeT);
  const T rc2 = *at(hist, 4u * D->sT + nodeT);
  Node<T> s{};
  moments<L>(P, f, h1, h2, rphi, rc1, rc2, s);
  float* out = dst + D->out_off * nplanes + i;
  for (int k = 0; k < nf; ++k) {
    const int id = ids.id[k];
    const T v = id == kFieldPhi ? s.phi : id == kFieldC1 ? s.c1 : id == kFieldC2 ? s.c2
                                                                                 : s.c1 + P.Keq * s.c2;
    out[(long long)k * n] = (float)v;
  }
}

}  // namespace

template <class S, class T>
hipError_t launch_batch_gather_moments(const BatchCase* cases, const KParams<T>* kps, int parity,
                                       int ncases, long long max_n, const int (&ids)[9], int nf,
                                       int nplanes, float* dst, hipStream_t stream) {
  GatherIds g;
  for (int k = 0; k < 9; ++k) g.id[k] = ids[k];
  const dim3 grid((unsigned)((max_n + 255) / 256), ncases);
  hipLaunchKernelGGL((gather_moments_kernel<S, T>), grid, dim3(256), 0, stream,
                     (CPtr<BatchCase>)cases, (KPtr<T>)kps, parity, g, nf, nplanes, dst);
  return hipGetLastError();
}

#define PFLB_GM_INST(S, T)                                                                      \
  template hipError_t launch_batch_gather_moments<S, T>(const BatchCase*, const KParams<T>*, int, \
                                                        int, long long, const int (&)[9], int,  \
                                                        int, float*, hipStream_t);
PFLB_GM_INST(double, double)
PFLB_GM_INST(float, float)
PFLB_GM_INST(__half, float)
PFLB_GM_INST(__hip_bfloat16, float)
#undef PFLB_GM_INST

template <class T>
hipError_t launch_batch_gather(const BatchCase* cases, int ncases, long long max_n,
                               const int (&ids)[9], int nf, int nplanes, float* dst,
                               hipStream_t stream) {
  GatherIds g;
  for (int k = 0; k < 9; ++k) g.id[k] = ids[k];
  const dim3 grid((unsigned)((max_n + 255) / 256), ncases, nf);
  hipLaunchKernelGGL(gather_kernel<T>, grid, dim3(256), 0, stream, (CPtr<BatchCase>)cases, g, nplanes, dst);
  return hipGetLastError();
}

template hipError_t launch_batch_gather<double>(const BatchCase*, int, long long, const int (&)[9],
                                                int, int, float*, hipStream_t);
template hipError_t launch_batch_gather<float>(const BatchCase*, int, long long, const int (&)[9],
                                               int, int, float*, hipStream_t);

#define PFLB_BATCH_INST(S, T)                                                                    \
  template hipError_t launch_batch2d<S, T>(const BatchCase*, const int*, const int*, int,        \
                                           const int*, int, const KParams<T>*, int, int, int,      \
                                           hipStream_t);
PFLB_BATCH_INST(double, double)
PFLB_BATCH_INST(float, float)
PFLB_BATCH_INST(__half, float)
PFLB_BATCH_INST(__hip_bfloat16, float)
#undef PFLB_BATCH_INST

}  // namespace pflb
