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
#include "kernels.hpp"

namespace pflb {

namespace {

using L = D2Q9;
using Lay = Layout<D2Q9, D2Q9>;

// map a (possibly out of range) coordinate onto the node whose moments the
// stencil reads there: periodic wrap, or the mirror ghost at a wall
__device__ inline int fold(int v, int n, int wall) {
  if (v < 0) return wall ? 0 : v + n;
  if (v >= n) return wall ? n - 1 : v - n;
  return v;
}

// halo ring of a TX x TY tile: top row, bottom row, left column, right column
template <int TX, int TY>
__device__ inline void halo_pos(int k, int& hx, int& hy) {
  constexpr int LX = TX + 2;
  if (k < LX) {
    hx = k - 1;
    hy = -1;
  } else if (k < 2 * LX) {
    hx = k - LX - 1;
    hy = TY;
  } else if (k < 2 * LX + TY) {
    hx = -1;
    hy = k - 2 * LX;
  } else {
    hx = TX;
    hy = k - 2 * LX - TY;
  }
}

template <bool NTS, class S, class T>
__device__ inline void load_fh(const S* __restrict__ src, long long st, long long node, T (&f)[9],
                               T (&h1)[9], T (&h2)[9]) {
  load_set<L, NTS>(src, st, node, Lay::F0, f);
  load_set<L, NTS>(src, st, node, Lay::H10, h1);
  load_set<L, NTS>(src, st, node, Lay::H20, h2);
}

template <class S, class T, int TX, int TY, bool NTS, int MODE>
__global__ __launch_bounds__(TX* TY) void step2d_kernel(const S* __restrict__ src,
                                                        S* __restrict__ dst, T* __restrict__ hist,
                                                        T* __restrict__ fields, KParams<T> P,
                                                        int tiles_x, int ntiles) {
  constexpr int NT = TX * TY, LX = TX + 2, LY = TY + 2, NHALO = 2 * LX + 2 * TY;
  static_assert(NHALO <= NT, "one halo node per thread at most");
  __shared__ T sphi[LY][LX];
  __shared__ T spsi[LY][LX];

  // XCD-aware tile order: work-groups are dealt round-robin to the 8 XCDs
  // (group b runs on XCD b % 8), so XCD k gets the contiguous tile run
  // [k*per, (k+1)*per).  Groups past the last tile exit before any barrier.
  const int per = (ntiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int x0 = (tile % tiles_x) * TX;
  const int y0 = (tile / tiles_x) * TY;

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nx = P.nx, ny = P.ny;
  const long long st = P.stride;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  // a ragged tile: the slot one past the last node is read by that node's
  // stencil, so its thread fills it with the wrapped or mirrored node
  const bool own_slot = x <= nx && y <= ny;
  const long long node = (long long)y * nx + x;
  const long long own_src =
      active ? node : (long long)fold(y, ny, P.wall[1]) * nx + fold(x, nx, P.wall[0]);

  int hx = 0, hy = 0;
  bool halo = false;
  long long halo_src = 0;
  if (tid < NHALO) {
    halo_pos<TX, TY>(tid, hx, hy);
    const int gx = x0 + hx, gy = y0 + hy;
    halo = gx <= nx && gy <= ny;  // beyond a ragged tile no node reads it
    halo_src = (long long)fold(gy, ny, P.wall[1]) * nx + fold(gx, nx, P.wall[0]);
  }

  // ---- 1. all global loads first
  T f[9], h1[9], h2[9], g[9], hf[9], hh1[9], hh2[9];
  T hs[kHist2D];
  if (own_slot) load_fh<NTS>(src, st, own_src, f, h1, h2);
  if (active) {
    load_set<L, NTS>(src, st, node, Lay::G0, g);
#pragma unroll
    for (int k = 0; k < kHist2D; ++k) hs[k] = hist[k * st + node];
  }
  if (halo) load_fh<NTS>(src, st, halo_src, hf, hh1, hh2);

  // ---- 2. moments to LDS (deviations: the stencils only take differences
  //         and zero-sum weighted sums)
  Node<T> s{};
  if (own_slot) {
    moments<L>(P, f, h1, h2, s);
    sphi[ty + 1][tx + 1] = s.dphi;
    spsi[ty + 1][tx + 1] = s.dc1 + P.Keq * s.dc2;
  }
  if (halo) {
    Node<T> q;
    moments<L>(P, hf, hh1, hh2, q);
    sphi[hy + 1][hx + 1] = q.dphi;
    spsi[hy + 1][hx + 1] = q.dc1 + P.Keq * q.dc2;
  }
  __syncthreads();
  if (!active) return;

  // ---- 3. isotropic central stencils (Sec. III C) on D2Q9 weights
  T gphi[3] = {0, 0, 0}, gpsi[3] = {0, 0, 0}, lap = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const T a = sphi[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]];
    const T b = spsi[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]];
    const T wc = T(L::w[i] / L::cs2);
    gphi[0] += wc * T(L::cx[i]) * a;
    gphi[1] += wc * T(L::cy[i]) * a;
    gpsi[0] += wc * T(L::cx[i]) * b;
    gpsi[1] += wc * T(L::cy[i]) * b;
    lap += T(2) * wc * (a - s.dphi);
  }

  Flow<T> fl;
  flow_macros<L>(P, g, s, gphi, lap, fl);

  if (MODE == kModeMacros) {
    fields[kFieldPhi * st + node] = s.phi;
    fields[kFieldP * st + node] = fl.p;
    fields[kFieldUx * st + node] = fl.u[0];
    fields[kFieldUy * st + node] = fl.u[1];
    fields[kFieldUz * st + node] = T(0);
    fields[kFieldC1 * st + node] = s.c1;
    fields[kFieldC2 * st + node] = s.c2;
    fields[kFieldMu * st + node] = fl.mu;
    fields[kFieldPsi * st + node] = s.c1 + P.Keq * s.c2;
    return;
  }

  // backward-difference time derivatives against the history (R1)
  const T dJphi[3] = {s.phi * fl.u[0] - hs[2] * hs[0], s.phi * fl.u[1] - hs[2] * hs[1], T(0)};
  const T dJ1[3] = {s.c1 * fl.u[0] - hs[3] * hs[0], s.c1 * fl.u[1] - hs[3] * hs[1], T(0)};
  const T dJ2[3] = {s.c2 * fl.u[0] - hs[4] * hs[0], s.c2 * fl.u[1] - hs[4] * hs[1], T(0)};
  hist[0 * st + node] = fl.u[0];
  hist[1 * st + node] = fl.u[1];
  hist[2 * st + node] = s.phi;
  hist[3 * st + node] = s.c1;
  hist[4 * st + node] = s.c2;

  // push streaming: X_i(x + c_i) <- X_i*(x), or half-way bounce-back into
  // the opposite slot of the own node when the link crosses a wall; each
  // post-collision value is stored as soon as it is formed
  auto dest = [&](int i, int& j) -> long long {
    int xt = x + L::cx[i], yt = y + L::cy[i];
    bool bounce = false;
    if (xt < 0 || xt >= nx) {
      if (P.wall[0]) bounce = true;
      else xt = xt < 0 ? xt + nx : xt - nx;
    }
    if (yt < 0 || yt >= ny) {
      if (P.wall[1]) bounce = true;
      else yt = yt < 0 ? yt + ny : yt - ny;
    }
    j = bounce ? L::opp[i] : i;
    return bounce ? node : (long long)yt * nx + xt;
  };
  collide<L, L>(
      P, f, g, h1, h2, s, gphi, gpsi, fl, dJphi, dJ1, dJ2,
      [&](int i, T v) {
        int j;
        const long long t = dest(i, j);
        store_one<L, NTS>(dst, (Lay::F0 + j) * st + t, i, v);
      },
      [&](int i, T v) {
        int j;
        const long long t = dest(i, j);
        store_one<L, NTS>(dst, (Lay::G0 + j) * st + t, i, v);
      },
      [&](int i, T a, T b) {
        int j;
        const long long t = dest(i, j);
        store_one<L, NTS>(dst, (Lay::H10 + j) * st + t, i, a);
        store_one<L, NTS>(dst, (Lay::H20 + j) * st + t, i, b);
      });
}

template <class S, class T, int TX, int TY, bool NTS, int MODE>
hipError_t launch_variant(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P,
                          hipStream_t stream) {
  const int tiles_x = (P.nx + TX - 1) / TX;
  const int tiles_y = (P.ny + TY - 1) / TY;
  const int ntiles = tiles_x * tiles_y;
  const int nblocks = ((ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL((step2d_kernel<S, T, TX, TY, NTS, MODE>), dim3(nblocks), dim3(TX * TY), 0,
                     stream, src, dst, hist, fields, P, tiles_x, ntiles);
  return hipGetLastError();
}

}  // namespace

// variant table: tile TX x TY and non-temporal population traffic
const char* step2d_variant_name(int v) {
  static const char* names[kVariants2D] = {"64x4",    "32x8",    "32x4",    "128x4",
                                          "64x4 nt", "32x8 nt", "32x4 nt", "128x4 nt"};
  return v >= 0 && v < kVariants2D ? names[v] : "?";
}

template <class S, class T>
hipError_t launch_step2d(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P, int mode,
                         int variant, hipStream_t stream) {
  if (mode == kModeMacros)
    return launch_variant<S, T, 64, 4, false, kModeMacros>(src, dst, hist, fields, P, stream);
  switch (variant) {
    case 1: return launch_variant<S, T, 32, 8, false, kModeStep>(src, dst, hist, fields, P, stream);
    case 2: return launch_variant<S, T, 32, 4, false, kModeStep>(src, dst, hist, fields, P, stream);
    case 3: return launch_variant<S, T, 128, 4, false, kModeStep>(src, dst, hist, fields, P, stream);
    case 4: return launch_variant<S, T, 64, 4, true, kModeStep>(src, dst, hist, fields, P, stream);
    case 5: return launch_variant<S, T, 32, 8, true, kModeStep>(src, dst, hist, fields, P, stream);
    case 6: return launch_variant<S, T, 32, 4, true, kModeStep>(src, dst, hist, fields, P, stream);
    case 7: return launch_variant<S, T, 128, 4, true, kModeStep>(src, dst, hist, fields, P, stream);
    default: return launch_variant<S, T, 64, 4, false, kModeStep>(src, dst, hist, fields, P, stream);
  }
}

template hipError_t launch_step2d<double, double>(const double*, double*, double*, double*,
                                                  const KParams<double>&, int, int, hipStream_t);
template hipError_t launch_step2d<float, float>(const float*, float*, float*, float*,
                                                const KParams<float>&, int, int, hipStream_t);
template hipError_t launch_step2d<__half, float>(const __half*, __half*, float*, float*,
                                                 const KParams<float>&, int, int, hipStream_t);
template hipError_t launch_step2d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         float*, float*, const KParams<float>&, int,
                                                         int, hipStream_t);

}  // namespace pflb
