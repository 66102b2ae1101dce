// 2-D fused step on D2Q9 (f, g, h1, h2 all D2Q9).
//
// One launch = one time step.  A work-group owns a TX x TY tile of nodes, one
// node per thread:
//   1. each thread loads f, h1, h2 of its node (27 values, coalesced along x),
//      forms phi, c1, c2, psi and puts the deviations of phi, psi in LDS;
//   2. the ring of halo nodes around the tile is filled the same way (its
//      populations are re-read, mostly from L2: no extra HBM traffic when the
//      neighbouring tile ran on the same XCD);
//   3. after one barrier each thread takes the 9-point gradient / Laplacian
//      stencils from LDS, loads its g populations and history, collides all
//      four sets and pushes the post-collision values to x + c_i of the other
//      lattice (periodic wrap or half-way bounce-back).
// Work-group ids are remapped so that the tiles one XCD runs form a
// contiguous band of rows: halo rows are then shared through that XCD's L2.
#include "kernels.hpp"

namespace pflb {

namespace {

constexpr int TX = 64;
constexpr int TY = 4;
constexpr int NT = TX * TY;
constexpr int LX = TX + 2;
constexpr int LY = TY + 2;
constexpr int NHALO = 2 * LX + 2 * TY;

using L = D2Q9;
using Lay = Layout<D2Q9, D2Q9>;

// map a (possibly out of range) coordinate onto the node whose moments the
// stencil reads there: periodic wrap, or the mirror ghost at a wall
__device__ inline int fold(int v, int n, int wall) {
  if (v < 0) return wall ? 0 : v + n;
  if (v >= n) return wall ? n - 1 : v - n;
  return v;
}

template <class S, class T>
__device__ inline void node_moments(const S* __restrict__ src, const KParams<T>& P, long long node,
                                    T (&f)[9], T (&h1)[9], T (&h2)[9], Node<T>& s) {
  load_set<L>(src, P.stride, node, Lay::F0, f);
  load_set<L>(src, P.stride, node, Lay::H10, h1);
  load_set<L>(src, P.stride, node, Lay::H20, h2);
  moments<L>(P, f, h1, h2, s);
}

template <class S, class T, int MODE>
__global__ __launch_bounds__(NT) void step2d_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                    T* __restrict__ hist, T* __restrict__ fields,
                                                    KParams<T> P, int tiles_x, int ntiles) {
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
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  const long long node = (long long)y * nx + x;

  // LDS holds the deviations dphi and dpsi = dc1 + Keq dc2: the stencils
  // only ever take differences and weighted sums with zero total weight
  T f[9], h1[9], h2[9];
  Node<T> s{};
  if (active) {
    node_moments(src, P, node, f, h1, h2, s);
    sphi[ty + 1][tx + 1] = s.dphi;
    spsi[ty + 1][tx + 1] = s.dc1 + P.Keq * s.dc2;
  } else if (x <= nx && y <= ny) {
    // a ragged tile: the slot one past the last node is read by the stencil
    // of that node; fill it with the wrapped or mirrored node's moments
    const int sx = fold(x, nx, P.wall[0]), sy = fold(y, ny, P.wall[1]);
    T hf[9], hh1[9], hh2[9];
    Node<T> hs;
    node_moments(src, P, (long long)sy * nx + sx, hf, hh1, hh2, hs);
    sphi[ty + 1][tx + 1] = hs.dphi;
    spsi[ty + 1][tx + 1] = hs.dc1 + P.Keq * hs.dc2;
  }
  // halo ring: top row, bottom row, left column, right column
  for (int k = tid; k < NHALO; k += NT) {
    int hx, hy;
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
    const int gx = x0 + hx, gy = y0 + hy;
    if (gx > nx || gy > ny) continue;  // beyond a ragged tile: read by no node
    const int sx = fold(gx, nx, P.wall[0]);
    const int sy = fold(gy, ny, P.wall[1]);
    T hf[9], hh1[9], hh2[9];
    Node<T> hs;
    node_moments(src, P, (long long)sy * nx + sx, hf, hh1, hh2, hs);
    sphi[hy + 1][hx + 1] = hs.dphi;
    spsi[hy + 1][hx + 1] = hs.dc1 + P.Keq * hs.dc2;
  }
  __syncthreads();
  if (!active) return;

  // isotropic central stencils (Sec. III C) on D2Q9 weights
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

  T g[9];
  load_set<L>(src, P.stride, node, Lay::G0, g);
  Flow<T> fl;
  flow_macros<L>(P, g, s, gphi, lap, fl);

  if (MODE == kModeMacros) {
    const long long st = P.stride;
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
  const long long st = P.stride;
  const T uo0 = hist[0 * st + node], uo1 = hist[1 * st + node];
  const T phio = hist[2 * st + node], c1o = hist[3 * st + node], c2o = hist[4 * st + node];
  const T dJphi[3] = {s.phi * fl.u[0] - phio * uo0, s.phi * fl.u[1] - phio * uo1, T(0)};
  const T dJ1[3] = {s.c1 * fl.u[0] - c1o * uo0, s.c1 * fl.u[1] - c1o * uo1, T(0)};
  const T dJ2[3] = {s.c2 * fl.u[0] - c2o * uo0, s.c2 * fl.u[1] - c2o * uo1, T(0)};
  hist[0 * st + node] = fl.u[0];
  hist[1 * st + node] = fl.u[1];
  hist[2 * st + node] = s.phi;
  hist[3 * st + node] = s.c1;
  hist[4 * st + node] = s.c2;

  collide<L, L>(P, f, g, h1, h2, s, gphi, gpsi, fl, dJphi, dJ1, dJ2);

  // push streaming: X_i(x + c_i) <- X_i*(x); half-way bounce-back at walls
#pragma unroll
  for (int i = 0; i < 9; ++i) {
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
    const int j = bounce ? L::opp[i] : i;
    const long long t = bounce ? node : (long long)yt * nx + xt;
    store_one<L>(dst, (Lay::F0 + j) * st + t, i, f[i]);
    store_one<L>(dst, (Lay::G0 + j) * st + t, i, g[i]);
    store_one<L>(dst, (Lay::H10 + j) * st + t, i, h1[i]);
    store_one<L>(dst, (Lay::H20 + j) * st + t, i, h2[i]);
  }
}

}  // namespace

template <class S, class T>
hipError_t launch_step2d(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P, int mode,
                         hipStream_t stream) {
  const int tiles_x = (P.nx + TX - 1) / TX;
  const int tiles_y = (P.ny + TY - 1) / TY;
  const int ntiles = tiles_x * tiles_y;
  const int nblocks = ((ntiles + 7) / 8) * 8;
  if (mode == kModeMacros)
    hipLaunchKernelGGL((step2d_kernel<S, T, kModeMacros>), dim3(nblocks), dim3(NT), 0, stream, src,
                       dst, hist, fields, P, tiles_x, ntiles);
  else
    hipLaunchKernelGGL((step2d_kernel<S, T, kModeStep>), dim3(nblocks), dim3(NT), 0, stream, src,
                       dst, hist, fields, P, tiles_x, ntiles);
  return hipGetLastError();
}

template hipError_t launch_step2d<double, double>(const double*, double*, double*, double*,
                                                  const KParams<double>&, int, hipStream_t);
template hipError_t launch_step2d<float, float>(const float*, float*, float*, float*,
                                                const KParams<float>&, int, hipStream_t);
template hipError_t launch_step2d<__half, float>(const __half*, __half*, float*, float*,
                                                 const KParams<float>&, int, hipStream_t);
template hipError_t launch_step2d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         float*, float*, const KParams<float>&, int,
                                                         hipStream_t);

}  // namespace pflb
