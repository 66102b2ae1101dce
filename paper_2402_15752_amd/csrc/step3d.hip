// 3-D fused step: D3Q19 for the flow set g and for the 19-point stencils,
// D3Q7 for f, h1, h2.
//
// One launch = one time step.  A work-group owns a TX x TY column tile and
// marches along z over a chunk of LZ planes.  LDS holds a ring of three
// planes of phi and psi = c1 + Keq c2 over the tile and its one-node halo.
// Per plane z the group
//   1. fills plane z+1 of the ring: each thread loads f, h1, h2 (21 values)
//      of its own column at z+1 and keeps them in registers for the next
//      iteration, and the halo ring of that plane is computed from re-read
//      populations (L2 hits: neighbouring tiles march the same planes);
//   2. collides plane z: 19-point stencils from the three ring planes, own
//      g (19 values) and history loaded, all four sets collided and pushed to
//      x + c_i of the other lattice (periodic wrap or half-way bounce-back).
// Interior moments are computed once per node; only the halo ring and the
// first two planes of a chunk are recomputed.
#include "kernels.hpp"

namespace pflb {

namespace {

constexpr int TX = 32;
constexpr int TY = 8;
constexpr int NT = TX * TY;
constexpr int LX = TX + 2;
constexpr int LY = TY + 2;
constexpr int NHALO = 2 * LX + 2 * TY;
constexpr int LZ = 64;

using LF = D3Q7;
using LG = D3Q19;
using Lay = Layout<D3Q7, D3Q19>;

__device__ inline int fold(int v, int n, int wall) {
  if (v < 0) return wall ? 0 : v + n;
  if (v >= n) return wall ? n - 1 : v - n;
  return v;
}

template <class S, class T>
__device__ inline void node_moments(const S* __restrict__ src, const KParams<T>& P, long long node,
                                    T (&f)[7], T (&h1)[7], T (&h2)[7], Node<T>& s) {
  load_set<LF>(src, P.stride, node, Lay::F0, f);
  load_set<LF>(src, P.stride, node, Lay::H10, h1);
  load_set<LF>(src, P.stride, node, Lay::H20, h2);
  moments<LF>(P, f, h1, h2, s);
}

template <class T>
struct Ring {
  T phi[3][LY][LX];
  T psi[3][LY][LX];
};

// Fill ring slot `slot` with plane zp (folded onto the domain for the
// stencils): the deviations dphi and dpsi = dc1 + Keq dc2.  Own-column
// populations of that plane are returned in f, h1, h2 with their moments
// when the own node exists.
template <class S, class T>
__device__ inline void fill_plane(const S* __restrict__ src, const KParams<T>& P, Ring<T>& R,
                                  int slot, int zp, int x0, int y0, int tx, int ty, T (&f)[7],
                                  T (&h1)[7], T (&h2)[7], Node<T>& s) {
  const int nx = P.nx, ny = P.ny;
  const int gz = fold(zp, P.nz, P.wall[2]);
  const long long plane = (long long)gz * nx * ny;
  const int x = x0 + tx, y = y0 + ty;
  if (x <= nx && y <= ny) {
    const int sx = fold(x, nx, P.wall[0]), sy = fold(y, ny, P.wall[1]);
    node_moments(src, P, plane + (long long)sy * nx + sx, f, h1, h2, s);
    R.phi[slot][ty + 1][tx + 1] = s.dphi;
    R.psi[slot][ty + 1][tx + 1] = s.dc1 + P.Keq * s.dc2;
  }
  const int tid = tx + TX * ty;
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
    if (gx > nx || gy > ny) continue;
    const int sx = fold(gx, nx, P.wall[0]), sy = fold(gy, ny, P.wall[1]);
    T hf[7], hh1[7], hh2[7];
    Node<T> hs;
    node_moments(src, P, plane + (long long)sy * nx + sx, hf, hh1, hh2, hs);
    R.phi[slot][hy + 1][hx + 1] = hs.dphi;
    R.psi[slot][hy + 1][hx + 1] = hs.dc1 + P.Keq * hs.dc2;
  }
}

__device__ inline int slot_of(int z) { return (z + 3) % 3; }

template <class S, class T, int MODE>
__global__ __launch_bounds__(NT) void step3d_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                    T* __restrict__ hist, T* __restrict__ fields,
                                                    KParams<T> P, int tiles_x, int tiles_xy,
                                                    int ntiles) {
  __shared__ Ring<T> R;
  // XCD-aware order (see the 2-D kernel): XCD k runs a contiguous tile range
  const int per = (ntiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int txy = tile % tiles_xy;
  const int z0 = (tile / tiles_xy) * LZ;
  const int x0 = (txy % tiles_x) * TX;
  const int y0 = (txy / tiles_x) * TY;
  const int z1 = z0 + LZ < P.nz ? z0 + LZ : P.nz;

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nx = P.nx, ny = P.ny;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  const long long nxy = (long long)nx * ny;
  const long long st = P.stride;

  T f[7], h1[7], h2[7], nf[7], nh1[7], nh2[7];
  Node<T> s{}, ns{};
  fill_plane(src, P, R, slot_of(z0 - 1), z0 - 1, x0, y0, tx, ty, nf, nh1, nh2, ns);
  fill_plane(src, P, R, slot_of(z0), z0, x0, y0, tx, ty, f, h1, h2, s);

  for (int z = z0; z < z1; ++z) {
    fill_plane(src, P, R, slot_of(z + 1), z + 1, x0, y0, tx, ty, nf, nh1, nh2, ns);
    __syncthreads();
    if (active) {
      const int sm = slot_of(z - 1), s0 = slot_of(z), sp = slot_of(z + 1);
      // isotropic central stencils (Sec. III C) on D3Q19 weights
      T gphi[3] = {0, 0, 0}, gpsi[3] = {0, 0, 0}, lap = 0;
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        const int sl = LG::cz[i] < 0 ? sm : (LG::cz[i] > 0 ? sp : s0);
        const T a = R.phi[sl][ty + 1 + LG::cy[i]][tx + 1 + LG::cx[i]];
        const T b = R.psi[sl][ty + 1 + LG::cy[i]][tx + 1 + LG::cx[i]];
        const T wc = T(LG::w[i] / LG::cs2);
        if (LG::cx[i]) {
          gphi[0] += wc * T(LG::cx[i]) * a;
          gpsi[0] += wc * T(LG::cx[i]) * b;
        }
        if (LG::cy[i]) {
          gphi[1] += wc * T(LG::cy[i]) * a;
          gpsi[1] += wc * T(LG::cy[i]) * b;
        }
        if (LG::cz[i]) {
          gphi[2] += wc * T(LG::cz[i]) * a;
          gpsi[2] += wc * T(LG::cz[i]) * b;
        }
        lap += T(2) * wc * (a - s.dphi);
      }
      const long long node = (long long)z * nxy + (long long)y * nx + x;
      T g[19];
      load_set<LG>(src, st, node, Lay::G0, g);
      Flow<T> fl;
      flow_macros<LG>(P, g, s, gphi, lap, fl);
      if (MODE == kModeMacros) {
        fields[kFieldPhi * st + node] = s.phi;
        fields[kFieldP * st + node] = fl.p;
        fields[kFieldUx * st + node] = fl.u[0];
        fields[kFieldUy * st + node] = fl.u[1];
        fields[kFieldUz * st + node] = fl.u[2];
        fields[kFieldC1 * st + node] = s.c1;
        fields[kFieldC2 * st + node] = s.c2;
        fields[kFieldMu * st + node] = fl.mu;
        fields[kFieldPsi * st + node] = s.c1 + P.Keq * s.c2;
      } else {
        // backward-difference time derivatives against the history (R1)
        T uo[3], dJphi[3], dJ1[3], dJ2[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) uo[a] = hist[a * st + node];
        const T phio = hist[3 * st + node], c1o = hist[4 * st + node], c2o = hist[5 * st + node];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          dJphi[a] = s.phi * fl.u[a] - phio * uo[a];
          dJ1[a] = s.c1 * fl.u[a] - c1o * uo[a];
          dJ2[a] = s.c2 * fl.u[a] - c2o * uo[a];
          hist[a * st + node] = fl.u[a];
        }
        hist[3 * st + node] = s.phi;
        hist[4 * st + node] = s.c1;
        hist[5 * st + node] = s.c2;

        collide<LF, LG>(P, f, g, h1, h2, s, gphi, gpsi, fl, dJphi, dJ1, dJ2);

        // push streaming with periodic wrap or half-way bounce-back
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          int xt = x + LG::cx[i], yt = y + LG::cy[i], zt = z + LG::cz[i];
          bool bounce = false;
          if (xt < 0 || xt >= nx) {
            if (P.wall[0]) bounce = true;
            else xt = xt < 0 ? xt + nx : xt - nx;
          }
          if (yt < 0 || yt >= ny) {
            if (P.wall[1]) bounce = true;
            else yt = yt < 0 ? yt + ny : yt - ny;
          }
          if (zt < 0 || zt >= P.nz) {
            if (P.wall[2]) bounce = true;
            else zt = zt < 0 ? zt + P.nz : zt - P.nz;
          }
          const long long t = bounce ? node : (long long)zt * nxy + (long long)yt * nx + xt;
          store_one<LG>(dst, (Lay::G0 + (bounce ? LG::opp[i] : i)) * st + t, i, g[i]);
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          int xt = x + LF::cx[i], yt = y + LF::cy[i], zt = z + LF::cz[i];
          bool bounce = false;
          if (xt < 0 || xt >= nx) {
            if (P.wall[0]) bounce = true;
            else xt = xt < 0 ? xt + nx : xt - nx;
          }
          if (yt < 0 || yt >= ny) {
            if (P.wall[1]) bounce = true;
            else yt = yt < 0 ? yt + ny : yt - ny;
          }
          if (zt < 0 || zt >= P.nz) {
            if (P.wall[2]) bounce = true;
            else zt = zt < 0 ? zt + P.nz : zt - P.nz;
          }
          const int j = bounce ? LF::opp[i] : i;
          const long long t = bounce ? node : (long long)zt * nxy + (long long)yt * nx + xt;
          store_one<LF>(dst, (Lay::F0 + j) * st + t, i, f[i]);
          store_one<LF>(dst, (Lay::H10 + j) * st + t, i, h1[i]);
          store_one<LF>(dst, (Lay::H20 + j) * st + t, i, h2[i]);
        }
      }
    }
    __syncthreads();  // ring slot of plane z-1 is refilled next iteration
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      f[i] = nf[i];
      h1[i] = nh1[i];
      h2[i] = nh2[i];
    }
    s = ns;
  }
}

}  // namespace

template <class S, class T>
hipError_t launch_step3d(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P, int mode,
                         hipStream_t stream) {
  const int tiles_x = (P.nx + TX - 1) / TX;
  const int tiles_y = (P.ny + TY - 1) / TY;
  const int tiles_z = (P.nz + LZ - 1) / LZ;
  const int tiles_xy = tiles_x * tiles_y;
  const int ntiles = tiles_xy * tiles_z;
  const int nblocks = ((ntiles + 7) / 8) * 8;
  if (mode == kModeMacros)
    hipLaunchKernelGGL((step3d_kernel<S, T, kModeMacros>), dim3(nblocks), dim3(NT), 0, stream, src,
                       dst, hist, fields, P, tiles_x, tiles_xy, ntiles);
  else
    hipLaunchKernelGGL((step3d_kernel<S, T, kModeStep>), dim3(nblocks), dim3(NT), 0, stream, src,
                       dst, hist, fields, P, tiles_x, tiles_xy, ntiles);
  return hipGetLastError();
}

template hipError_t launch_step3d<double, double>(const double*, double*, double*, double*,
                                                  const KParams<double>&, int, hipStream_t);
template hipError_t launch_step3d<float, float>(const float*, float*, float*, float*,
                                                const KParams<float>&, int, hipStream_t);
template hipError_t launch_step3d<__half, float>(const __half*, __half*, float*, float*,
                                                 const KParams<float>&, int, hipStream_t);
template hipError_t launch_step3d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         float*, float*, const KParams<float>&, int,
                                                         hipStream_t);

}  // namespace pflb
