// 3-D fused step: D3Q19 for the flow set g and for the 19-point stencils,
// D3Q7 for f, h1, h2.
//
// One launch = one time step.  A work-group owns a TX x TY column tile and
// marches along z over a chunk of LZ planes.  LDS holds a ring of four
// planes of the deviations of phi and psi = c1 + Keq c2 over the tile and
// its one-node halo.  Per plane z the group
//   1. loads f, h1, h2 (21 values) of its own nodes at z+1 -- kept in
//      registers for the next plane -- and of at most one halo node at z+1
//      (re-read from L2: neighbouring tiles march the same planes on the
//      same XCD); the prefetching variants also load g and history of plane
//      z here, before the barrier (more loads in flight per wave, fewer
//      waves: it doubles the registers);
//   2. puts the moments of plane z+1 in the ring, then one barrier;
//   3. collides plane z: 19-point stencils from ring planes z-1, z, z+1,
//      all four sets collided and pushed to x + c_i of the other lattice
//      (periodic wrap or half-way bounce-back).
// With four ring slots a plane's slot is reused two barriers after its last
// reader, so one barrier per plane suffices.  Interior moments are computed
// once per node; only the halo ring and the first two planes of a chunk are
// recomputed.
#include "kernels.hpp"

namespace pflb {

namespace {

using LF = D3Q7;
using LG = D3Q19;
using Lay = Layout<D3Q7, D3Q19>;

__device__ inline int fold(int v, int n, int wall) {
  if (v < 0) return wall ? 0 : v + n;
  if (v >= n) return wall ? n - 1 : v - n;
  return v;
}

__device__ inline int slot_of(int z) { return (z + 4) & 3; }

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
__device__ inline void load_fh(const S* __restrict__ src, long long st, long long node, T (&f)[7],
                               T (&h1)[7], T (&h2)[7]) {
  load_set<LF, NTS>(src, st, node, Lay::F0, f);
  load_set<LF, NTS>(src, st, node, Lay::H10, h1);
  load_set<LF, NTS>(src, st, node, Lay::H20, h2);
}

template <class T, int TX, int TY>
struct Ring {
  T phi[4][TY + 2][TX + 2];
  T psi[4][TY + 2][TX + 2];
};

template <class S, class T, int TX, int TY, int LZ, bool NTS, bool PREF, int MODE>
__global__ __launch_bounds__(TX* TY) void step3d_kernel(const S* __restrict__ src,
                                                        S* __restrict__ dst, T* __restrict__ hist,
                                                        T* __restrict__ fields, KParams<T> P,
                                                        int tiles_x, int tiles_xy, int ntiles) {
  constexpr int NT = TX * TY, LX = TX + 2, NHALO = 2 * LX + 2 * TY;
  static_assert(NHALO <= NT, "one halo node per thread at most");
  __shared__ Ring<T, TX, TY> R;
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
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  const bool own_slot = x <= nx && y <= ny;  // ragged tile: fill the slot past the end
  const long long nxy = (long long)nx * ny;
  const long long st = P.stride;
  const long long own_col = (long long)fold(y, ny, P.wall[1]) * nx + fold(x, nx, P.wall[0]);

  int hx = 0, hy = 0;
  bool halo = false;
  long long halo_col = 0;
  if (tid < NHALO) {
    halo_pos<TX, TY>(tid, hx, hy);
    const int gx = x0 + hx, gy = y0 + hy;
    halo = gx <= nx && gy <= ny;
    halo_col = (long long)fold(gy, ny, P.wall[1]) * nx + fold(gx, nx, P.wall[0]);
  }

  // moments of plane zp for the own slot and the halo slot of the ring
  auto put = [&](int zp, const T (&f)[7], const T (&h1)[7], const T (&h2)[7], Node<T>& s,
                 const T (&hf)[7], const T (&hh1)[7], const T (&hh2)[7]) {
    const int sl = slot_of(zp);
    if (own_slot) {
      moments<LF>(P, f, h1, h2, s);
      R.phi[sl][ty + 1][tx + 1] = s.dphi;
      R.psi[sl][ty + 1][tx + 1] = s.dc1 + P.Keq * s.dc2;
    }
    if (halo) {
      Node<T> q;
      moments<LF>(P, hf, hh1, hh2, q);
      R.phi[sl][hy + 1][hx + 1] = q.dphi;
      R.psi[sl][hy + 1][hx + 1] = q.dc1 + P.Keq * q.dc2;
    }
  };

  T f[7], h1[7], h2[7];  // own populations of the plane being collided
  Node<T> s{};
  {
    // prologue: planes z0-1 and z0
    T af[7], ah1[7], ah2[7], hf[7], hh1[7], hh2[7];
    const long long pm = (long long)fold(z0 - 1, nz, P.wall[2]) * nxy;
    const long long p0 = (long long)z0 * nxy;
    if (own_slot) load_fh<NTS>(src, st, pm + own_col, af, ah1, ah2);
    if (halo) load_fh<NTS>(src, st, pm + halo_col, hf, hh1, hh2);
    Node<T> tmp;
    put(z0 - 1, af, ah1, ah2, tmp, hf, hh1, hh2);
    if (own_slot) load_fh<NTS>(src, st, p0 + own_col, f, h1, h2);
    if (halo) load_fh<NTS>(src, st, p0 + halo_col, hf, hh1, hh2);
    put(z0, f, h1, h2, s, hf, hh1, hh2);
  }

  for (int z = z0; z < z1; ++z) {
    const long long node = (long long)z * nxy + (long long)y * nx + x;
    const long long pn = (long long)fold(z + 1, nz, P.wall[2]) * nxy;
    // ---- 1. global loads of this plane
    T g[19], hs[kHist3D], nf[7], nh1[7], nh2[7], hf[7], hh1[7], hh2[7];
    auto load_g = [&] {
      load_set<LG, NTS>(src, st, node, Lay::G0, g);
#pragma unroll
      for (int k = 0; k < kHist3D; ++k) hs[k] = hist[k * st + node];
    };
    if (PREF && active) load_g();
    if (own_slot) load_fh<NTS>(src, st, pn + own_col, nf, nh1, nh2);
    if (halo) load_fh<NTS>(src, st, pn + halo_col, hf, hh1, hh2);
    // ---- 2. moments of plane z+1 into the ring
    Node<T> ns{};
    put(z + 1, nf, nh1, nh2, ns, hf, hh1, hh2);
    __syncthreads();
    // ---- 3. collide plane z
    if (active) {
      if (!PREF) load_g();
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
        T dJphi[3], dJ1[3], dJ2[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          dJphi[a] = s.phi * fl.u[a] - hs[3] * hs[a];
          dJ1[a] = s.c1 * fl.u[a] - hs[4] * hs[a];
          dJ2[a] = s.c2 * fl.u[a] - hs[5] * hs[a];
          hist[a * st + node] = fl.u[a];
        }
        hist[3 * st + node] = s.phi;
        hist[4 * st + node] = s.c1;
        hist[5 * st + node] = s.c2;

        // push streaming with periodic wrap or half-way bounce-back; each
        // post-collision value is stored as soon as it is formed
        auto dest = [&](int cx, int cy, int cz, bool& bounce) -> long long {
          int xt = x + cx, yt = y + cy, zt = z + cz;
          bounce = false;
          if (xt < 0 || xt >= nx) {
            if (P.wall[0]) bounce = true;
            else xt = xt < 0 ? xt + nx : xt - nx;
          }
          if (yt < 0 || yt >= ny) {
            if (P.wall[1]) bounce = true;
            else yt = yt < 0 ? yt + ny : yt - ny;
          }
          if (zt < 0 || zt >= nz) {
            if (P.wall[2]) bounce = true;
            else zt = zt < 0 ? zt + nz : zt - nz;
          }
          return bounce ? node : (long long)zt * nxy + (long long)yt * nx + xt;
        };
        collide<LF, LG>(
            P, f, g, h1, h2, s, gphi, gpsi, fl, dJphi, dJ1, dJ2,
            [&](int i, T v) {
              bool b;
              const long long t = dest(LF::cx[i], LF::cy[i], LF::cz[i], b);
              store_one<LF, NTS>(dst, (Lay::F0 + (b ? LF::opp[i] : i)) * st + t, i, v);
            },
            [&](int i, T v) {
              bool b;
              const long long t = dest(LG::cx[i], LG::cy[i], LG::cz[i], b);
              store_one<LG, NTS>(dst, (Lay::G0 + (b ? LG::opp[i] : i)) * st + t, i, v);
            },
            [&](int i, T a, T c) {
              bool b;
              const long long t = dest(LF::cx[i], LF::cy[i], LF::cz[i], b);
              const int j = b ? LF::opp[i] : i;
              store_one<LF, NTS>(dst, (Lay::H10 + j) * st + t, i, a);
              store_one<LF, NTS>(dst, (Lay::H20 + j) * st + t, i, c);
            });
      }
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      f[i] = nf[i];
      h1[i] = nh1[i];
      h2[i] = nh2[i];
    }
    s = ns;
  }
}

template <class S, class T, int TX, int TY, int LZ, bool NTS, bool PREF, int MODE>
hipError_t launch_variant(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P,
                          hipStream_t stream) {
  const int tiles_x = (P.nx + TX - 1) / TX;
  const int tiles_y = (P.ny + TY - 1) / TY;
  const int tiles_z = (P.nz + LZ - 1) / LZ;
  const int tiles_xy = tiles_x * tiles_y;
  const int ntiles = tiles_xy * tiles_z;
  const int nblocks = ((ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL((step3d_kernel<S, T, TX, TY, LZ, NTS, PREF, MODE>), dim3(nblocks), dim3(TX * TY),
                     0, stream, src, dst, hist, fields, P, tiles_x, tiles_xy, ntiles);
  return hipGetLastError();
}

}  // namespace

const char* step3d_variant_name(int v) {
  static const char* names[kVariants3D] = {"32x8",    "64x4",    "32x4",         "32x8 nt",
                                          "64x4 nt", "32x4 nt", "32x8 prefetch", "32x8 prefetch nt"};
  return v >= 0 && v < kVariants3D ? names[v] : "?";
}

template <class S, class T>
hipError_t launch_step3d(const S* src, S* dst, T* hist, T* fields, const KParams<T>& P, int mode,
                         int variant, hipStream_t stream) {
  constexpr int M = kModeStep;
  if (mode == kModeMacros)
    return launch_variant<S, T, 32, 8, 64, false, false, kModeMacros>(src, dst, hist, fields, P,
                                                                      stream);
  switch (variant) {
    case 1: return launch_variant<S, T, 64, 4, 64, false, false, M>(src, dst, hist, fields, P, stream);
    case 2: return launch_variant<S, T, 32, 4, 64, false, false, M>(src, dst, hist, fields, P, stream);
    case 3: return launch_variant<S, T, 32, 8, 64, true, false, M>(src, dst, hist, fields, P, stream);
    case 4: return launch_variant<S, T, 64, 4, 64, true, false, M>(src, dst, hist, fields, P, stream);
    case 5: return launch_variant<S, T, 32, 4, 64, true, false, M>(src, dst, hist, fields, P, stream);
    case 6: return launch_variant<S, T, 32, 8, 64, false, true, M>(src, dst, hist, fields, P, stream);
    case 7: return launch_variant<S, T, 32, 8, 64, true, true, M>(src, dst, hist, fields, P, stream);
    default: return launch_variant<S, T, 32, 8, 64, false, false, M>(src, dst, hist, fields, P, stream);
  }
}

template hipError_t launch_step3d<double, double>(const double*, double*, double*, double*,
                                                  const KParams<double>&, int, int, hipStream_t);
template hipError_t launch_step3d<float, float>(const float*, float*, float*, float*,
                                                const KParams<float>&, int, int, hipStream_t);
template hipError_t launch_step3d<__half, float>(const __half*, __half*, float*, float*,
                                                 const KParams<float>&, int, int, hipStream_t);
template hipError_t launch_step3d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         float*, float*, const KParams<float>&, int,
                                                         int, hipStream_t);

}  // namespace pflb
