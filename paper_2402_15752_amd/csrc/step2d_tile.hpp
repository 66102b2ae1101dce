// The per-tile body of the 2-D fused step on D2Q9 (f, g, h1, h2 all D2Q9).
//
// A work-group owns a TX x TY tile of nodes, one node per thread:
//   1. every global load the thread needs is issued first: f, h1, h2 of its
//      node (27 values, coalesced along x), its g populations and history,
//      and f, h1, h2 of at most one node of the halo ring around the tile
//      with that node's history references (re-read from L2: the
//      neighbouring tile ran on the same XCD);
//   2. phi, c1, c2 of the tile and its halo go to LDS;
//   3. after one barrier each thread takes the 9-point gradient / Laplacian
//      stencils from LDS, collides all four sets and pushes the
//      post-collision values to x + c_i of the other lattice (periodic wrap
//      or half-way bounce-back), each f, h1, h2 value relative to the
//      moments of the node it lands on (read from the same LDS).
//
// Two histories alternate like the two lattices: the step reads the
// previous level's (u, phi, c1, c2) from `hin` -- at its own nodes for the
// time derivatives and the references, at the halo nodes for their
// references -- and writes this level's to `hout`, so no work-group
// overwrites a value another one may still read.
#pragma once

#include "addr.hpp"
#include "kernels.hpp"

namespace pflb {

template <class Off>
struct Geo2 {
  int nx, ny;
  int px;  // row pitch (nodes)
  int wall_x, wall_y;
  int tiles_x, ntiles;
  Off sS;  // bytes between two population planes
  Off sT;  // bytes between two history / field planes
  const float* closure;  // per-node corrections of c1, c2 (learned closure: the
                         // plane of s1, then that of s2) or null
};

// One TX x TY tile of the fused 2-D step (moments, stencils, macros,
// history, collision, push), shared by the single-lattice and the batched
// kernels.  `tile` is the tile index in row-major order over the grid.
// MODEL kModelOne selects the one-scalar model (Sec. III D): h3 in the h1
// planes, no h2 traffic, no psi stencil, history (u, phi, c);
// kModelTwoDirichlet adds the Dirichlet faces' anti-bounce-back of h1, h2
// (a compiled variant: the check costs the plain step ~5%).
template <class S, class T, int TX, int TY, int NTM, int MODE, class Off, int MODEL = kModelTwo>
__device__ inline void step2d_tile(const S* __restrict__ src, S* __restrict__ dst,
                                   const T* __restrict__ hin, T* __restrict__ hout,
                                   T* __restrict__ fields, const KParams<T>& P, const Geo2<Off>& G,
                                   int tile) {
  using L = D2Q9;
  using Lay = Layout<D2Q9, D2Q9>;
  constexpr bool ONE = MODEL == kModelOne;
  constexpr bool LOC = MODEL == kModelTwoLocal;  // no psi stencil, no h halo
  // the scalar halo: psi stencil, and h1, h2 stored relative to the node's own c1, c2
  constexpr bool HALO_H = !ONE && !LOC;
  constexpr int NT = TX * TY, LX = TX + 2, LY = TY + 2, NHALO = 2 * LX + 2 * TY;
  static_assert(NHALO <= NT, "one halo node per thread at most");
  constexpr Off BS = sizeof(S);
  // non-temporal hints: bit 0 the own node's loads, bit 1 the stores, bit 2
  // the halo node's loads (lines a neighbouring tile reads again)
  constexpr bool NTL = NTM & 1, NTW = NTM & 2, NTH = NTM & 4;
  __shared__ T sphi[LY][LX];
  __shared__ T spi[LY][LX];  // pressure brackets: the references of the flow set
  __shared__ T sc1[HALO_H ? LY : 1][LX];
  __shared__ T sc2[HALO_H ? LY : 1][LX];

  const int x0 = (tile % G.tiles_x) * TX;
  const int y0 = (tile / G.tiles_x) * TY;

  const S* __restrict__ sF = at(src, (size_t)Lay::F0 * G.sS);
  const S* __restrict__ sG = at(src, (size_t)Lay::G0 * G.sS);
  const S* __restrict__ sH1 = at(src, (size_t)Lay::H10 * G.sS);
  const S* __restrict__ sH2 = at(src, (size_t)Lay::H20 * G.sS);

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nx = G.nx, ny = G.ny;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  // a ragged tile: the slot one past the last node is read by that node's
  // stencil, so its thread fills it with the wrapped or mirrored node
  const bool own_slot = x <= nx && y <= ny;
  const Off node = Off(fold(y, ny, G.wall_y) * G.px + fold(x, nx, G.wall_x)) * BS;
  const Off nodeT = node * Off(sizeof(T) / sizeof(S));  // bytes, history / fields

  int hx = 0, hy = 0;
  bool halo = false;
  Off halo_node = 0;
  if (tid < NHALO) {
    halo_pos<TX, TY>(tid, hx, hy);
    const int gx = x0 + hx, gy = y0 + hy;
    halo = gx <= nx && gy <= ny;  // beyond a ragged tile no node reads it
    halo_node = Off(fold(gy, ny, G.wall_y) * G.px + fold(gx, nx, G.wall_x)) * BS;
  }
  const Off halo_nodeT = halo_node * Off(sizeof(T) / sizeof(S));

  // history planes: ux, uy, phi, c1, c2 (one-scalar: ux, uy, phi, c)
  constexpr int kPhi = 2, kC1 = 3, kC2 = 4;
  constexpr int NH = ONE ? kHist2D - 1 : kHist2D;

  // ---- 1. all global loads first
  T f[9], h1[9], h2[9], g[9], hf[9], hh1[9], hh2[9];
  T hs[kHist2D];
  T hr[3] = {T(0), T(0), T(0)};  // references (phi, c1, c2) of the halo node
  T hpi = T(0);                  // and its pressure bracket (rest slot of g)
  if (own_slot) {
    load_q<L, NTL, false>(sF, G.sS, node, f);
    load_q<L, NTL, false>(sH1, G.sS, node, h1);
    if (!ONE) load_q<L, NTL, false>(sH2, G.sS, node, h2);
    load_q<L, NTL, false>(sG, G.sS, node, g);
#pragma unroll
    for (int k = 0; k < NH; ++k) hs[k] = *at(hin, plane<false>(k, G.sT) + nodeT);
  }
  if (halo) {
    load_q<L, NTH, false>(sF, G.sS, halo_node, hf);
    hpi = Codec<S, T>::ld(ld_pop<NTH>(at(sG, halo_node)), T(L::w[0]));
    hr[0] = *at(hin, plane<false>(kPhi, G.sT) + halo_nodeT);
    if (HALO_H) {
      load_q<L, NTH, false>(sH1, G.sS, halo_node, hh1);
      load_q<L, NTH, false>(sH2, G.sS, halo_node, hh2);
      hr[1] = *at(hin, plane<false>(kC1, G.sT) + halo_nodeT);
      hr[2] = *at(hin, plane<false>(kC2, G.sT) + halo_nodeT);
    }
  }

  // ---- 2. moments to LDS
  Node<T> s{};
  if (own_slot) {
    if constexpr (ONE) {
      moments_one<L>(P, f, h1, hs[kPhi], s);
    } else {
      moments<L>(P, f, h1, h2, hs[kPhi], HALO_H ? hs[kC1] : P.ref_c1, HALO_H ? hs[kC2] : P.ref_c2,
                 s);
      if (HALO_H) {
        sc1[ty + 1][tx + 1] = s.c1;
        sc2[ty + 1][tx + 1] = s.c2;
      }
    }
    sphi[ty + 1][tx + 1] = s.phi;
    spi[ty + 1][tx + 1] = g[0];
  }
  if (halo) {
    spi[hy + 1][hx + 1] = hpi;
    if constexpr (!HALO_H) {
      sphi[hy + 1][hx + 1] = hr[0] + phase_sum<L>(hf);
    } else {
      Node<T> q;
      moments<L>(P, hf, hh1, hh2, hr[0], hr[1], hr[2], q);
      sphi[hy + 1][hx + 1] = q.phi;
      sc1[hy + 1][hx + 1] = q.c1;
      sc2[hy + 1][hx + 1] = q.c2;
    }
  }
  __syncthreads();
  if (!active) return;

  // ---- 3. isotropic central stencils (Sec. III C) on D2Q9 weights
  auto nb = [&](const T (&a)[HALO_H ? LY : 1][LX], int i) -> T {
    return a[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]];
  };
  auto nbp = [&](int i) -> T { return sphi[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]]; };
  T gphi[3], gpsi[3] = {T(0), T(0), T(0)};
  grad_pairs<L, T>(nbp, gphi);
  if (P.local_phase) {
    const T uo[3] = {hs[0], hs[1], T(0)};
    local_grad_phi<L>(P, f, s.phi, uo, hs[kPhi], gphi);
  }
  const T lap = lap_of<L, T>(nbp, s.phi);
  if constexpr (HALO_H) {
    // grad psi = grad c1 + Keq grad c2 (psi = c1 + Keq c2)
    T gc1[3], gc2[3];
    grad_pairs<L, T>([&](int i) { return nb(sc1, i); }, gc1);
    grad_pairs<L, T>([&](int i) { return nb(sc2, i); }, gc2);
#pragma unroll
    for (int a = 0; a < 2; ++a) gpsi[a] = gc1[a] + P.Keq * gc2[a];
  }

  // the flow populations relative to the own pressure bracket pi0: a value
  // arriving from x - c_i was stored relative to the bracket of that node
  // (of the node itself when the link bounced off a wall)
  const PushXY<Off> push(x, y, nx, ny, G.px, G.wall_x, G.wall_y, BS);
  const T pi0 = g[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const bool back = (push.bits & link_mask(-L::cx[i], -L::cy[i], 0)) != 0;
    const T src = back ? pi0 : spi[ty + 1 - L::cy[i]][tx + 1 - L::cx[i]];
    g[i] += kp<L, T>(i) * (src - pi0);
  }
  Flow<T> fl;
  flow_macros<L>(P, g, s, gphi, lap, pi0, fl);

  if (MODE == kModeMacros) {
    auto put_field = [&](int k, T v) { *at(fields, plane<false>(k, G.sT) + nodeT) = v; };
    put_field(kFieldPhi, s.phi);
    put_field(kFieldP, fl.p);
    put_field(kFieldUx, fl.u[0]);
    put_field(kFieldUy, fl.u[1]);
    put_field(kFieldUz, T(0));
    put_field(kFieldC1, s.c1);
    put_field(kFieldC2, s.c2);
    put_field(kFieldMu, fl.mu);
    put_field(kFieldPsi, s.c1 + P.Keq * s.c2);
    return;
  }

  // backward-difference time derivatives against the history (R1); the
  // one-scalar model keeps c in the c1 slot
  const T cA = ONE ? s.c : s.c1;
  const T dJphi[3] = {s.phi * fl.u[0] - hs[kPhi] * hs[0], s.phi * fl.u[1] - hs[kPhi] * hs[1], T(0)};
  const T dJ1[3] = {cA * fl.u[0] - hs[kC1] * hs[0], cA * fl.u[1] - hs[kC1] * hs[1], T(0)};
  T dJ2[3] = {T(0), T(0), T(0)};
  if constexpr (!ONE) {
    dJ2[0] = s.c2 * fl.u[0] - hs[kC2] * hs[0];
    dJ2[1] = s.c2 * fl.u[1] - hs[kC2] * hs[1];
  }
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const T v = k < 2 ? fl.u[k] : (k == kPhi ? s.phi : (k == kC1 ? cA : s.c2));
    *at(hout, plane<false>(k, G.sT) + nodeT) = v;
  }

  // push streaming: X_i(x + c_i) <- X_i*(x), or half-way bounce-back into
  // the opposite slot of the own node when the link crosses a wall; each
  // post-collision value is stored as soon as it is formed
  auto bounced = [&](int i) { return (push.bits & link_mask(L::cx[i], L::cy[i], 0)) != 0; };
  auto target = [&](int i) -> Off {
    const int cx = L::cx[i], cy = L::cy[i];
    Off t = node;
    if (cx) t += cx < 0 ? push.dxm : push.dxp;
    if (cy) t += cy < 0 ? push.dym : push.dyp;
    return bounced(i) ? plane<false>(L::opp[i], G.sS) + node + skew<L, S, Off>(L::opp[i])
                      : plane<false>(i, G.sS) + t + skew<L, S, Off>(i);
  };
  // The collisions emit X_i* - w_i R(x), R(x) the node's own reference (its
  // moment at the previous level); the value stored at the target y is
  // X_i* - w_i R'(y), with R'(y) the moment of y at this level, which y's
  // history will hold when the value is read: the neighbour's for a pushed
  // link, the node's own new moment for the rest direction and for a bounced
  // link (both return to x).  `ring` is the LDS array of that moment.
  auto rebase = [&](int i, T v, T rown, const T (&ring)[HALO_H ? LY : 1][LX]) -> T {
    const T rt = bounced(i) ? ring[ty + 1][tx + 1] : ring[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]];
    return v + T(L::w[i]) * (rown - rt);
  };
  auto rebase_phi = [&](int i, T v, T rown) -> T {
    const T rt = bounced(i) ? s.phi : sphi[ty + 1 + L::cy[i]][tx + 1 + L::cx[i]];
    return v + T(L::w[i]) * (rown - rt);
  };
  S* __restrict__ dF = at(dst, (size_t)Lay::F0 * G.sS);
  S* __restrict__ dG = at(dst, (size_t)Lay::G0 * G.sS);
  S* __restrict__ dH1 = at(dst, (size_t)Lay::H10 * G.sS);
  S* __restrict__ dH2 = at(dst, (size_t)Lay::H20 * G.sS);
  const T rphi = hs[kPhi];
  auto emit_f = [&](int i, T v) {
    st_pop<NTW>(at(dF, target(i)),
                Codec<S, T>::st(rebase_phi(i, v, rphi), T(1.0 / L::w[i])));
  };
  // flow set: the new bracket pi, as stored, is the reference of the values
  // this node emits and goes to its own rest slot
  const T pi_st = stored<S, T>(fl.pi, T(L::w[0]), T(1.0 / L::w[0]));
  st_pop<NTW>(at(dG, target(0)), Codec<S, T>::st(fl.pi, T(1.0 / L::w[0])));
  auto emit_g = [&](int i, T v) {
    st_pop<NTW>(at(dG, target(i)),
                Codec<S, T>::st(v + kp<L, T>(i) * (pi0 - pi_st), T(1.0 / L::w[i])));
  };
  // Dirichlet faces this node's links reach (0 for every interior node)
  const int dmask = MODEL == kModelTwoDirichlet ? push.bits & P.dirichlet : 0;
  if constexpr (ONE) {
    T n[3];
    normal(P, gphi, n);
    collide_g<L>(P, g, gphi, fl, emit_g);
    collide_f<L>(P, f, s, n, fl, dJphi, emit_f);
    collide_h3<L>(P, h1, s, fl, dJ1, [&](int i, T v) {
      st_pop<NTW>(at(dH1, target(i)), Codec<S, T>::st(v, T(1.0 / L::w[i])));
    });
    return;
  }
  if constexpr (LOC) {
    // local scheme, Eq. (39): grad c_k from the first moment of the own h_k
    // (deviations carry the same first moment), u, d_t(c_k u) and n of the step
    T n[3];
    normal(P, gphi, n);
    T q1[3] = {T(0), T(0), T(0)}, q2[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (L::cx[i]) {
        q1[0] += T(L::cx[i]) * h1[i];
        q2[0] += T(L::cx[i]) * h2[i];
      }
      if (L::cy[i]) {
        q1[1] += T(L::cy[i]) * h1[i];
        q2[1] += T(L::cy[i]) * h2[i];
      }
    }
    const T f1 = P.d1w * s.omphi * s.c1, f2 = P.d2w * s.phi * s.c2;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T g1 = (s.c1 * fl.u[a] - q1[a] - T(0.5) * dJ1[a] + f1 * n[a]) * P.itc1;
      const T g2 = (s.c2 * fl.u[a] - q2[a] - T(0.5) * dJ2[a] - f2 * n[a]) * P.itc2;
      gpsi[a] = g1 + P.Keq * g2;
    }
  }
  const T rc1 = HALO_H ? hs[kC1] : T(0), rc2 = HALO_H ? hs[kC2] : T(0);
  collide<L, L>(
      P, f, g, h1, h2, s, gphi, gpsi, fl, dJphi, dJ1, dJ2, emit_f, emit_g,
      [&](int i, T a, T b) {
        const Off t = target(i);
        if constexpr (HALO_H) {
          a = rebase(i, a, rc1, sc1);
          b = rebase(i, b, rc2, sc2);
        }
        // half-way anti-bounce-back at a Dirichlet face (the x face first at a
        // corner): h_opp(i) = -h_i* + 2 w_i c_wall; the link returns to the own
        // node, so relative to its new c1, c2 (the bounced value already is)
        if (MODEL == kModelTwoDirichlet && dmask) {
          const int hit = push.bits & link_mask(L::cx[i], L::cy[i], 0);
          if (hit & dmask) {
            const int f = (hit & 1) ? 0 : (hit & 2) ? 1 : (hit & 4) ? 2 : 3;
            if ((dmask >> f) & 1) {
              a = T(2.0 * L::w[i]) * (P.cw[f][0] - s.c1) - a;
              b = T(2.0 * L::w[i]) * (P.cw[f][1] - s.c2) - b;
            }
          }
        }
        st_pop<NTW>(at(dH1, t), Codec<S, T>::st(a, T(1.0 / L::w[i])));
        st_pop<NTW>(at(dH2, t), Codec<S, T>::st(b, T(1.0 / L::w[i])));
      },
      G.closure ? T(G.closure[y * nx + x]) : T(0),
      G.closure ? T(G.closure[(long long)nx * ny + y * nx + x]) : T(0));
}

}  // namespace pflb
