// 3-D fused step: D3Q19 for the flow set g and for the 19-point stencils,
// D3Q7 for f, h1, h2.
//
// One launch = one time step.  A work-group owns a TX x TY column tile and
// marches along z over a chunk of planes.  LDS holds a ring of four
// planes of phi, c1 and c2 over the tile and its one-node halo.  Per plane
// z the group
//   1. loads f, h1, h2 (21 values) and their references (phi, c1, c2 of
//      the previous level, from the history) of its own nodes at z+1 --
//      kept for the next plane (in registers, or in LDS) -- and of at most
//      one halo node at z+1 (re-read from L2: neighbouring tiles march the
//      same planes on the same XCD); the prefetching variants also load g
//      and the velocity history of plane z here, before the barrier;
//   2. puts the moments of plane z+1 in the ring, then one barrier;
//   3. collides plane z: 19-point stencils from ring planes z-1, z, z+1,
//      all four sets collided and pushed to x + c_i of the other lattice
//      (periodic wrap or half-way bounce-back), each f, h1, h2 value
//      relative to the moments of the node it lands on (read from the ring).
// The histories alternate like the lattices (read `hin`, write `hout`), so
// no work-group overwrites a reference another one still reads.
// With four ring slots a plane's slot is reused two barriers after its last
// reader, so one barrier per plane suffices.  Interior moments are computed
// once per node; only the halo ring and the first two planes of a chunk are
// recomputed.
//
// Addressing.  A value is reached by a byte offset plane * stride + node,
// split into a per-lane part (the node's column within its z plane, and the
// x / y step of a push) and a uniform part (set, plane, skew, z plane and
// z step of a push).  With FP32 or FP64 storage, when the lattice, the
// history and the field buffer each span < 4 GiB (the usual case), every
// access is a buffer access over one resource per allocation: the address
// unit adds the scalar part to the vector part, so loads cost no vector
// instruction and a push store one at most.  16-bit lattices, and larger
// FP32 / FP64 ones whose sets stay below 4 GiB (one tile shape), take
// 32-bit offsets from a 64-bit base per set; larger ones 64-bit offsets.
// Push targets come from per-lane x / y neighbour deltas and
// per-plane z deltas computed once; bounce-back is a per-lane select, not
// a branch.
//
// Scalar registers.  The loop body reads the lattice constants through a
// pointer and the plane stride through values that the compiler must treat
// as new on every use (opaque()), so it rematerialises them where they are
// needed instead of keeping ~80 loop-invariant scalars live across the
// z loop, which overflows the scalar file and spills into vector lanes.
#include <atomic>
#include <cmath>
#include <type_traits>

#include "addr.hpp"
#include "kernels.hpp"

namespace pflb {

namespace {

using LF = D3Q7;
using LG = D3Q19;
using Lay = Layout<D3Q7, D3Q19>;

template <class Off>
struct Geo3 {
  int nx, ny, nz;
  int px;   // row pitch (nodes)
  int wall_x, wall_y, wall_z;
  int tiles_x, tiles_xy, ntiles;
  int nchunks;  // z chunks per column tile
  Off sS;   // bytes between two population planes
  Off sT;   // bytes between two history / field planes
  Off nxy;  // bytes between two z-planes of a population plane (px ny sizeof(S))
};

__device__ inline int slot_of(int z) { return (z + 4) & 3; }

enum { kCarryRegs = 0, kCarryLate = 1, kCarryLds = 2 };

template <class T, int TX, int TY, bool PSI>
struct Ring {
  // phi, c1, c2 of four planes over the tile and its halo, exactly the
  // values the nodes' histories keep (the references of their populations)
  T phi[4][TY + 2][TX + 2];
  T pi[4][TY + 2][TX + 2];  // pressure brackets: the references of the flow set
  T c1[PSI ? 4 : 1][TY + 2][TX + 2];  // no scalar ring with the local gradient scheme
  T c2[PSI ? 4 : 1][TY + 2][TX + 2];
};

// LOC: grad(c1 + Keq c2) by the local scheme of Eq. (39) from the own h1, h2
// of the plane being collided -- no scalar ring, no h1, h2 of the halo; h1,
// h2 then keep the uniform reference (c1_ref, c2_ref).
template <class S, class T, int TX, int TY, int NT, bool PREF, int CARRY, int WPE, int MODE, class Off,
          bool LOC, bool BUF>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WPE))) void step3d_kernel(const S* __restrict__ src,
                                                        S* __restrict__ dst,
                                                        const T* __restrict__ hin,
                                                        T* __restrict__ hout,
                                                        T* __restrict__ fields,
                                                        KPtr<T> Pg, Geo3<Off> G) {
  constexpr int NTH = TX * TY, LX = TX + 2, NHALO = 2 * LX + 2 * TY;
  static_assert(NHALO <= NTH, "one halo node per thread at most");
  // non-temporal hints: bit 0 f / h loads, bit 1 stores, bit 2 g loads
  constexpr bool NTL = NT & 1, NTW = NT & 2, NTG = NT & 4;
  constexpr Off BS = sizeof(S);
  constexpr int kPhi = 3, kC1 = 4, kC2 = 5;  // history planes: ux, uy, uz, phi, c1, c2
  // where the own f, h1, h2 of a plane wait for its collision one z step
  // after their load: registers, L2 (LATE: read again), or LDS (LDSC)
  constexpr bool LATE = CARRY == kCarryLate, LDSC = CARRY == kCarryLds;
  __shared__ Ring<T, TX, TY, !LOC> R;
  // LDSC: the lane's own f, h1, h2 of the plane being collided (each lane
  // reads and writes only its own column: no barrier)
  __shared__ T own[LDSC ? 21 : 1][LDSC ? NTH : 1];
  // XCD-aware order (see the 2-D kernel): XCD k runs a contiguous tile range
  const int per = (G.ntiles + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= G.ntiles) return;
  const int txy = tile % G.tiles_xy;
  const int zc = tile / G.tiles_xy;  // z chunk: planes [z0, z1), balanced to one plane
  const int z0 = (int)((long long)zc * G.nz / G.nchunks);
  const int x0 = (txy % G.tiles_x) * TX;
  const int y0 = (txy / G.tiles_x) * TY;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int z1 = (int)((long long)(zc + 1) * G.nz / G.nchunks);

  // Population sets: with BUF one buffer resource spans each lattice and a
  // set's first plane joins the uniform offset; otherwise each set has a
  // 64-bit base (scalar arithmetic, once).  The history and the field
  // buffer are reached the same way.
  using VS = View<BUF, const S, Off>;
  using VD = View<BUF, S, Off>;
  const Off lat_bytes = BUF ? Off(Lay::QTOT) * G.sS : Off(0);
  const VS sF(BUF ? src : at(src, (size_t)Lay::F0 * G.sS), lat_bytes);
  const VS sG(BUF ? src : at(src, (size_t)Lay::G0 * G.sS), lat_bytes);
  const VS sH1(BUF ? src : at(src, (size_t)Lay::H10 * G.sS), lat_bytes);
  const VS sH2(BUF ? src : at(src, (size_t)Lay::H20 * G.sS), lat_bytes);
  const View<BUF, const T, Off> vin(hin, BUF ? Off(kHist3D) * G.sT : Off(0));
  const View<BUF, T, Off> vout(hout, BUF ? Off(kHist3D) * G.sT : Off(0));
  // byte offset of plane i of population set `set` from that set's view
  auto pp = [&](int set, int i) -> Off { return plane<true>((BUF ? set : 0) + i, G.sS); };
  // The (lane, uniform) parts of an access at column `col` of the z plane at
  // byte offset `zb`, plus the access's own uniform offset u (set, plane)
  // and constant k (skew).  BUF keeps the z plane in the uniform part; the
  // global form adds it to the column once per plane (the node's offset)
  // and u and k to that per access, k as the instruction's offset.
  struct Acc {
    Off lane, uni;
  };
  auto acc = [&](Off col, Off zb, Off u, Off k) -> Acc {
    if constexpr (BUF)
      return Acc{col, u + zb + k};
    else
      return Acc{Off(0), u + (zb + col) + k};
  };

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < nx && y < ny;
  const bool own_slot = x <= nx && y <= ny;  // ragged tile: fill the slot past the end
  // Every lane loads its own column, lanes past the slot that of node 0 (its
  // values are not used): unconditional loads, so the compiler need not
  // zero their registers for a skipped branch.
  const Off own_col =
      own_slot ? Off(fold(y, ny, G.wall_y) * G.px + fold(x, nx, G.wall_x)) * BS : Off(0);
  constexpr Off TS = Off(sizeof(T) / sizeof(S));  // population bytes -> history bytes

  int hx = 0, hy = 0;
  bool halo = false;
  Off halo_col = 0;
  if (tid < NHALO) {
    halo_pos<TX, TY>(tid, hx, hy);
    const int gx = x0 + hx, gy = y0 + hy;
    halo = gx <= nx && gy <= ny;
    halo_col = Off(fold(gy, ny, G.wall_y) * G.px + fold(gx, nx, G.wall_x)) * BS;
  }

  const PushXY<Off> push(x, y, nx, ny, G.px, G.wall_x, G.wall_y, BS);

  // Loads of a node: `col` its byte offset within a z plane (per lane),
  // `zb` the byte offset of its z plane (uniform).
  // the 7 populations of a D3Q7 set
  auto ldq = [&](const VS& v, int set, Off col, Off zb, T (&x)[7]) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const Acc a = acc(col, zb, pp(set, i), skew<LF, S, Off>(i));
      x[i] = Codec<S, T>::ld(v.template ld<NTL>(a.lane, a.uni), T(LF::w[i]));
    }
  };
  // history and field planes (T values): the column and z plane in T bytes
  auto ldh = [&](Off col, Off zb, int k) -> T {
    const Acc a = acc(col * TS, zb * TS, plane<true>(k, G.sT), Off(0));
    return vin.template ld<false>(a.lane, a.uni);
  };
  auto load_fh = [&](Off col, Off zb, T (&f)[7], T (&h1)[7], T (&h2)[7]) {
    ldq(sF, Lay::F0, col, zb, f);
    ldq(sH1, Lay::H10, col, zb, h1);
    ldq(sH2, Lay::H20, col, zb, h2);
  };
  // the references (phi, c1, c2 of the previous level) of a node
  auto load_ref = [&](Off col, Off zb, T (&r)[3]) {
    r[0] = ldh(col, zb, kPhi);
    if (!LOC) {
      r[1] = ldh(col, zb, kC1);
      r[2] = ldh(col, zb, kC2);
    } else {
      r[1] = T(0);
      r[2] = T(0);
    }
  };
  // the pressure bracket a node's flow populations are stored relative to
  // (the rest slot of its g)
  auto load_pi = [&](Off col, Off zb) -> T {
    const Acc a = acc(col, zb, pp(Lay::G0, 0), Off(0));
    return Codec<S, T>::ld(sG.template ld<NTG>(a.lane, a.uni), T(LG::w[0]));
  };
  // moments of plane zp of the own node into the ring
  auto put_own = [&](const KParams<T>& P, int zp, const T (&f)[7], const T (&h1)[7],
                     const T (&h2)[7], const T (&r)[3], T pi, Node<T>& s) {
    moments<LF>(P, f, h1, h2, r[0], LOC ? P.ref_c1 : r[1], LOC ? P.ref_c2 : r[2], s);
    if (own_slot) {
      const int sl = slot_of(zp);
      R.phi[sl][ty + 1][tx + 1] = s.phi;
      R.pi[sl][ty + 1][tx + 1] = pi;
      if (!LOC) {
        R.c1[sl][ty + 1][tx + 1] = s.c1;
        R.c2[sl][ty + 1][tx + 1] = s.c2;
      }
    }
  };
  // load plane zp of the lane's halo node and put its moments in the ring,
  // in one conditional block (the halo needs h1, h2 only for the scalar ring)
  auto halo_plane = [&](const KParams<T>& P, int zp, Off pbase) {
    if (!halo) return;
    const int sl = slot_of(zp);
    T hf[7], hr[3];
    ldq(sF, Lay::F0, halo_col, pbase, hf);
    load_ref(halo_col, pbase, hr);
    R.pi[sl][hy + 1][hx + 1] = load_pi(halo_col, pbase);
    if constexpr (LOC) {
      R.phi[sl][hy + 1][hx + 1] = hr[0] + phase_sum<LF>(hf);
    } else {
      T hh1[7], hh2[7];
      ldq(sH1, Lay::H10, halo_col, pbase, hh1);
      ldq(sH2, Lay::H20, halo_col, pbase, hh2);
      Node<T> q;
      moments<LF>(P, hf, hh1, hh2, hr[0], hr[1], hr[2], q);
      R.phi[sl][hy + 1][hx + 1] = q.phi;
      R.c1[sl][hy + 1][hx + 1] = q.c1;
      R.c2[sl][hy + 1][hx + 1] = q.c2;
    }
  };

  T f[7], h1[7], h2[7];  // own populations of the plane being collided
  T r[3];                // and their references
  Node<T> s{};
  {
    // prologue: planes z0-1 and z0
    const KParams<T>& P = params(Pg);
    T af[7], ah1[7], ah2[7], ar[3];
    const Off pm = Off(fold(z0 - 1, nz, G.wall_z)) * G.nxy;
    const Off p0 = Off(z0) * G.nxy;
    load_fh(own_col, pm, af, ah1, ah2);
    load_ref(own_col, pm, ar);
    const T apm = load_pi(own_col, pm);
    halo_plane(P, z0 - 1, pm);
    Node<T> tmp;
    put_own(P, z0 - 1, af, ah1, ah2, ar, apm, tmp);
    load_fh(own_col, p0, f, h1, h2);
    load_ref(own_col, p0, r);
    const T ap0 = load_pi(own_col, p0);
    halo_plane(P, z0, p0);
    put_own(P, z0, f, h1, h2, r, ap0, s);
    if constexpr (LDSC) {
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        own[i][tid] = f[i];
        own[7 + i][tid] = h1[i];
        own[14 + i][tid] = h2[i];
      }
    }
  }
  // LATE: the own f, h1, h2 of plane z are read again (L1 / L2 hits when
  // the lines survive the plane step) right before collide_f and
  // collide_h, instead of being held in registers from the previous plane
  // through the whole g collision; only the node state and references are
  // carried.  LDSC: they wait in LDS, each lane's own slots: collide_f
  // takes this plane's f out of them and puts the next plane's in (held in
  // registers since its load), collide_h the same for h1, h2.  Through the
  // flow collision 21 values fewer are live than with registers only.

  for (int z = z0; z < z1; ++z) {
    const KParams<T>& P = params(Pg);
    const Off zoff = Off(z) * G.nxy;  // bytes, population arrays (uniform)
    const Off node = zoff + own_col;  // the global form's per-lane offset of the node
    const Off pn = Off(fold(z + 1, nz, G.wall_z)) * G.nxy;
    // ---- 1. global loads of this plane
    T g[19], uo[3], nf[7], nh1[7], nh2[7], nr[3];
    auto load_g = [&] {
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        const Acc a = acc(own_col, zoff, pp(Lay::G0, i), skew<LG, S, Off>(i));
        g[i] = Codec<S, T>::ld(sG.template ld<NTG>(a.lane, a.uni), T(LG::w[i]));
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) uo[k] = ldh(own_col, zoff, k);
    };
    if (PREF && active) load_g();
    load_fh(own_col, pn, nf, nh1, nh2);
    load_ref(own_col, pn, nr);
    const T npi = load_pi(own_col, pn);
    // ---- 2. moments of plane z+1 into the ring
    halo_plane(P, z + 1, pn);
    Node<T> ns;
    put_own(P, z + 1, nf, nh1, nh2, nr, npi, ns);
    __syncthreads();
    // ---- 3. collide plane z
    if (active) {
      if (!PREF) load_g();
      const int sm = slot_of(z - 1), s0 = slot_of(z), sp = slot_of(z + 1);
      auto slot = [&](int i) { return LG::cz[i] < 0 ? sm : (LG::cz[i] > 0 ? sp : s0); };
      // isotropic central stencils (Sec. III C) on D3Q19 weights
      auto nbp = [&](int i) -> T { return R.phi[slot(i)][ty + 1 + LG::cy[i]][tx + 1 + LG::cx[i]]; };
      T gphi[3], gpsi[3] = {T(0), T(0), T(0)};
      grad_pairs<LG, T>(nbp, gphi);
      const T lap = lap_of<LG, T>(nbp, s.phi);
      if (P.local_phase) {
        if (LATE) ldq(sF, Lay::F0, own_col, zoff, f);
        if constexpr (LDSC) {
#pragma unroll
          for (int i = 0; i < 7; ++i) f[i] = own[i][tid];
        }
        local_grad_phi<LF>(P, f, s.phi, uo, r[0], gphi);
      }
      if constexpr (!LOC) {
        // grad psi = grad c1 + Keq grad c2 (psi = c1 + Keq c2)
        T gc1[3], gc2[3];
        grad_pairs<LG, T>([&](int i) { return R.c1[slot(i)][ty + 1 + LG::cy[i]][tx + 1 + LG::cx[i]]; },
                          gc1);
        grad_pairs<LG, T>([&](int i) { return R.c2[slot(i)][ty + 1 + LG::cy[i]][tx + 1 + LG::cx[i]]; },
                          gc2);
#pragma unroll
        for (int a = 0; a < 3; ++a) gpsi[a] = gc1[a] + P.Keq * gc2[a];
      }
      // z bounce bits of this plane (uniform) with the lane's x / y ones
      int bits = push.bits;
      if (z == 0 && G.wall_z) bits |= 16;
      if (z == nz - 1 && G.wall_z) bits |= 32;
      // Walls is uniform over the wave: true only where a lane of it has a
      // wall link (the first and last planes of a walled z axis, the columns
      // of walled x / y faces); elsewhere no link needs the wall selects.
      const bool walls = __ballot(bits != 0) != 0;
      // the flow populations relative to the own pressure bracket pi0: a
      // value arriving from x - c_i was stored relative to the bracket of
      // that node (of the node itself when the link bounced off a wall)
      const T pi0 = R.pi[s0][ty + 1][tx + 1];
      g[0] = pi0;
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        const bool back = (bits & link_mask(-LG::cx[i], -LG::cy[i], -LG::cz[i])) != 0;
        const int sl = LG::cz[i] > 0 ? sm : (LG::cz[i] < 0 ? sp : s0);
        const T src = back ? pi0 : R.pi[sl][ty + 1 - LG::cy[i]][tx + 1 - LG::cx[i]];
        g[i] += kp<LG, T>(i) * (src - pi0);
      }
      Flow<T> fl;
      flow_macros<LG>(P, g, s, gphi, lap, pi0, fl);
      if (MODE == kModeMacros) {
        const View<BUF, T, Off> vf(fields, BUF ? Off(kNumFields) * G.sT : Off(0));
        auto put_field = [&](int k, T v) {
          const Acc a = acc(own_col * TS, zoff * TS, plane<true>(k, G.sT), Off(0));
          vf.template st<false>(a.lane, a.uni, v);
        };
        put_field(kFieldPhi, s.phi);
        put_field(kFieldP, fl.p);
        put_field(kFieldUx, fl.u[0]);
        put_field(kFieldUy, fl.u[1]);
        put_field(kFieldUz, fl.u[2]);
        put_field(kFieldC1, s.c1);
        put_field(kFieldC2, s.c2);
        put_field(kFieldMu, fl.mu);
        put_field(kFieldPsi, s.c1 + P.Keq * s.c2);
      } else {
        // backward-difference time derivatives against the history (R1):
        // the references are the previous level's phi, c1, c2
        T dJphi[3], dJ1[3], dJ2[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          dJphi[a] = s.phi * fl.u[a] - r[0] * uo[a];
          dJ1[a] = s.c1 * fl.u[a] - (LOC ? ldh(own_col, zoff, kC1) : r[1]) * uo[a];
          dJ2[a] = s.c2 * fl.u[a] - (LOC ? ldh(own_col, zoff, kC2) : r[2]) * uo[a];
        }
#pragma unroll
        for (int k = 0; k < kHist3D; ++k) {
          const T v = k < 3 ? fl.u[k] : (k == kPhi ? s.phi : (k == kC1 ? s.c1 : s.c2));
          const Acc h = acc(own_col * TS, zoff * TS, plane<true>(k, G.sT), Off(0));
          vout.template st<false>(h.lane, h.uni, v);
        }

        // z push deltas of this plane (uniform)
        Off dzm = Off(0) - G.nxy, dzp = G.nxy;
        if (z == 0) dzm = Off(nz - 1) * G.nxy;
        if (z == nz - 1) dzp = Off(0) - Off(nz - 1) * G.nxy;
        // byte offset of the push target of direction i (plane i of set
        // `set`), or of the bounce-back target (plane opp(i), this node); the
        // plane skew of direction i is -c_ix nodes, that of opp(i) +c_ix.
        // Without walls in the wave a store takes its push target as a
        // per-lane part (the node and its x / y step) and a uniform part
        // (plane, skew, z plane and step).  With walls both whole offsets
        // are formed and selected per lane (the plane offsets are opaque to
        // the compiler, which would otherwise branch around each one).
        auto bounced = [&](int cx, int cy, int cz) {
          return walls && (bits & link_mask(cx, cy, cz)) != 0;
        };
        struct Tgt {
          Off lane, uni;
        };
        auto target = [&](int set, int i, int o, int cx, int cy, int cz) -> Tgt {
          const Off sk = cx > 0 ? Off(0) - BS : (cx < 0 ? BS : Off(0));
          if constexpr (BUF) {
            Off lane = own_col;
            if (cx) lane += cx < 0 ? push.dxm : push.dxp;
            if (cy) lane += cy < 0 ? push.dym : push.dyp;
            Off uni = pp(set, i) + zoff + sk;
            if (cz) uni += cz < 0 ? dzm : dzp;
            if (!walls) return Tgt{lane, uni};
            const Off back_t = pp(set, o) + zoff - sk + own_col;
            return Tgt{(bits & link_mask(cx, cy, cz)) ? back_t : lane + uni, Off(0)};
          } else {
            // the whole offset per lane: the node, its x / y / z step, then
            // plane and skew
            Off tn = node;
            if (cx) tn += cx < 0 ? push.dxm : push.dxp;
            if (cy) tn += cy < 0 ? push.dym : push.dyp;
            if (cz) tn += cz < 0 ? dzm : dzp;
            const Off push_t = pp(set, i) + tn + sk;
            if (!walls) return Tgt{push_t, Off(0)};
            const Off back_t = pp(set, o) + node - sk;
            return Tgt{(bits & link_mask(cx, cy, cz)) ? back_t : push_t, Off(0)};
          }
        };
        // The collisions emit X_i* - w_i R(x), R(x) the node's own reference
        // (its moment at the previous level); the D3Q7 value stored at the
        // target y is X_i* - w_i R'(y), with R'(y) the moment of y at this
        // level, which y's history will hold when the value is read: the
        // neighbour's for a pushed link, the node's own new moment for the
        // rest direction and for a bounced link (both return to x)
        auto rebase = [&](int i, T v, T rown, const T (&ring)[4][TY + 2][TX + 2]) -> S {
          const int sl = LF::cz[i] < 0 ? sm : (LF::cz[i] > 0 ? sp : s0);
          const T rt = bounced(LF::cx[i], LF::cy[i], LF::cz[i])
                           ? ring[s0][ty + 1][tx + 1]
                           : ring[sl][ty + 1 + LF::cy[i]][tx + 1 + LF::cx[i]];
          return store_shifted<S, T>(v, rown - rt, T(LF::w[i]), T(1.0 / LF::w[i]));
        };
        const VD dF(BUF ? dst : at(dst, (size_t)Lay::F0 * G.sS), lat_bytes);
        const VD dG(BUF ? dst : at(dst, (size_t)Lay::G0 * G.sS), lat_bytes);
        const VD dH1(BUF ? dst : at(dst, (size_t)Lay::H10 * G.sS), lat_bytes);
        const VD dH2(BUF ? dst : at(dst, (size_t)Lay::H20 * G.sS), lat_bytes);
        T n[3];
        normal(P, gphi, n);
        // flow set: the new bracket pi, as stored, is the reference of the
        // values this node emits and goes to its own rest slot
        const T pi_st = stored<S, T>(fl.pi, T(LG::w[0]), T(1.0 / LG::w[0]));
        {
          const Acc a = acc(own_col, zoff, pp(Lay::G0, 0), Off(0));
          dG.template st<NTW>(a.lane, a.uni, Codec<S, T>::st(fl.pi, T(1.0 / LG::w[0])));
        }
        collide_g<LG>(P, g, gphi, fl, [&](int i, T v) {
          const Tgt t = target(Lay::G0, i, LG::opp[i], LG::cx[i], LG::cy[i], LG::cz[i]);
          dG.template st<NTW>(t.lane, t.uni,
                              Codec<S, T>::st(v + kp<LG, T>(i) * (pi0 - pi_st), T(1.0 / LG::w[i])));
        });
        if (LATE) ldq(sF, Lay::F0, own_col, zoff, f);
        if constexpr (LDSC) {
          // this plane's f out of its slots, the next plane's in
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            f[i] = own[i][tid];
            own[i][tid] = nf[i];
          }
        }
        collide_f<LF>(P, f, s, n, fl, dJphi, [&](int i, T v) {
          const Tgt t = target(Lay::F0, i, LF::opp[i], LF::cx[i], LF::cy[i], LF::cz[i]);
          dF.template st<NTW>(t.lane, t.uni, rebase(i, v, r[0], R.phi));
        });
        if (LATE) {
          ldq(sH1, Lay::H10, own_col, zoff, h1);
          ldq(sH2, Lay::H20, own_col, zoff, h2);
        }
        if constexpr (LDSC) {
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            h1[i] = own[7 + i][tid];
            own[7 + i][tid] = nh1[i];
            h2[i] = own[14 + i][tid];
            own[14 + i][tid] = nh2[i];
          }
        }
        if constexpr (LOC) {
          // local scheme, Eq. (39): grad c_k from the first moment of the
          // own h_k (deviations carry the same first moment)
          T q1[3], q2[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            q1[a] = h1[1 + 2 * a] - h1[2 + 2 * a];  // D3Q7: +axis a, -axis a
            q2[a] = h2[1 + 2 * a] - h2[2 + 2 * a];
          }
          const T f1 = P.d1w * s.omphi * s.c1, f2 = P.d2w * s.phi * s.c2;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const T g1 = (s.c1 * fl.u[a] - q1[a] - T(0.5) * dJ1[a] + f1 * n[a]) * P.itc1;
            const T g2 = (s.c2 * fl.u[a] - q2[a] - T(0.5) * dJ2[a] - f2 * n[a]) * P.itc2;
            gpsi[a] = g1 + P.Keq * g2;
          }
        }
        collide_h<LF>(P, h1, h2, s, n, gphi, gpsi, fl, dJ1, dJ2, [&](int i, T a, T c) {
          const Tgt t1 = target(Lay::H10, i, LF::opp[i], LF::cx[i], LF::cy[i], LF::cz[i]);
          // (the global form reaches h1 and h2 at the same offset from their bases)
          const Tgt t2 = BUF ? target(Lay::H20, i, LF::opp[i], LF::cx[i], LF::cy[i], LF::cz[i]) : t1;
          if constexpr (!LOC) {
            dH1.template st<NTW>(t1.lane, t1.uni, rebase(i, a, r[1], R.c1));
            dH2.template st<NTW>(t2.lane, t2.uni, rebase(i, c, r[2], R.c2));
          } else {
            dH1.template st<NTW>(t1.lane, t1.uni, Codec<S, T>::st(a, T(1.0 / LF::w[i])));
            dH2.template st<NTW>(t2.lane, t2.uni, Codec<S, T>::st(c, T(1.0 / LF::w[i])));
          }
        });
      }
    }
    if (CARRY == kCarryRegs) {
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        f[i] = nf[i];
        h1[i] = nh1[i];
        h2[i] = nh2[i];
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = nr[k];
    s = ns;
  }
}

// Work-groups the device holds at once for a kernel (groups per CU x CUs),
// from the compiled resource usage; cached per kernel and device.
int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n > 0) return n;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
    n = 256;
  cache[dev].store(n, std::memory_order_relaxed);
  return n;
}

// Number of z chunks per column tile.  Every tile is one work-group, and a
// launch runs in rounds of `slots` resident groups; a last round that is
// only partly filled leaves CUs idle for a whole chunk.  Pick the chunk
// count whose tiles fill their rounds best, weighted by the two extra
// planes of moments each chunk loads at its start.
int choose_chunks(int tiles_xy, int nz, int slots) {
  int best = 1;
  double best_eff = -1.0;
  const int max_chunks = nz / 8 > 1 ? nz / 8 : 1;
  for (int c = 1; c <= max_chunks; ++c) {
    const double rounds = (double)tiles_xy * c / slots;
    const double fill = rounds / std::ceil(rounds);
    const double len = (double)nz / c;
    const double eff = fill * len / (len + 2.0);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = c;
    }
  }
  return best;
}

template <class S, class T, int TX, int TY, int NT, bool PREF, int CARRY, int WPE, int MODE,
          class Off, bool LOC, bool BUF>
hipError_t launch_variant(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                          const KParams<T>* Pdev, hipStream_t stream) {
  constexpr auto kernel = step3d_kernel<S, T, TX, TY, NT, PREF, CARRY, WPE, MODE, Off, LOC, BUF>;
  static std::atomic<int> per_cu{0};
  int groups = per_cu.load(std::memory_order_relaxed);
  if (groups < 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&groups, reinterpret_cast<const void*>(kernel),
                                                     TX * TY, 0) != hipSuccess ||
        groups < 1)
      groups = 1;
    per_cu.store(groups, std::memory_order_relaxed);
  }
  Geo3<Off> G;
  G.nx = P.nx;
  G.ny = P.ny;
  G.nz = P.nz;
  G.px = P.px;
  G.wall_x = P.wall[0];
  G.wall_y = P.wall[1];
  G.wall_z = P.wall[2];
  G.tiles_x = (P.nx + TX - 1) / TX;
  const int tiles_y = (P.ny + TY - 1) / TY;
  G.tiles_xy = G.tiles_x * tiles_y;
  G.nchunks = choose_chunks(G.tiles_xy, P.nz, groups * device_cus());
  G.ntiles = G.tiles_xy * G.nchunks;
  G.sS = Off(P.stride * (long long)sizeof(S));
  G.sT = Off(P.stride * (long long)sizeof(T));
  G.nxy = Off((long long)P.px * P.ny * (long long)sizeof(S));
  const int nblocks = ((G.ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(TX * TY), 0, stream, src, dst, hin, hout, fields,
                     (KPtr<T>)Pdev, G);
  return hipGetLastError();
}

}  // namespace

const char* step3d_variant_name(int v) {
  static const char* names[kVariants3D] = {
      "64x4 late",         "64x4 late nt-st", "32x8 late",          "64x4",
      "64x4 nt-st",        "64x4 nt-g-st",    "64x4 late nt-g-st",  "64x4 late w4",
      "64x4 lds nt-st",    "128x4 nt-st"};
  return v >= 0 && v < kVariants3D ? names[v] : "?";
}

namespace {

// the variant switch of one gradient scheme (LOC: Eq. (39))
template <class S, class T, bool LOC>
hipError_t launch_scheme(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                         const KParams<T>* Pdev, int mode, int variant, hipStream_t stream) {
  constexpr int M = kModeStep;
  using U = uint32_t;
  if (!fits_u32(LG::Q, P.stride, sizeof(S), sizeof(T), kNumFields)) {
    // very large grids: 64-bit offsets, one tile shape
    if (mode == kModeMacros)
      return launch_variant<S, T, 64, 4, 0, false, false, 1, kModeMacros, uint64_t, LOC, false>(
          src, dst, hin, hout, fields, P, Pdev, stream);
    return launch_variant<S, T, 64, 4, 0, false, true, 1, M, uint64_t, LOC, false>(
        src, dst, hin, hout, fields, P, Pdev, stream);
  }
  // Buffer addressing for FP32 / FP64 storage.  16-bit lattices keep the
  // global form: there the scalar work of the uniform offsets (a product
  // and two sums per access) costs more than the vector adds it removes
  // (1.08 against 1.04 ms per 256^3 FP16 step; FP32 1.29 against 1.32).
  constexpr bool kBuf = sizeof(S) >= 4;
  if (kBuf && !fits_buffer(Lay::QTOT, P.stride, sizeof(S), sizeof(T), kNumFields)) {
    // every set below 4 GiB but not the whole lattice: 32-bit offsets from
    // a 64-bit base per set, one tile shape
    if (mode == kModeMacros)
      return launch_variant<S, T, 64, 4, 0, false, false, 1, kModeMacros, U, LOC, false>(
          src, dst, hin, hout, fields, P, Pdev, stream);
    return launch_variant<S, T, 64, 4, 2, false, false, 1, M, U, LOC, false>(
        src, dst, hin, hout, fields, P, Pdev, stream);
  }
  // the field read-out takes the scheme's references of h1, h2 (per node for
  // the central stencil, uniform for the local scheme)
  if (mode == kModeMacros)
    return launch_variant<S, T, 64, 4, 0, false, false, 1, kModeMacros, U, LOC, kBuf>(
        src, dst, hin, hout, fields, P, Pdev, stream);
#define PFLB_V3(TX, TY, NT, PREF, LATE, WPE) \
  launch_variant<S, T, TX, TY, NT, PREF, LATE, WPE, M, U, LOC, kBuf>(src, dst, hin, hout, fields, P, Pdev, stream)
  // NT: non-temporal hints (bit 0 f / h loads, bit 1 stores, bit 2 g loads);
  // CARRY: f / h carried in registers (false), re-read before their
  // collision (true), or carried through LDS (kCarryLds); WPE: minimum
  // waves per SIMD the register allocator must allow (1: free)
  switch (variant) {
    case 1: return PFLB_V3(64, 4, 2, false, true, 1);
    case 2: return PFLB_V3(32, 8, 0, false, true, 1);
    case 3: return PFLB_V3(64, 4, 0, false, false, 1);
    case 4: return PFLB_V3(64, 4, 2, false, false, 1);
    case 5: return PFLB_V3(64, 4, 6, false, false, 1);
    case 6: return PFLB_V3(64, 4, 6, false, true, 1);
    case 7: return PFLB_V3(64, 4, 0, false, true, 4);
    case 8: return PFLB_V3(64, 4, 2, false, kCarryLds, 1);
    case 9: return PFLB_V3(128, 4, 2, false, false, 1);
    default: return PFLB_V3(64, 4, 0, false, true, 1);
  }
#undef PFLB_V3
}

}  // namespace

template <class S, class T>
hipError_t launch_step3d(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                         const KParams<T>* Pdev, int mode, int variant, hipStream_t stream) {
  if (P.local_grad)
    return launch_scheme<S, T, true>(src, dst, hin, hout, fields, P, Pdev, mode, variant, stream);
  return launch_scheme<S, T, false>(src, dst, hin, hout, fields, P, Pdev, mode, variant, stream);
}

template hipError_t launch_step3d<double, double>(const double*, double*, const double*, double*, double*,
                                                  const KParams<double>&, const KParams<double>*,
                                                  int, int, hipStream_t);
template hipError_t launch_step3d<float, float>(const float*, float*, const float*, float*, float*,
                                                const KParams<float>&, const KParams<float>*, int,
                                                int, hipStream_t);
template hipError_t launch_step3d<__half, float>(const __half*, __half*, const float*, float*, float*,
                                                 const KParams<float>&, const KParams<float>*, int,
                                                 int, hipStream_t);
template hipError_t launch_step3d<__hip_bfloat16, float>(const __hip_bfloat16*, __hip_bfloat16*,
                                                         const float*, float*, float*,
                                                         const KParams<float>&,
                                                         const KParams<float>*, int, int,
                                                         hipStream_t);

}  // namespace pflb
