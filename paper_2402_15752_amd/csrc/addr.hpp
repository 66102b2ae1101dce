// Addressing helpers shared by the step kernels.
//
// Every population set (f, g, h1, h2), the history and the field buffer is
// reached from a 64-bit set base held in scalar registers plus an Off-typed
// byte offset plane * stride + node.  With Off = uint32_t (each set below
// 4 GiB) a load or store takes the scalar-base + 32-bit-vector-offset form
// and an address costs one VGPR; Off = uint64_t serves larger sets.  The 3-D
// step reaches allocations below 4 GiB as buffers instead (View below).
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pflb {

// a uniform value the optimiser may not hoist or merge across uses
template <class X>
__device__ inline X opaque(X v) {
  asm volatile("" : "+s"(v));
  return v;
}

// the lattice constants as seen by a kernel: the constant address space
// makes every read a scalar load of memory no store of the kernel touches
template <class T>
using KPtr = const __attribute__((address_space(4))) KParams<T>*;

template <class T>
__device__ inline const KParams<T>& params(KPtr<T> p) {
  return *(const KParams<T>*)opaque(p);
}

// byte offset of plane k from a set base.  PIN (for kernels with a loop):
// formed on the scalar unit at each use, a product the compiler may neither
// hoist out of the loop -- ~40 loop-invariant offsets overflow the scalar
// file -- nor fold into a 64-bit vector multiply-add.  Without a loop the
// plain product is cheaper (no scheduling barrier per use).
template <bool PIN, class Off>
__device__ inline Off plane(int k, Off stride) {
  if constexpr (PIN)
    return k == 0 ? Off(0) : opaque(Off(k) * opaque(stride));
  else
    return Off(k) * stride;
}

// Plane skew of the population sets.  Plane i of a set is stored shifted by
// -c_ix nodes: the push store of direction i (to x + c_i) then starts a
// wave's run on the aligned address the own node x would have, and the
// one-node misalignment moves to the loads, which do not pay for it (a run
// of stores shifted by one node costs 14% (FP32) to 24% (16-bit) of the
// bandwidth on MI355X, a run of shifted loads nothing).  The padding of
// every plane (>= 64 values past the last node) absorbs the shift; plane 0
// of every set is the rest direction and is not shifted.  Every access to a
// population plane adds skew<L, S>(i): loads, push and bounce-back stores
// and the initialisation.
template <class L, class S, class Off>
__device__ constexpr Off skew(int i) {
  return L::cx[i] > 0 ? Off(0) - Off(sizeof(S)) : (L::cx[i] < 0 ? Off(sizeof(S)) : Off(0));
}

// the same in elements, for element-indexed accesses
template <class L>
__device__ constexpr long long skew_el(int i) {
  return -(long long)L::cx[i];
}

template <class P, class Off>
__device__ inline P* at(P* base, Off off) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + off);
}

// A population, history or field buffer as a kernel reaches it.  An access
// names a per-lane byte offset (`lane`: the node and its x / y push step)
// and a uniform one (`uni`: set, plane, skew, z plane and z push step).
// BUF (the whole buffer below 4 GiB): a buffer resource over the
// allocation; the address unit adds the two offsets (vector register +
// scalar register), so an access costs no vector instruction.  Otherwise a
// 64-bit base plus one Off-typed offset, lane + uni, formed per access.
template <bool BUF, class P, class Off>
struct View;

template <class P, class Off>
struct View<false, P, Off> {
  P* base;
  __device__ View(P* b, Off) : base(b) {}
  template <bool NT>
  __device__ typename std::remove_const<P>::type ld(Off lane, Off uni) const {
    return ld_pop<NT>(at(base, uni + lane));
  }
  template <bool NT>
  __device__ void st(Off lane, Off uni, P v) const {
    st_pop<NT>(at(base, uni + lane), v);
  }
};

template <class P, class Off>
struct View<true, P, Off> {
  static_assert(std::is_same<Off, uint32_t>::value, "buffer offsets are 32-bit");
  using V = typename std::remove_const<P>::type;
  // cache policy of the non-temporal accesses (the bit the compiler sets for
  // a non-temporal global load or store)
  static constexpr int kNT = 2;
  __amdgpu_buffer_rsrc_t r;
  // bytes: size of the allocation (the range every access stays in); the
  // fourth word is the raw-buffer format of this GPU family
  __device__ View(P* b, Off bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<V*>(b), (short)0, (int)bytes, 0x00020000)) {}
  template <bool NT>
  __device__ V ld(Off lane, Off uni) const {
    constexpr int aux = NT ? kNT : 0;
    if constexpr (sizeof(V) == 2)
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b16(r, (int)lane, (int)uni, aux));
    else if constexpr (sizeof(V) == 4)
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, (int)lane, (int)uni, aux));
    else
      return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane, (int)uni, aux));
  }
  template <bool NT>
  __device__ void st(Off lane, Off uni, V v) const {
    constexpr int aux = NT ? kNT : 0;
    if constexpr (sizeof(V) == 2)
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)lane, (int)uni, aux);
    else if constexpr (sizeof(V) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)lane, (int)uni, aux);
    else
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(unsigned int __attribute__((ext_vector_type(2))), v), r, (int)lane, (int)uni,
          aux);
  }
};

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

// one set of Q populations of the node at byte offset `node` of a set base
template <class L, bool NTS, bool PIN, class S, class T, class Off>
__device__ inline void load_q(const S* __restrict__ base, Off sS, Off node, T (&x)[L::Q]) {
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    x[i] = Codec<S, T>::ld(ld_pop<NTS>(at(base, plane<PIN>(i, sS) + node + skew<L, S, Off>(i))),
                           T(L::w[i]));
}

// Push deltas of one lane (bytes, modular arithmetic in Off) and its
// bounce-back bits: bit 0 x-, 1 x+, 2 y-, 3 y+ (4 z-, 5 z+ are per plane).
// A periodic axis wraps to the far side; a walled axis sets the bit and the
// link bounces back into the opposite slot of the own node.
template <class Off>
struct PushXY {
  Off dxm, dxp, dym, dyp;
  int bits;
  __device__ PushXY(int x, int y, int nx, int ny, int px, int wall_x, int wall_y, Off bs) {
    const Off row = Off(px) * bs;  // rows are px nodes apart
    dxm = Off(0) - bs;
    dxp = bs;
    dym = Off(0) - row;
    dyp = row;
    bits = 0;
    if (x == 0) {
      if (wall_x) bits |= 1;
      dxm = Off(nx - 1) * bs;
    }
    if (x == nx - 1) {
      if (wall_x) bits |= 2;
      dxp = Off(0) - Off(nx - 1) * bs;
    }
    if (y == 0) {
      if (wall_y) bits |= 4;
      dym = Off(ny - 1) * row;
    }
    if (y == ny - 1) {
      if (wall_y) bits |= 8;
      dyp = Off(0) - Off(ny - 1) * row;
    }
  }
};

// bounce-back mask of direction (cx, cy, cz)
__device__ constexpr int link_mask(int cx, int cy, int cz) {
  return (cx < 0 ? 1 : 0) | (cx > 0 ? 2 : 0) | (cy < 0 ? 4 : 0) | (cy > 0 ? 8 : 0) |
         (cz < 0 ? 16 : 0) | (cz > 0 ? 32 : 0);
}

// true when the whole lattice (qtot planes), the history and the field
// buffer each span < 4 GiB: one buffer resource and 32-bit offsets reach
// every value of each
inline bool fits_buffer(int qtot, long long stride, size_t s_pop, size_t s_cmp, int nfields) {
  const unsigned long long lim = (1ull << 32) - 1;
  return (unsigned long long)qtot * stride * s_pop < lim &&
         (unsigned long long)nfields * stride * s_cmp < lim;
}

// true when every population set (at most qset planes), the history and the
// field buffer span < 4 GiB, so 32-bit byte offsets reach every value
inline bool fits_u32(int qset, long long stride, size_t s_pop, size_t s_cmp, int nfields) {
  const unsigned long long lim = 1ull << 32;
  return (unsigned long long)qset * stride * s_pop < lim &&
         (unsigned long long)nfields * stride * s_cmp < lim;
}

}  // namespace pflb
