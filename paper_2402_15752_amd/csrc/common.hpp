// Per-node arithmetic of the coupled phase-field LB step, shared by the 2-D
// and 3-D kernels.  Everything here works on values held in registers; the
// kernels own loads, stencils and streaming.
//
// Notation follows the paper: phi (order parameter), c1, c2 (two-scalar
// concentrations), psi = c1 + Keq c2, D_m (mixed diffusivity), mu_phi
// (chemical potential), F (total force), p, u, rho, mu.
//
// Deviation form.  The f, h1, h2 populations are held, stored and streamed
// as deviations from a reference, dX_i = X_i - w_i R.  The reference of the
// populations that arrive at a node is that node's own moment of the
// previous time level -- phi, c1, c2 as the time-derivative history keeps
// them -- so the stored values are the change of a population over one
// step plus its flux part: small numbers, resolved well by FP32 and even by
// 16-bit storage, and their sum is the change of the moment (phi = R +
// sum dX_i), which keeps the conserved sums accurate.  A node writing
// population i to its neighbour y = x + c_i stores X_i* - w_i R(y), with
// R(y) the neighbour's moment at this level (the stencils already hold it);
// the reader at y adds back w_i R(y) from its history.  The scalar sets of
// the one-scalar model and of the local gradient scheme, which have no
// scalar halo, keep a uniform reference (c1_ref, c2_ref).  g is held
// relative to a per-node pressure bracket carried in its rest slot (see
// Flow below).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace pflb {

// Constants of one lattice, precomputed on the host in FP64 and rounded
// once to the compute type T.
template <class T>
struct KParams {
  int nx, ny, nz;
  int px;             // row pitch of the planes (nodes)
  int wall[3];        // 1: half-way bounce-back walls on both faces of the axis
  long long stride;   // elements between two population / field planes
  // relaxation of the constant-tau sets as delta = 2 - 1/tau = 2 (tau - 1/2)/tau
  // and delta/2 = 1 - 1/(2 tau): accurate even when tau is close to 1/2
  T del_f, hdel_f, del_h1, hdel_h1, del_h2, hdel_h2;
  T beta4, kappa;     // 4 beta and k of the chemical potential
  T rho1, rho2, drho, rho_ref;
  T grav[3];
  T mu1, mu2, ln_mu1, ln_mu2;
  int visc_exp;       // 1: exponential law, Eq. (4.3); 0: linear law, Eq. (1.8)
  T D1D2, KD1, D2, Keq, A, half_A;
  T four_over_W;
  T neps2;            // n_eps^2 of the regularised normal
  T ref_c1, ref_c2;   // uniform reference of h1, h2 where they have no per-node one
  int href;           // 1: h1, h2 stored relative to the node's own c1, c2 (two-scalar,
                      // central stencil); 0: relative to ref_c1, ref_c2
  int one_scalar;     // 1: one-scalar model, h3 in the h1 planes (Sec. III D)
  T D1K;              // D1 Keq of D_eff = D1 Keq phi + D2 (1 - phi)
  int dirichlet;      // bit f: face f (x-, x+, y-, y+) holds Dirichlet c1, c2
  T cw[4][2];         // (c1, c2) imposed at each face
  int local_grad;     // 1: grad c_k from the moments of h_k (Eq. (39))
  T itc1, itc2;       // 1 / (tau_hk cs^2)
  T d1w, d2w;         // 4 D_k / W
  int local_phase;    // 1: grad phi by the local scheme after Eq. (39)
  T itf;              // 1 / (tau_f cs^2)
  T ec2;              // (tau_f cs^2 n_eps)^2
  T mw;               // 4 M / W
};

// ------------------------------------------------------------ storage codec
//
// FP64 and FP32 lattices store the deviation dX_i itself.  16-bit lattices
// store dX_i / w_i, so that every direction has the same relative precision.

template <class S, class T>
struct Codec;

template <>
struct Codec<double, double> {
  __device__ static double ld(double s, double) { return s; }
  __device__ static double st(double x, double) { return x; }
};

template <>
struct Codec<float, float> {
  __device__ static float ld(float s, float) { return s; }
  __device__ static float st(float x, float) { return x; }
};

template <>
struct Codec<__half, float> {
  // w x as one fma with the FP16 operand read in place (v_fma_mix_f32)
  __device__ static float ld(__half s, float w) { return __builtin_fmaf(w, __half2float(s), 0.0f); }
  __device__ static __half st(float x, float inv_w) { return __float2half_rn(x * inv_w); }
};

template <>
struct Codec<__hip_bfloat16, float> {
  __device__ static float ld(__hip_bfloat16 s, float w) { return w * __bfloat162float(s); }
  __device__ static __hip_bfloat16 st(float x, float inv_w) { return __float2bfloat16(x * inv_w); }
};

// x + w d stored: for FP64 and FP32 storage exactly that sum; 16-bit storage
// keeps (x + w d) / w and forms it as x / w + d, one fused operation
template <class S, class T>
__device__ inline S store_shifted(T x, T d, T w, T inv_w) {
  return Codec<S, T>::st(x + w * d, inv_w);
}
template <>
__device__ inline __half store_shifted<__half, float>(float x, float d, float, float inv_w) {
  return __float2half_rn(__builtin_fmaf(x, inv_w, d));
}
template <>
__device__ inline __hip_bfloat16 store_shifted<__hip_bfloat16, float>(float x, float d, float,
                                                                      float inv_w) {
  return __float2bfloat16(__builtin_fmaf(x, inv_w, d));
}

// the value a population of weight w stored as x reads back as (x itself
// for FP64 and FP32 storage)
template <class S, class T>
__device__ inline T stored(T x, T w, T inv_w) {
  return Codec<S, T>::ld(Codec<S, T>::st(x, inv_w), w);
}

// --------------------------------------------------------------- helpers

// Quotient, reciprocal square root and exponential of the per-node formulas.
// FP64 keeps the correctly rounded forms.  In FP32 they are the hardware's
// one-ulp instructions (v_rcp_f32, v_rsq_f32, v_exp_f32 of x log2 e): a
// correctly rounded FP32 division expands into 12 instructions and expf
// into 17, and the step with 16-bit storage is bound by instruction issue
// about as much as by HBM.
__device__ inline double div_t(double a, double b) { return a / b; }
__device__ inline float div_t(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double rsqrt_t(double x) { return 1.0 / sqrt(x); }
__device__ inline float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double exp_t(double x) { return exp(x); }
__device__ inline float exp_t(float x) { return __expf(x); }

template <class T>
__device__ inline bool finite_t(T x) {
  return x == x && x - x == T(0);
}

// c_i . v over the nonzero components of direction i only.  The lattice
// components are 0 or +-1 and i is a constant after unrolling, so this is
// one to three adds; written as the full sum, the 0 * v terms could not be
// dropped by the compiler (0 * inf is not 0) and would cost an FMA each.
template <class L, class T>
__device__ inline T cdot(int i, const T (&v)[3]) {
  T r = T(0);
  bool have = false;
  auto add = [&](int c, T x) {
    if (!c) return;
    const T t = c > 0 ? x : -x;
    r = have ? r + t : t;
    have = true;
  };
  add(L::cx[i], v[0]);
  add(L::cy[i], v[1]);
  add(L::cz[i], v[2]);
  return r;
}

// Macroscopic state of one node at the current time level.
template <class T>
struct Node {
  T dphi, phi, omphi;  // phi - phi_ref, phi, 1 - phi
  T dc1, dc2, c1, c2;  // c_k - c_k,ref and c_k
  T Dm;                // mixed diffusivity (one-scalar model: D_eff)
  T c, dc, ct;         // one-scalar model: c, c - c_ref, c / K_eff
};

// --------------------------------------------------- moments and recovery
//
// phi = sum f_i; S_k = sum h_k,i; D_m = D1 D2 / (Keq D1 (1-phi) + D2 phi)
// (Sec. II C).  The implicit recovery c1 = S1 + a e, c2 = S2 - a e with
// a = A D_m / 2 and e = Keq c2 phi - c1 (1-phi) (Sec. III C) is linear; its
// exact solution is e = (Keq phi S2 - (1-phi) S1) / (1 + a (Keq phi + 1 - phi)).
// rphi, rc1, rc2: the references of the node's stored f, h1, h2.

// phi of a node from its stored f: the same additions, in the same order,
// wherever a kernel needs it (own node, halo node, field read-out), so that
// every copy of a node's phi is bitwise the value its history keeps
template <class LF, class T>
__device__ inline T phase_sum(const T (&df)[LF::Q]) {
  T s0 = df[0];
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) s0 += df[i];
  return s0;
}

template <class LF, class T>
__device__ inline void moments(const KParams<T>& P, const T (&df)[LF::Q], const T (&dh1)[LF::Q],
                               const T (&dh2)[LF::Q], T rphi, T rc1, T rc2, Node<T>& s) {
  const T s0 = phase_sum<LF>(df);
  T s1 = dh1[0], s2 = dh2[0];
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) {
    s1 += dh1[i];
    s2 += dh2[i];
  }
  s.dphi = s0;
  s.phi = rphi + s0;
  s.omphi = (T(1) - rphi) - s0;
  s.Dm = div_t(P.D1D2, P.KD1 * s.omphi + P.D2 * s.phi);
  const T a = P.half_A * s.Dm;
  const T S1 = rc1 + s1, S2 = rc2 + s2;
  const T Kphi = P.Keq * s.phi;
  const T e = div_t(Kphi * S2 - s.omphi * S1, T(1) + a * (Kphi + s.omphi));
  s.dc1 = s1 + a * e;
  s.dc2 = s2 - a * e;
  s.c1 = rc1 + s.dc1;
  s.c2 = rc2 + s.dc2;
}

// grad phi by the local scheme after Eq. (39) (Sec. III C): with
// C = sum c_i f_i - phi u + d_t(phi u) / 2, D = -tau_f cs^2 and
// B = 4 M phi (1 - phi) / W, |grad phi| = (-|C| - B) / D and
// grad phi = C / (D + B / |grad phi|) = -(|C| + B) C / (tau_f cs^2 |C|),
// the last form free of the cancellation in D + B / |grad phi| where
// |C| << B.  Its direction C / |C| is undefined where C vanishes (at an
// equilibrium start C is round-off everywhere), so |C| in the denominator is
// regularised as sqrt(|C|^2 + ec^2), ec = tau_f cs^2 n_eps, the scale of C
// at a gradient of n_eps.  u is the previous level's, uo (this level's needs
// grad phi through the force), d_t(phi u) = (phi - phi_old) uo.  The stored
// deviations df carry the first moment of f (their references have none).
template <class LF, class T>
__device__ inline void local_grad_phi(const KParams<T>& P, const T (&df)[LF::Q], T phi,
                                      const T (&uo)[3], T phi_old, T (&gphi)[3]) {
  const T k = T(0.5) * (phi - phi_old) - phi;
  T C[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) C[a] = k * uo[a];
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) {
    if (LF::cx[i]) C[0] += LF::cx[i] > 0 ? df[i] : -df[i];
    if (LF::cy[i]) C[1] += LF::cy[i] > 0 ? df[i] : -df[i];
    if (LF::cz[i]) C[2] += LF::cz[i] > 0 ? df[i] : -df[i];
  }
  const T cn2 = C[0] * C[0] + C[1] * C[1] + C[2] * C[2];
  const T B = P.mw * phi * (T(1) - phi);
  const T fac = -(sqrt(cn2) + B) * P.itf * rsqrt_t(cn2 + P.ec2);
#pragma unroll
  for (int a = 0; a < 3; ++a) gphi[a] = fac * C[a];
}

// One-scalar model (Sec. II D, III D): c = sum h3_i; the phase parts of c at
// interfacial equilibrium (c~1 = Keq c~2, c = c~1 phi + c~2 (1 - phi)) give
// c~2 = c / K_eff, c1 = Keq phi c~2, c2 = (1 - phi) c~2 with
// K_eff = Keq phi + 1 - phi; D_eff = D1 Keq phi + D2 (1 - phi) goes to Dm.
template <class LF, class T>
__device__ inline void moments_one(const KParams<T>& P, const T (&df)[LF::Q],
                                   const T (&dh3)[LF::Q], T rphi, Node<T>& s) {
  const T s0 = phase_sum<LF>(df);
  T s1 = dh3[0];
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) s1 += dh3[i];
  s.dphi = s0;
  s.phi = rphi + s0;
  s.omphi = (T(1) - rphi) - s0;
  s.dc = s1;
  s.c = P.ref_c1 + s1;
  s.ct = div_t(s.c, P.Keq * s.phi + s.omphi);
  s.c1 = P.Keq * s.phi * s.ct;
  s.c2 = s.omphi * s.ct;
  s.dc1 = s.c1 - P.ref_c1;
  s.dc2 = s.c2 - P.ref_c2;
  s.Dm = P.D1K * s.phi + P.D2 * s.omphi;
}

// ---------------------------------------------------------- flow macros
//
// rho = phi (rho1 - rho2) + rho2; F = mu_phi grad phi + (rho - rho_ref) g;
// u = (sum c_i g_i + F/2) / rho;
// p = cs^2/(1-w0) [sum_{i!=0} g_i + (rho1-rho2) u.grad phi / 2 + rho s_0(u)];
// mu from Eq. (4.3) or Eq. (1.8)   (Sec. II B, III B)
template <class T>
struct Flow {
  T u[3];
  T F[3];
  T pi;     // bracket of the pressure formula: p = cs^2 / (1 - w0) * pi
  T dpi;    // its change from the node's reference pi0
  T j[3];   // momentum rho u = sum c_i g_i + F / 2
  T p, rho, mu, mu_phi;
  T inv_rho;  // 1 / rho
};

// The flow populations are held relative to the pressure part of the
// equilibrium, d_i = g_i - v_i pi0 (i > 0, v_i = w_i / (1 - w0)), with pi0
// the node's pressure bracket of the previous level: the pressure, the
// largest part of every g_i, then enters the sums and the collision only as
// the small change pi - pi0, and FP32 rounding stays relative to the flow
// itself.  The rest population g_0 takes no part in the method (the
// pressure sums i > 0, the momentum has c_0 = 0), so its slot carries pi0.
// sum_{i>0} v_i = 1 and sum_i v_i c_i = 0 hold exactly for the weights kp
// below, so sum_{i>0} g_i = pi0 + sum d_i and sum c_i g_i = sum c_i d_i.
template <class LG, class T>
__device__ inline void flow_macros(const KParams<T>& P, const T (&g)[LG::Q], const Node<T>& s,
                                   const T (&gphi)[3], T lap, T pi0, Flow<T>& fl) {
  constexpr T cs2 = T(LG::cs2);
  // 4 beta phi (phi-1)(phi-1/2) - k lap phi
  fl.mu_phi = -P.beta4 * s.phi * s.omphi * (s.phi - T(0.5)) - P.kappa * lap;
  fl.rho = s.phi * P.drho + P.rho2;
  const T buoy = fl.rho - P.rho_ref;
  T m[3] = {0, 0, 0};
  T sg = 0;
#pragma unroll
  for (int i = 1; i < LG::Q; ++i) {
    sg += g[i];
    if (LG::cx[i]) m[0] += T(LG::cx[i]) * g[i];
    if (LG::cy[i]) m[1] += T(LG::cy[i]) * g[i];
    if (LG::cz[i]) m[2] += T(LG::cz[i]) * g[i];
  }
  const T inv_rho = div_t(T(1), fl.rho);
  fl.inv_rho = inv_rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    fl.F[a] = fl.mu_phi * gphi[a] + buoy * P.grav[a];
    fl.j[a] = m[a] + T(0.5) * fl.F[a];
    fl.u[a] = fl.j[a] * inv_rho;
  }
  const T uu = fl.u[0] * fl.u[0] + fl.u[1] * fl.u[1] + fl.u[2] * fl.u[2];
  const T udg = fl.u[0] * gphi[0] + fl.u[1] * gphi[1] + fl.u[2] * gphi[2];
  const T s0 = T(LG::w[0]) * (-uu * T(0.5 / LG::cs2));
  fl.dpi = sg + T(0.5) * P.drho * udg + fl.rho * s0;
  fl.pi = pi0 + fl.dpi;
  fl.p = T(cs2 / (1.0 - LG::w[0])) * fl.pi;
  if (P.visc_exp)
    fl.mu = exp_t(s.c1 * P.ln_mu1 + s.c2 * P.ln_mu2);
  else
    fl.mu = s.phi * (P.mu1 - P.mu2) + P.mu2;
}

// ------------------------------------------------------------- collision
//
// SRT collision of the four sets at one node (Sec. III A-C):
//   X_i* = X_i - (X_i - X_i^eq)/tau + (1 - 1/(2 tau)) S_i  [+ ~H_i for h1, h2]
// with the equilibria, source terms F_i, G_i, H_k,i and ~H_k,i of the paper,
// written on the deviations df, dh1, dh2 (g as is).  Arrays are overwritten
// with the post-collision values.
//
// The same algebra is arranged so that rounding carries no bias into the
// moments the method conserves or relaxes slowly:
//  - with neq = X - X^eq and delta = 2 - 1/tau,
//      X* = (X^eq - neq) + delta neq + (delta/2) S,
//    so tau - 1/2 (hence M, D_k, nu) enters through delta, stored to full
//    relative precision, instead of through 1 - 1/tau;
//  - the rest-direction equilibrium closes the zeroth moment exactly
//    (X_0^eq = X - sum_{i>0} X_i^eq), so rounded weights cannot create or
//    destroy phase, solute or pressure;
//  - first-moment terms use K_i ~ w_i/cs^2 chosen so that
//    sum_i K_i c_ix^2 = 1 holds exactly in the compute type, so the momentum
//    of g^eq is rho u without a rounded-weight factor.

// Per-direction first-moment constant K_i ~ w_i / cs^2 of lattice L in type
// T: the axis value rounded once, the other directions carrying c_x != 0
// completing sum_i K_i c_ix^2 = 1 exactly.
template <class L, class T>
__device__ constexpr T kw(int i) {
  constexpr T k_axis = T(L::w[1] / L::cs2);
  constexpr int n_diag = L::Q == 9 ? 4 : (L::Q == 19 ? 8 : 0);
  if (i == 0) return T(0);
  const int nnz = (L::cx[i] != 0) + (L::cy[i] != 0) + (L::cz[i] != 0);
  if (nnz == 1) return k_axis;
  return (T(1) - T(2) * k_axis) / T(n_diag);
}

// Pressure weights v_i = w_i / (1 - w0) (i > 0) of lattice L in type T,
// completed so that sum_{i>0} v_i = 1 holds exactly.  With
// p = cs^2/(1-w0) Pi (Sec. III B) the pressure part of g_i^eq is
// p w_i / cs^2 = v_i Pi, which sums back to Pi with no rounded-weight factor.
template <class L, class T>
__device__ constexpr T kp(int i) {
  constexpr T v_axis = T(L::w[1] / (1.0 - L::w[0]));
  constexpr int n_axis = 2 * L::D;
  constexpr int n_other = L::Q - 1 - n_axis;
  if (i == 0) return T(0);
  const int nnz = (L::cx[i] != 0) + (L::cy[i] != 0) + (L::cz[i] != 0);
  if (nnz == 1 || n_other == 0) return v_axis;
  return (T(1) - T(n_axis) * v_axis) / T(n_other);
}

// regularised unit normal n = grad phi / sqrt(|grad phi|^2 + n_eps^2)
template <class T>
__device__ inline void normal(const KParams<T>& P, const T (&gphi)[3], T (&n)[3]) {
  const T gg = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
  const T rn = rsqrt_t(gg + P.neps2);
  n[0] = gphi[0] * rn;
  n[1] = gphi[1] * rn;
  n[2] = gphi[2] * rn;
}

// True for the direction of each opposite pair whose first nonzero
// component is positive.
template <class L>
__device__ constexpr bool first_of_pair(int i) {
  return L::cx[i] > 0 || (L::cx[i] == 0 && (L::cy[i] > 0 || (L::cy[i] == 0 && L::cz[i] > 0)));
}

// Isotropic central gradient (Sec. III C) on the weights of lattice L,
// grad v = sum_i w_i c_i v(x + c_i) / cs^2, summed over opposite pairs as
// w_i c_i (v(x + c_i) - v(x - c_i)) / cs^2: the difference of two nearby
// values is formed first, so the sum is taken of small numbers.  v(i) reads
// the value at x + c_i.
template <class L, class T, class V>
__device__ inline void grad_pairs(V&& v, T (&g)[3]) {
  g[0] = g[1] = g[2] = T(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (!first_of_pair<L>(i)) continue;
    const T d = v(i) - v(L::opp[i]);
    const T wc = T(L::w[i] / L::cs2);
    if (L::cx[i]) g[0] += L::cx[i] > 0 ? wc * d : -(wc * d);
    if (L::cy[i]) g[1] += L::cy[i] > 0 ? wc * d : -(wc * d);
    if (L::cz[i]) g[2] += L::cz[i] > 0 ? wc * d : -(wc * d);
  }
}

// isotropic Laplacian sum_i 2 w_i (v(x + c_i) - v(x)) / cs^2 (Sec. III C)
template <class L, class T, class V>
__device__ inline T lap_of(V&& v, T v0) {
  T lap = T(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) lap += T(2.0 * L::w[i] / L::cs2) * (v(i) - v0);
  return lap;
}

template <class T>
__device__ inline T relax(T x, T xeq, T del, T hdel, T src) {
  const T neq = x - xeq;
  return del * neq + (xeq - neq) + hdel * src;
}

// The collisions below hand each post-collision population to emit(i, X_i*)
// as soon as it is formed, so a kernel can stream it out at once and keep
// few values live.  The rest-direction equilibrium needs the sum of the
// others; that sum is formed in a first, cheap pass instead of holding all
// equilibria in registers.

// phase field: f^eq = w phi (1 + c.u/cs^2), F_i = w [c.d_t(phi u)/cs^2 + c.n 4 phi (1-phi)/W]
template <class LF, class T, class Emit>
__device__ inline void collide_f(const KParams<T>& P, const T (&df)[LF::Q], const Node<T>& s,
                                 const T (&n)[3], const Flow<T>& fl, const T (&dJphi)[3],
                                 Emit&& emit) {
  const T sharp = P.four_over_W * s.phi * s.omphi;
  auto eq = [&](int i) {
    const T cu = cdot<LF>(i, fl.u);
    return T(LF::w[i]) * s.dphi + kw<LF, T>(i) * s.phi * cu;
  };
  T rest = s.dphi;
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) rest -= eq(i);
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    const T cn = cdot<LF>(i, n);
    const T cj = cdot<LF>(i, dJphi);
    const T Fi = i == 0 ? T(0) : kw<LF, T>(i) * cj + T(LF::w[i]) * cn * sharp;
    emit(i, relax(df[i], i == 0 ? rest : eq(i), P.del_f, P.hdel_f, Fi));
  }
}

// flow: g^eq = p/cs^2 (w_i - delta_i0) + rho s_i(u),
//       G_i = w [c.F/cs^2 + (rho1-rho2)(c.u)(c.grad phi)/cs^2], tau_g = 1/2 + mu/(rho cs^2)
// on d_i = g_i - v_i pi0 (see Flow): d_i^eq = v_i (pi - pi0) + rho s_i; the
// emitted values are g_i* - v_i pi0, i > 0 (the rest direction is not a
// population of the method's output: its slot holds the new pi).
template <class LG, class T, class Emit>
__device__ inline void collide_g(const KParams<T>& P, const T (&g)[LG::Q], const T (&gphi)[3],
                                 const Flow<T>& fl, Emit&& emit) {
  constexpr T inv_csg = T(1.0 / LG::cs2);
  constexpr T half_inv_csg2 = T(0.5 / (LG::cs2 * LG::cs2));
  const T nu = fl.mu * inv_csg * fl.inv_rho;  // tau_g - 1/2
  const T tau_g = T(0.5) + nu;
  const T del_g = div_t(T(2) * nu, tau_g);
  const T hdel_g = T(0.5) * del_g;
  const T uu = fl.u[0] * fl.u[0] + fl.u[1] * fl.u[1] + fl.u[2] * fl.u[2];
  const T iso = uu * T(0.5) * inv_csg;
  // p/cs^2 w_i = v_i pi with pi the bracket of the pressure formula; the
  // first-moment term w_i rho c_i.u / cs^2 is formed from the momentum
  // j = rho u itself, not from rho times the rounded u, so that the
  // collision hands the populations their momentum back without the
  // rounding of u (a bias that otherwise recurs every step)
  // Opposite links share every term: c.u, c.F, c.grad phi and c.j change
  // sign, so the even part of the equilibrium (pressure and second-order
  // terms) is formed once per pair and the odd ones enter with both signs,
  // in expressions of the same shape -- the same roundings (and fused
  // multiply-adds) the two links would get one by one.
#pragma unroll
  for (int i = 1; i < LG::Q; ++i) {
    if (!first_of_pair<LG>(i)) continue;
    const int o = LG::opp[i];
    const T cu = cdot<LG>(i, fl.u);
    const T cF = cdot<LG>(i, fl.F);
    const T cg = cdot<LG>(i, gphi);
    const T cj = cdot<LG>(i, fl.j);
    const T even = kp<LG, T>(i) * fl.dpi + T(LG::w[i]) * fl.rho * (cu * cu * half_inv_csg2 - iso);
    const T dcu = P.drho * cu;
    emit(i, relax(g[i], even + kw<LG, T>(i) * cj, del_g, hdel_g, kw<LG, T>(i) * (cF + dcu * cg)));
    emit(o, relax(g[o], even - kw<LG, T>(i) * cj, del_g, hdel_g, kw<LG, T>(i) * (dcu * cg - cF)));
  }
}

// two-scalar sets: h_k^eq = w c_k (1 + c.u/cs^2),
//   H_1 = w [c.d_t(c1 u)/cs^2 + c.n 4 (1-phi) c1/W + A D_m (Keq c2 phi - c1 (1-phi))],
//   H_2 = w [c.d_t(c2 u)/cs^2 - c.n 4 phi c2/W + A D_m (c1 (1-phi) - Keq c2 phi)],
//   ~H_1 = -w D_m grad phi . grad psi = -~H_2
// `xs1`, `xs2` are per-node corrections of c1 and c2 per step: the learned
// closure's on a coarse grid, 0 otherwise.  They are carried the same way as
// ~H (h_k loses w_i s_k), with (s1, s2) = J^-1 (xs1, xs2) and J the Jacobian
// of the implicit recovery (c1, c2) = R(S1, S2) (Sec. III C, see moments):
//   s1 = (1 + a (1 - phi)) xs1 - a Keq phi xs2,
//   s2 = -a (1 - phi) xs1 + (1 + a Keq phi) xs2,   a = A D_m / 2,
// so that the recovered c_k is lowered by xs_k (exactly where phi and D_m do
// not change over the step), not by the part of it that the exchange in the
// recovery leaves (s1 + s2 = xs1 + xs2).
template <class LF, class T, class Emit>
__device__ inline void collide_h(const KParams<T>& P, const T (&dh1)[LF::Q], const T (&dh2)[LF::Q],
                                 const Node<T>& s, const T (&n)[3], const T (&gphi)[3],
                                 const T (&gpsi)[3], const Flow<T>& fl, const T (&dJ1)[3],
                                 const T (&dJ2)[3], Emit&& emit, T xs1 = T(0), T xs2 = T(0)) {
  const T M1 = P.A * s.Dm * (P.Keq * s.c2 * s.phi - s.c1 * s.omphi);
  const T aux = s.Dm * (gphi[0] * gpsi[0] + gphi[1] * gpsi[1] + gphi[2] * gpsi[2]);
  const T ra = P.half_A * s.Dm, ra1 = ra * s.omphi, ra2 = ra * (P.Keq * s.phi);
  const T cs1 = xs1 + (ra1 * xs1 - ra2 * xs2), cs2 = xs2 + (ra2 * xs2 - ra1 * xs1);
  const T aux1 = aux + cs1, aux2 = aux - cs2;
  const T fl1 = P.four_over_W * s.omphi * s.c1;
  const T fl2 = P.four_over_W * s.phi * s.c2;
  auto cu_of = [&](int i) {
    return cdot<LF>(i, fl.u);
  };
  T r1 = s.dc1, r2 = s.dc2;
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) {
    const T cu = cu_of(i);
    r1 -= T(LF::w[i]) * s.dc1 + kw<LF, T>(i) * s.c1 * cu;
    r2 -= T(LF::w[i]) * s.dc2 + kw<LF, T>(i) * s.c2 * cu;
  }
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    const T w = T(LF::w[i]);
    const T cu = cu_of(i);
    const T e1 = i == 0 ? r1 : w * s.dc1 + kw<LF, T>(i) * s.c1 * cu;
    const T e2 = i == 0 ? r2 : w * s.dc2 + kw<LF, T>(i) * s.c2 * cu;
    const T cn = cdot<LF>(i, n);
    const T cj1 = cdot<LF>(i, dJ1);
    const T cj2 = cdot<LF>(i, dJ2);
    const T k = kw<LF, T>(i);
    const T H1 = k * cj1 + w * (cn * fl1 + M1);
    const T H2 = k * cj2 - w * (cn * fl2 + M1);
    emit(i, relax(dh1[i], e1, P.del_h1, P.hdel_h1, H1) - w * aux1,
         relax(dh2[i], e2, P.del_h2, P.hdel_h2, H2) + w * aux2);
  }
}

// one-scalar set (Sec. III D): h3_0^eq = c + (w0 - 1) c / K_eff,
//   h3_i^eq = w_i c / K_eff + w_i c_i.(c u) / cs^2, H3_i = w_i c_i.d_t(c u) / cs^2,
//   tau_h3 = 1/2 + D_eff / cs^2 per node.  On the deviations dh3_i = h3_i - w_i c_ref
//   the rest direction closes the zeroth moment as for the other sets.
template <class LF, class T, class Emit>
__device__ inline void collide_h3(const KParams<T>& P, const T (&dh3)[LF::Q], const Node<T>& s,
                                  const Flow<T>& fl, const T (&dJ)[3], Emit&& emit) {
  const T nu = s.Dm * T(1.0 / LF::cs2);  // tau_h3 - 1/2
  const T del = div_t(T(2) * nu, T(0.5) + nu);
  const T hdel = T(0.5) * del;
  const T dct = s.ct - P.ref_c1;
  auto eq = [&](int i) {
    return T(LF::w[i]) * dct + kw<LF, T>(i) * s.c * cdot<LF>(i, fl.u);
  };
  T rest = s.dc;
#pragma unroll
  for (int i = 1; i < LF::Q; ++i) rest -= eq(i);
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    const T H = i == 0 ? T(0) : kw<LF, T>(i) * cdot<LF>(i, dJ);
    emit(i, relax(dh3[i], i == 0 ? rest : eq(i), del, hdel, H));
  }
}

// All four sets at one node, post-collision values handed to the emitters.
template <class LF, class LG, class T, class EF, class EG, class EH>
__device__ inline void collide(const KParams<T>& P, const T (&df)[LF::Q], const T (&g)[LG::Q],
                               const T (&dh1)[LF::Q], const T (&dh2)[LF::Q], const Node<T>& s,
                               const T (&gphi)[3], const T (&gpsi)[3], const Flow<T>& fl,
                               const T (&dJphi)[3], const T (&dJ1)[3], const T (&dJ2)[3],
                               EF&& emit_f, EG&& emit_g, EH&& emit_h, T xs1 = T(0),
                               T xs2 = T(0)) {
  T n[3];
  normal(P, gphi, n);
  collide_g<LG>(P, g, gphi, fl, emit_g);
  collide_f<LF>(P, df, s, n, fl, dJphi, emit_f);
  collide_h<LF>(P, dh1, dh2, s, n, gphi, gpsi, fl, dJ1, dJ2, emit_h, xs1, xs2);
}

// ------------------------------------------------------------- equilibria
// Equilibrium populations of the initial fields, as deviations from the
// node's own references (init only): the node's initial phi and, with
// per-node scalar references, its initial c1, c2.
template <class LF, class LG, class T>
__device__ inline void equilibria(const KParams<T>& P, T phi, T c1, T c2, const T (&u)[3], T p,
                                  T (&df)[LF::Q], T (&g)[LG::Q], T (&dh1)[LF::Q],
                                  T (&dh2)[LF::Q]) {
  const T rc1 = P.href ? c1 : P.ref_c1, rc2 = P.href ? c2 : P.ref_c2;
  constexpr T inv_csf = T(1.0 / LF::cs2);
  constexpr T inv_csg = T(1.0 / LG::cs2);
  constexpr T half_inv_csg2 = T(0.5 / (LG::cs2 * LG::cs2));
  const T rho = phi * P.drho + P.rho2;
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T dphi = T(0), dc1 = c1 - rc1, dc2 = c2 - rc2;
  // one-scalar model: h3 (in the h1 slot) of c = c1 + c2, h2 = 0
  const T c = c1 + c2;
  const T dct = c / (P.Keq * phi + (T(1) - phi)) - P.ref_c1;
  T rest3 = c - P.ref_c1;
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    const T cu = cdot<LF>(i, u);
    df[i] = T(LF::w[i]) * (dphi + phi * cu * inv_csf);
    if (P.one_scalar) {
      dh1[i] = T(LF::w[i]) * (dct + c * cu * inv_csf);
      dh2[i] = T(0);
      if (i > 0) rest3 -= dh1[i];
    } else {
      dh1[i] = T(LF::w[i]) * (dc1 + c1 * cu * inv_csf);
      dh2[i] = T(LF::w[i]) * (dc2 + c2 * cu * inv_csf);
    }
  }
  if (P.one_scalar) dh1[0] = rest3;
  // flow set relative to the pressure part of its equilibrium (see Flow):
  // d_i = rho s_i(u), and the rest slot holds pi = (1 - w0) p / cs^2
  g[0] = p * T((1.0 - LG::w[0]) / LG::cs2);
#pragma unroll
  for (int i = 1; i < LG::Q; ++i) {
    const T cu = cdot<LG>(i, u);
    g[i] = rho * (T(LG::w[i]) * (cu * inv_csg + cu * cu * half_inv_csg2 - uu * T(0.5) * inv_csg));
  }
}

// ------------------------------------------------- population load / store
//
// NTS selects non-temporal loads and stores for the population streams:
// each value is read once and written once per step, so they need not
// displace the halo and history lines in the caches.

template <bool NTS, class S>
__device__ inline S ld_pop(const S* p) {
  if constexpr (!NTS) {
    return *p;
  } else if constexpr (sizeof(S) == 2) {
    return __builtin_bit_cast(S, __builtin_nontemporal_load((const unsigned short*)p));
  } else {
    return __builtin_nontemporal_load(p);
  }
}

template <bool NTS, class S>
__device__ inline void st_pop(S* p, S v) {
  if constexpr (!NTS) {
    *p = v;
  } else if constexpr (sizeof(S) == 2) {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short*)p);
  } else {
    __builtin_nontemporal_store(v, p);
  }
}

template <class L, bool NTS = false, class S, class T>
__device__ inline void store_one(S* __restrict__ dst, long long idx, int i, T x) {
  st_pop<NTS>(dst + idx, Codec<S, T>::st(x, T(1.0 / L::w[i])));
}

}  // namespace pflb
