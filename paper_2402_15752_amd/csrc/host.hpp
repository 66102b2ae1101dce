// Host-side helpers shared by the single-lattice and the batched C-ABI:
// parameter validation, workspace geometry and the lattice constants.
#pragma once

#include <cmath>
#include <cstdio>

#include "../../include/cplb.h"
#include "kernels.hpp"

namespace pflb {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Geometry {
  int dim, qtot, nhist;
  int px;            // row pitch (nodes between two rows); rows are packed, px = nx
  long long n;       // nodes
  long long cells;   // px ny nz: the nodes and the row padding of a plane
  long long stride;  // elements per plane
  size_t s_pop, s_cmp;
  size_t lat_bytes, hist_bytes, field_bytes, part_bytes, kp_bytes, total;
};

inline int validate(const cplb_params* p, char* err, size_t errn) {
  auto fail = [&](const char* m) {
    snprintf(err, errn, "%s", m);
    return CPLB_EINVAL;
  };
  if (!p) return fail("null parameters");
  if (p->lattice != CPLB_D2Q9 && p->lattice != CPLB_D3Q19_D3Q7) return fail("unknown lattice");
  if (p->precision < CPLB_F64 || p->precision > CPLB_F32_S16B) return fail("unknown precision");
  if (p->visc_law != CPLB_VISC_LINEAR && p->visc_law != CPLB_VISC_EXP)
    return fail("unknown viscosity law");
  if (p->scalar_model != CPLB_TWO_SCALAR && p->scalar_model != CPLB_ONE_SCALAR)
    return fail("unknown scalar model");
  if (p->scalar_model == CPLB_ONE_SCALAR && p->lattice != CPLB_D2Q9)
    return fail("the one-scalar model runs on CPLB_D2Q9 only");
  const int d = p->lattice == CPLB_D2Q9 ? 2 : 3;
  for (int f = 0; f < 6; ++f) {
    if (p->scalar_bc[f] != CPLB_BC_NOFLUX && p->scalar_bc[f] != CPLB_BC_DIRICHLET)
      return fail("unknown scalar boundary");
    if (p->scalar_bc[f] != CPLB_BC_DIRICHLET) continue;
    if (d != 2) return fail("Dirichlet faces run on CPLB_D2Q9 only");
    if (f / 2 >= d || p->periodic[f / 2]) return fail("a Dirichlet face needs a walled axis");
    if (p->scalar_model != CPLB_TWO_SCALAR) return fail("Dirichlet faces take the two-scalar model");
    if (!std::isfinite(p->c_wall[f][0]) || !std::isfinite(p->c_wall[f][1]))
      return fail("non-finite wall value");
  }
  if (p->scalar_grad != CPLB_GRAD_CENTRAL && p->scalar_grad != CPLB_GRAD_LOCAL)
    return fail("unknown scalar gradient scheme");
  if (p->phase_grad != CPLB_GRAD_CENTRAL && p->phase_grad != CPLB_GRAD_LOCAL)
    return fail("unknown phase gradient scheme");
  if (p->scalar_grad == CPLB_GRAD_LOCAL) {
    if (p->scalar_model != CPLB_TWO_SCALAR) return fail("the local gradient scheme takes the two-scalar model");
    for (int f = 0; f < 6; ++f)
      if (p->scalar_bc[f] != CPLB_BC_NOFLUX)
        return fail("the local gradient scheme takes no-flux scalar walls");
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail("grid sizes must be >= 1");
  if (d == 2 && p->nz != 1) return fail("2-D lattice needs nz = 1");
  const int n3[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < d; ++a)
    if (!p->periodic[a] && n3[a] < 2) return fail("a walled axis needs at least 2 nodes");
  if ((double)p->nx * p->ny * p->nz > 2.0e9) return fail("grid too large (> 2e9 nodes)");
  if (!(p->rho1 > 0 && p->rho2 > 0 && p->mu1 > 0 && p->mu2 > 0))
    return fail("densities and viscosities must be positive");
  if (!(p->W > 0 && p->M > 0 && p->D1 > 0 && p->D2 > 0 && p->Keq > 0 && p->n_eps > 0))
    return fail("W, M, D1, D2, Keq, n_eps must be positive (every tau > 1/2)");
  if (!(p->sigma >= 0 && p->A >= 0)) return fail("sigma and A must be >= 0");
  if (d == 2 && p->g[2] != 0.0) return fail("2-D lattice: g[2] must be 0");
  if (p->ref[1] != 0.0) return fail("ref[1] (flow set) must be 0");
  const double all[] = {p->rho1, p->rho2, p->mu1,  p->mu2,  p->sigma, p->W,    p->M,
                        p->D1,   p->D2,   p->Keq,  p->A,    p->g[0],  p->g[1], p->g[2],
                        p->rho_ref, p->n_eps, p->ref[0], p->ref[1], p->ref[2], p->ref[3]};
  for (double v : all)
    if (!std::isfinite(v)) return fail("non-finite parameter");
  return CPLB_OK;
}

// Field-by-field equality of two parameter sets (== on every double, so
// -0.0 equals +0.0; the struct's padding bytes take no part).
inline bool same_params(const cplb_params& a, const cplb_params& b) {
  bool eq = a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lattice == b.lattice &&
            a.precision == b.precision && a.visc_law == b.visc_law &&
            a.scalar_model == b.scalar_model && a.scalar_grad == b.scalar_grad &&
            a.phase_grad == b.phase_grad;
  for (int k = 0; k < 3; ++k) eq = eq && a.periodic[k] == b.periodic[k] && a.g[k] == b.g[k];
  eq = eq && a.rho1 == b.rho1 && a.rho2 == b.rho2 && a.mu1 == b.mu1 && a.mu2 == b.mu2 &&
       a.sigma == b.sigma && a.W == b.W && a.M == b.M && a.D1 == b.D1 && a.D2 == b.D2 &&
       a.Keq == b.Keq && a.A == b.A && a.rho_ref == b.rho_ref && a.n_eps == b.n_eps;
  for (int k = 0; k < 4; ++k) eq = eq && a.ref[k] == b.ref[k];
  for (int f = 0; f < 6; ++f)
    eq = eq && a.scalar_bc[f] == b.scalar_bc[f] && a.c_wall[f][0] == b.c_wall[f][0] &&
         a.c_wall[f][1] == b.c_wall[f][1];
  return eq;
}

inline Geometry geometry(const cplb_params* p) {
  Geometry G{};
  G.dim = p->lattice == CPLB_D2Q9 ? 2 : 3;
  G.qtot = G.dim == 2 ? Layout<D2Q9, D2Q9>::QTOT : Layout<D3Q7, D3Q19>::QTOT;
  G.nhist = G.dim == 2 ? kHist2D : kHist3D;
  G.n = (long long)p->nx * p->ny * p->nz;
  // Row pitch of the planes.  Rows are packed (px = nx): padding each row to
  // a multiple of 32 nodes (128-byte row starts in FP32) or to an odd
  // multiple of 16 was measured slower on MI355X, by up to 25% for batches of
  // 120-wide lattices, with no gain at any width; the kernels address every
  // plane through px all the same.
  G.px = p->nx;
  G.cells = (long long)G.px * p->ny * p->nz;
  // planes padded to 64 elements plus one 64-element skew, so that the
  // same node of successive planes does not land on the same HBM channel
  G.stride = (G.cells + 63) / 64 * 64 + 64;
  switch (p->precision) {
    case CPLB_F64: G.s_pop = 8; G.s_cmp = 8; break;
    case CPLB_F32: G.s_pop = 4; G.s_cmp = 4; break;
    default: G.s_pop = 2; G.s_cmp = 4; break;
  }
  G.lat_bytes = align_up((size_t)G.qtot * G.stride * G.s_pop, kAlign);
  G.hist_bytes = align_up((size_t)G.nhist * G.stride * G.s_cmp, kAlign);
  G.field_bytes = align_up((size_t)kNumFields * G.stride * G.s_cmp, kAlign);
  G.part_bytes = align_up((size_t)(kReduceBlocks + 1) * 8 * sizeof(double), kAlign);
  G.kp_bytes = align_up(sizeof(KParams<double>), kAlign) + align_up(sizeof(KParams<float>), kAlign);
  // two histories, alternating like the two lattices: a step reads the
  // previous level's (u, phi, c1, c2) -- the references of the populations it
  // reads, also at the halo nodes other work-groups own -- from one and writes
  // this level's to the other
  G.total = 2 * G.lat_bytes + 2 * G.hist_bytes + G.field_bytes + G.part_bytes + G.kp_bytes;
  return G;
}

// Plane skew (elements) of population plane q of the lattice layout: plane i
// of a set is stored shifted by -c_ix nodes (see addr.hpp); host copies of
// whole planes (checkpoints) start there.
inline long long plane_skew_el(int dim, int q) {
  if (dim == 2) return -(long long)D2Q9::cx[q % 9];
  using Lay = Layout<D3Q7, D3Q19>;
  if (q < Lay::G0) return -(long long)D3Q7::cx[q];
  if (q < Lay::H10) return -(long long)D3Q19::cx[q - Lay::G0];
  return -(long long)D3Q7::cx[(q - Lay::H10) % 7];
}

// every 2-D set (9 planes), the history and the field buffer below 4 GiB:
// 32-bit byte offsets reach every value
inline bool fits_u32_planes(const Geometry& G) {
  const unsigned long long lim = 1ull << 32;
  return 9ull * G.stride * G.s_pop < lim &&
         (unsigned long long)kNumFields * G.stride * G.s_cmp < lim;
}

template <class T>
KParams<T> make_kparams(const cplb_params* p, const Geometry& G) {
  KParams<T> K{};
  K.nx = p->nx;
  K.px = G.px;
  K.ny = p->ny;
  K.nz = p->nz;
  for (int a = 0; a < 3; ++a) K.wall[a] = (a < G.dim && !p->periodic[a]) ? 1 : 0;
  K.stride = G.stride;
  const double csf = G.dim == 2 ? D2Q9::cs2 : D3Q7::cs2;
  // relaxation times from the transport coefficients (Sec. III)
  const double tau_f = 0.5 + p->M / csf;
  const double tau_h1 = 0.5 + p->D1 / csf;
  const double tau_h2 = 0.5 + p->D2 / csf;
  // delta = 2 - 1/tau = 2 (tau - 1/2) / tau, formed from tau - 1/2 directly
  K.del_f = T(2.0 * (p->M / csf) / tau_f);
  K.hdel_f = T((p->M / csf) / tau_f);
  K.del_h1 = T(2.0 * (p->D1 / csf) / tau_h1);
  K.hdel_h1 = T((p->D1 / csf) / tau_h1);
  K.del_h2 = T(2.0 * (p->D2 / csf) / tau_h2);
  K.hdel_h2 = T((p->D2 / csf) / tau_h2);
  // beta = 12 sigma / W, k = 3 sigma W / 2 (Sec. II B)
  K.beta4 = T(4.0 * 12.0 * p->sigma / p->W);
  K.kappa = T(1.5 * p->sigma * p->W);
  K.rho1 = T(p->rho1);
  K.rho2 = T(p->rho2);
  K.drho = T(p->rho1 - p->rho2);
  K.rho_ref = T(p->rho_ref);
  for (int a = 0; a < 3; ++a) K.grav[a] = T(p->g[a]);
  K.mu1 = T(p->mu1);
  K.mu2 = T(p->mu2);
  K.ln_mu1 = T(std::log(p->mu1));
  K.ln_mu2 = T(std::log(p->mu2));
  K.visc_exp = p->visc_law == CPLB_VISC_EXP;
  K.D1D2 = T(p->D1 * p->D2);
  K.KD1 = T(p->Keq * p->D1);
  K.D2 = T(p->D2);
  K.Keq = T(p->Keq);
  K.A = T(p->A);
  K.half_A = T(0.5 * p->A);
  K.four_over_W = T(4.0 / p->W);
  // one-scalar model (Sec. III D): D_eff = D1 Keq phi + D2 (1 - phi)
  K.one_scalar = p->scalar_model == CPLB_ONE_SCALAR;
  K.D1K = T(p->D1 * p->Keq);
  // local scheme for grad c_k (Eq. (39)): 1 / (tau_hk cs^2) and 4 D_k / W
  K.local_grad = p->scalar_grad == CPLB_GRAD_LOCAL;
  K.itc1 = T(1.0 / (tau_h1 * csf));
  K.itc2 = T(1.0 / (tau_h2 * csf));
  K.d1w = T(4.0 * p->D1 / p->W);
  K.d2w = T(4.0 * p->D2 / p->W);
  // local scheme for grad phi (after Eq. (39)): 1 / (tau_f cs^2) and 4 M / W
  K.local_phase = p->phase_grad == CPLB_GRAD_LOCAL;
  K.itf = T(1.0 / (tau_f * csf));
  K.ec2 = T((tau_f * csf * p->n_eps) * (tau_f * csf * p->n_eps));
  K.mw = T(4.0 * p->M / p->W);
  // Dirichlet faces x-, x+, y-, y+ (bit f) and their values
  K.dirichlet = 0;
  for (int f = 0; f < 4; ++f) {
    if (f / 2 < G.dim && p->scalar_bc[f] == CPLB_BC_DIRICHLET) K.dirichlet |= 1 << f;
    K.cw[f][0] = T(p->c_wall[f][0]);
    K.cw[f][1] = T(p->c_wall[f][1]);
  }
  K.neps2 = T(p->n_eps * p->n_eps);
  // references of the stored deviations: f always, and h1, h2 of the
  // two-scalar model with the central stencil, are stored relative to the
  // node's own phi, c1, c2 of the previous level; h1, h2 of the one-scalar
  // model and of the local gradient scheme (no scalar halo) relative to the
  // uniform ref[2], ref[3]; g is stored as is
  K.href = p->scalar_model == CPLB_TWO_SCALAR && p->scalar_grad == CPLB_GRAD_CENTRAL;
  K.ref_c1 = T(p->ref[2]);
  K.ref_c2 = T(p->ref[3]);
  return K;
}

}  // namespace pflb
