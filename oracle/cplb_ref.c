/*
 * cplb_ref.c -- plain FP64 CPU oracle of the coupled phase-field lattice
 * Boltzmann method of Chen, Zhan, Chai & Shi (arXiv 2402.15752).
 *
 * TEST INFRASTRUCTURE ONLY (see cplb_ref.h).  Slow and obvious on purpose:
 * separate passes over all nodes, no blocking, no fusion, a fixed summation
 * order i = 0..Q-1, compiled with -ffp-contract=off.
 *
 * One time step, in the order the quantities depend on each other:
 *   pass 1  (all nodes)  phi, D_m, c1, c2, psi = c1 + Keq c2      Sec. III A/C
 *   pass 2  (all nodes)  grad phi, lap phi, grad psi (isotropic central
 *                        stencils), n, mu_phi, rho, F, u, p, mu, tau_g  Sec. II/III
 *   pass 3  (all nodes)  time-derivative terms, SRT collision of f, g, h1, h2
 *                        with their source distributions               Sec. III
 *   pass 4  (all nodes)  streaming with periodic wrap or half-way bounce-back
 *   history <- (u, phi, c1, c2) of this time level
 *
 * Readings of the paper taken here (where it is silent):
 *   - d/dt(phi u), d/dt(c_k u): first-order backward difference between this
 *     time level and the previous one; the history starts at the initial
 *     fields, u = 0 unless given.
 *   - the unit normal n = grad phi / |grad phi| is regularised as
 *     grad phi / sqrt(|grad phi|^2 + n_eps^2): the same vector wherever
 *     |grad phi| >> n_eps, continuous where the gradient vanishes (drop
 *     centres, bulk phases), so that round-off cannot switch it on or off.
 *   - body force G = (rho - rho_ref) g.
 *   - next to a wall the stencils read a mirror ghost: a coordinate one step
 *     outside the domain maps back to the boundary node (zero normal gradient).
 *   - the implicit recovery of c1, c2 (Sec. III C) is solved exactly as the
 *     2x2 linear system it is.
 *   - (rho1-rho2) u grad(phi) : c_i c_i is read as (c_i.u)(c_i.grad phi).
 *   - 3-D: D3Q19 for the flow set and the stencils, D3Q7 (w0 = 1/4,
 *     w = 1/8, cs^2 = 1/4) for f, h1, h2.
 */
#include "cplb_ref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 19

typedef struct {
  int q;
  int c[MAXQ][3];
  double w[MAXQ];
  double cs2;
  int opp[MAXQ];
} lattice_t;

static void set_dir(lattice_t* L, int i, int cx, int cy, int cz, double w) {
  L->c[i][0] = cx;
  L->c[i][1] = cy;
  L->c[i][2] = cz;
  L->w[i] = w;
}

/* opposite direction found by search: c_opp = -c_i */
static void find_opposites(lattice_t* L) {
  for (int i = 0; i < L->q; i++) {
    L->opp[i] = -1;
    for (int j = 0; j < L->q; j++)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  }
}

/* D2Q9 (Qian et al., cited in Sec. IV): w0 = 4/9, axis 1/9, diagonal 1/36 */
static void make_d2q9(lattice_t* L) {
  L->q = 9;
  L->cs2 = 1.0 / 3.0;
  set_dir(L, 0, 0, 0, 0, 4.0 / 9.0);
  set_dir(L, 1, 1, 0, 0, 1.0 / 9.0);
  set_dir(L, 2, 0, 1, 0, 1.0 / 9.0);
  set_dir(L, 3, -1, 0, 0, 1.0 / 9.0);
  set_dir(L, 4, 0, -1, 0, 1.0 / 9.0);
  set_dir(L, 5, 1, 1, 0, 1.0 / 36.0);
  set_dir(L, 6, -1, 1, 0, 1.0 / 36.0);
  set_dir(L, 7, -1, -1, 0, 1.0 / 36.0);
  set_dir(L, 8, 1, -1, 0, 1.0 / 36.0);
  find_opposites(L);
}

/* D3Q19: w0 = 1/3, 6 axis links 1/18, 12 edge links 1/36 */
static void make_d3q19(lattice_t* L) {
  int i = 0;
  L->q = 19;
  L->cs2 = 1.0 / 3.0;
  set_dir(L, i++, 0, 0, 0, 1.0 / 3.0);
  for (int a = 0; a < 3; a++)
    for (int s = 1; s >= -1; s -= 2) {
      int c[3] = {0, 0, 0};
      c[a] = s;
      set_dir(L, i++, c[0], c[1], c[2], 1.0 / 18.0);
    }
  for (int a = 0; a < 3; a++)
    for (int b = a + 1; b < 3; b++)
      for (int sa = 1; sa >= -1; sa -= 2)
        for (int sb = 1; sb >= -1; sb -= 2) {
          int c[3] = {0, 0, 0};
          c[a] = sa;
          c[b] = sb;
          set_dir(L, i++, c[0], c[1], c[2], 1.0 / 36.0);
        }
  find_opposites(L);
}

/* D3Q7: w0 = 1/4, 6 axis links 1/8, cs^2 = 1/4 */
static void make_d3q7(lattice_t* L) {
  int i = 0;
  L->q = 7;
  L->cs2 = 0.25;
  set_dir(L, i++, 0, 0, 0, 0.25);
  for (int a = 0; a < 3; a++)
    for (int s = 1; s >= -1; s -= 2) {
      int c[3] = {0, 0, 0};
      c[a] = s;
      set_dir(L, i++, c[0], c[1], c[2], 0.125);
    }
  find_opposites(L);
}

struct cplb_ref {
  cplb_ref_params p;
  int d;
  long nx, ny, nz, N;
  lattice_t LF; /* lattice of f, h1, h2 */
  lattice_t LG; /* lattice of g and of the gradient / Laplacian stencils */
  /* populations at the current time level (post-streaming), Q planes of N */
  double *f, *g, *h1, *h2;
  /* post-collision populations */
  double *fs, *gs, *h1s, *h2s;
  /* pass-1 fields */
  double *phi, *c1, *c2, *psi, *Dm;
  double* ctot; /* c1 + c2; in the one-scalar model the moment c = sum h3_i itself */
  /* pass-2 fields */
  double *gphi, *gpsi, *lap, *nrm, *mu_phi, *rho, *F, *u, *pr, *mu, *tau_g;
  /* history: fields of the previous time level */
  double *u_old, *phi_old, *c1_old, *c2_old;
  int64_t step;
  int macros_valid;
  /* caller's per-node corrections of c1 and c2 (learned-closure extension:
     two planes of N values, s1 then s2), or NULL */
  const double* xs;
  char err[256];
};

static void set_err(cplb_ref_t* h, const char* m) {
  snprintf(h->err, sizeof(h->err), "%s", m);
}

const char* cplb_ref_last_error(const cplb_ref_t* h) { return h ? h->err : "null handle"; }

static double* alloc0(long n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

int cplb_ref_population_count(const cplb_ref_t* h, int set) {
  if (!h) return 0;
  return set == 1 ? h->LG.q : h->LF.q;
}

static int check_params(const cplb_ref_params* p, char* err) {
  const int d = p->lattice == CPLB_REF_D2Q9 ? 2 : 3;
  if (p->lattice != CPLB_REF_D2Q9 && p->lattice != CPLB_REF_D3Q19_D3Q7) {
    strcpy(err, "unknown lattice");
    return -1;
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || (d == 2 && p->nz != 1)) {
    strcpy(err, "bad grid size");
    return -1;
  }
  long n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < d; a++)
    if (!p->periodic[a] && n[a] < 2) {
      strcpy(err, "a walled axis needs at least 2 nodes");
      return -1;
    }
  if (p->visc_law != CPLB_REF_VISC_LINEAR && p->visc_law != CPLB_REF_VISC_EXP) {
    strcpy(err, "unknown viscosity law");
    return -1;
  }
  if (!(p->rho1 > 0 && p->rho2 > 0 && p->mu1 > 0 && p->mu2 > 0)) {
    strcpy(err, "densities and viscosities must be positive");
    return -1;
  }
  if (d == 2 && p->g[2] != 0.0) {
    strcpy(err, "2-D lattice: g[2] must be 0");
    return -1;
  }
  for (int f = 0; f < 6; f++) {
    if (p->scalar_bc[f] != CPLB_REF_NOFLUX && p->scalar_bc[f] != CPLB_REF_DIRICHLET) {
      strcpy(err, "unknown scalar boundary");
      return -1;
    }
    if (p->scalar_bc[f] == CPLB_REF_DIRICHLET) {
      if (f / 2 >= d || p->periodic[f / 2]) {
        strcpy(err, "a Dirichlet face needs a walled axis of the lattice");
        return -1;
      }
      if (p->scalar_model != CPLB_REF_TWO_SCALAR) {
        strcpy(err, "Dirichlet faces take the two-scalar model");
        return -1;
      }
    }
  }
  if (p->scalar_grad != CPLB_REF_GRAD_CENTRAL && p->scalar_grad != CPLB_REF_GRAD_LOCAL) {
    strcpy(err, "unknown scalar gradient scheme");
    return -1;
  }
  if (p->phase_grad != CPLB_REF_GRAD_CENTRAL && p->phase_grad != CPLB_REF_GRAD_LOCAL) {
    strcpy(err, "unknown phase gradient scheme");
    return -1;
  }
  if (p->scalar_model != CPLB_REF_TWO_SCALAR && p->scalar_model != CPLB_REF_ONE_SCALAR) {
    strcpy(err, "unknown scalar model");
    return -1;
  }
  if (!(p->W > 0 && p->sigma >= 0 && p->M > 0 && p->D1 > 0 && p->D2 > 0 && p->Keq > 0 && p->A >= 0 &&
        p->n_eps > 0)) {
    strcpy(err, "need W, M, D1, D2, Keq, n_eps > 0 and sigma, A >= 0");
    return -1;
  }
  /* tau_f, tau_h1, tau_h2 > 1/2 follow from M, D_k > 0 */
  return 0;
}

int cplb_ref_create(const cplb_ref_params* prm, cplb_ref_t** out) {
  if (!prm || !out) return CPLB_REF_EINVAL;
  *out = NULL;
  char err[256];
  if (check_params(prm, err)) return CPLB_REF_EINVAL;
  cplb_ref_t* h = (cplb_ref_t*)calloc(1, sizeof(cplb_ref_t));
  if (!h) return CPLB_REF_ENOMEM;
  h->p = *prm;
  h->d = prm->lattice == CPLB_REF_D2Q9 ? 2 : 3;
  if (h->d == 2) h->p.periodic[2] = 1;
  h->nx = prm->nx;
  h->ny = prm->ny;
  h->nz = prm->nz;
  h->N = h->nx * h->ny * h->nz;
  if (h->d == 2) {
    make_d2q9(&h->LF);
    make_d2q9(&h->LG);
  } else {
    make_d3q7(&h->LF);
    make_d3q19(&h->LG);
  }
  const long N = h->N;
  h->f = alloc0(h->LF.q * N);
  h->h1 = alloc0(h->LF.q * N);
  h->h2 = alloc0(h->LF.q * N);
  h->g = alloc0(h->LG.q * N);
  h->fs = alloc0(h->LF.q * N);
  h->h1s = alloc0(h->LF.q * N);
  h->h2s = alloc0(h->LF.q * N);
  h->gs = alloc0(h->LG.q * N);
  h->phi = alloc0(N);
  h->c1 = alloc0(N);
  h->c2 = alloc0(N);
  h->psi = alloc0(N);
  h->Dm = alloc0(N);
  h->ctot = alloc0(N);
  h->gphi = alloc0(3 * N);
  h->gpsi = alloc0(3 * N);
  h->lap = alloc0(N);
  h->nrm = alloc0(3 * N);
  h->mu_phi = alloc0(N);
  h->rho = alloc0(N);
  h->F = alloc0(3 * N);
  h->u = alloc0(3 * N);
  h->pr = alloc0(N);
  h->mu = alloc0(N);
  h->tau_g = alloc0(N);
  h->u_old = alloc0(3 * N);
  h->phi_old = alloc0(N);
  h->c1_old = alloc0(N);
  h->c2_old = alloc0(N);
  if (!h->f || !h->h1 || !h->h2 || !h->g || !h->fs || !h->h1s || !h->h2s || !h->gs || !h->phi ||
      !h->c1 || !h->c2 || !h->psi || !h->Dm || !h->ctot || !h->gphi || !h->gpsi || !h->lap || !h->nrm ||
      !h->mu_phi || !h->rho || !h->F || !h->u || !h->pr || !h->mu || !h->tau_g || !h->u_old ||
      !h->phi_old || !h->c1_old || !h->c2_old) {
    cplb_ref_destroy(h);
    return CPLB_REF_ENOMEM;
  }
  *out = h;
  return CPLB_REF_OK;
}

void cplb_ref_destroy(cplb_ref_t* h) {
  if (!h) return;
  double* all[] = {h->f,   h->g,     h->h1,  h->h2,     h->fs,      h->gs,      h->h1s,
                   h->h2s, h->phi,   h->c1,  h->c2,     h->psi,     h->Dm,      h->gphi,
                   h->gpsi, h->lap,  h->nrm, h->mu_phi, h->rho,     h->F,       h->u,
                   h->pr,  h->mu,    h->tau_g, h->u_old, h->phi_old, h->c1_old, h->c2_old,
                   h->ctot};
  for (size_t k = 0; k < sizeof(all) / sizeof(all[0]); k++) free(all[k]);
  free(h);
}

/* ---------------------------------------------------------------- helpers */

static void coords(const cplb_ref_t* h, long n, long* x, long* y, long* z) {
  *x = n % h->nx;
  *y = (n / h->nx) % h->ny;
  *z = n / (h->nx * h->ny);
}

/* Neighbour index for the stencils: periodic wrap, or mirror ghost on a
 * walled axis (a coordinate one step outside maps back onto the boundary
 * node, i.e. zero normal gradient). */
static long stencil_index(const cplb_ref_t* h, long x, long y, long z, const int* c) {
  long v[3] = {x + c[0], y + c[1], z + c[2]};
  long n[3] = {h->nx, h->ny, h->nz};
  for (int a = 0; a < 3; a++) {
    if (v[a] >= 0 && v[a] < n[a]) continue;
    if (h->p.periodic[a])
      v[a] = ((v[a] % n[a]) + n[a]) % n[a];
    else
      v[a] = v[a] < 0 ? -1 - v[a] : 2 * n[a] - 1 - v[a];
  }
  return v[0] + n[0] * (v[1] + n[1] * v[2]);
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double cdot(const int* c, const double* v) { return c[0] * v[0] + c[1] * v[1] + c[2] * v[2]; }

/* --------------------------------------------------------- equilibria */

/* f_i^eq = w_i phi (1 + c_i.u / cs^2)            (phase-field LB, Sec. III A) */
static double f_eq(const lattice_t* L, int i, double phi, const double* u) {
  return L->w[i] * phi * (1.0 + cdot(L->c[i], u) / L->cs2);
}

/* s_i(u) = w_i [c_i.u/cs^2 + (c_i.u)^2/(2 cs^4) - u.u/(2 cs^2)]   (Sec. III B) */
static double s_i(const lattice_t* L, int i, const double* u) {
  double cu = cdot(L->c[i], u);
  return L->w[i] * (cu / L->cs2 + cu * cu / (2.0 * L->cs2 * L->cs2) - dot3(u, u) / (2.0 * L->cs2));
}

/* g_i^eq = p/cs^2 (w_0 - 1) + rho s_0 for i = 0, p/cs^2 w_i + rho s_i else */
static double g_eq(const lattice_t* L, int i, double p, double rho, const double* u) {
  if (i == 0) return p / L->cs2 * (L->w[0] - 1.0) + rho * s_i(L, 0, u);
  return p / L->cs2 * L->w[i] + rho * s_i(L, i, u);
}

/* h_k,i^eq = w_i c_k (1 + c_i.u / cs^2)           (Sec. III C) */
static double h_eq(const lattice_t* L, int i, double c, const double* u) {
  return L->w[i] * c * (1.0 + cdot(L->c[i], u) / L->cs2);
}

/* one-scalar model (Sec. III D): h3_0^eq = c + (w_0 - 1) c / K_eff,
 * h3_i^eq = w_i c / K_eff + w_i c_i.(c u) / cs^2 for i != 0 */
static double h3_eq(const lattice_t* L, int i, double c, double Keff, const double* u) {
  if (i == 0) return c + (L->w[0] - 1.0) * c / Keff;
  return L->w[i] * c / Keff + L->w[i] * c * cdot(L->c[i], u) / L->cs2;
}

/* equilibrium concentration ratio across the interface, K_eff = Keq phi + 1 - phi
 * (Sec. II D) */
static double k_eff(const cplb_ref_params* P, double phi) { return P->Keq * phi + (1.0 - phi); }

/* ---------------------------------------------------------------- init */

int cplb_ref_init_fields(cplb_ref_t* h, const double* phi, const double* c1, const double* c2,
                         const double* u, const double* p) {
  if (!h || !phi || !c1 || !c2) return CPLB_REF_EINVAL;
  const long N = h->N;
  const int d = h->d;
  for (long n = 0; n < N; n++) {
    double un[3] = {0, 0, 0};
    if (u)
      for (int a = 0; a < d; a++) un[a] = u[a * N + n];
    double pn = p ? p[n] : 0.0;
    double rho = phi[n] * (h->p.rho1 - h->p.rho2) + h->p.rho2;
    const int one = h->p.scalar_model == CPLB_REF_ONE_SCALAR;
    for (int i = 0; i < h->LF.q; i++) {
      h->f[i * N + n] = f_eq(&h->LF, i, phi[n], un);
      if (one) {
        /* h3 carries the total c = c1 + c2 */
        h->h1[i * N + n] = h3_eq(&h->LF, i, c1[n] + c2[n], k_eff(&h->p, phi[n]), un);
        h->h2[i * N + n] = 0.0;
      } else {
        h->h1[i * N + n] = h_eq(&h->LF, i, c1[n], un);
        h->h2[i * N + n] = h_eq(&h->LF, i, c2[n], un);
      }
    }
    for (int i = 0; i < h->LG.q; i++) h->g[i * N + n] = g_eq(&h->LG, i, pn, rho, un);
    for (int a = 0; a < 3; a++) h->u_old[a * N + n] = un[a];
    h->phi_old[n] = phi[n];
    h->c1_old[n] = one ? c1[n] + c2[n] : c1[n];
    h->c2_old[n] = one ? 0.0 : c2[n];
  }
  h->step = 0;
  h->macros_valid = 0;
  return CPLB_REF_OK;
}

int cplb_ref_init_sdf(cplb_ref_t* h, const double* l, double c1_a, double c1_b, double c2_a,
                      double c2_b) {
  if (!h || !l) return CPLB_REF_EINVAL;
  const long N = h->N;
  double* phi = alloc0(N);
  double* c1 = alloc0(N);
  double* c2 = alloc0(N);
  if (!phi || !c1 || !c2) {
    free(phi);
    free(c1);
    free(c2);
    return CPLB_REF_ENOMEM;
  }
  for (long n = 0; n < N; n++) {
    /* hyperbolic-tangent profile of a signed distance, Sec. II A */
    phi[n] = 0.5 + 0.5 * tanh(2.0 * l[n] / h->p.W);
    c1[n] = c1_a + c1_b * phi[n];
    c2[n] = c2_a + c2_b * phi[n];
  }
  int rc = cplb_ref_init_fields(h, phi, c1, c2, NULL, NULL);
  free(phi);
  free(c1);
  free(c2);
  return rc;
}

/* -------------------------------------------------------------- pass 1 */

/* phi = sum f_i; D_m; implicit recovery of c1, c2; psi = c1 + Keq c2 */
static void pass1(cplb_ref_t* h) {
  const long N = h->N;
  const cplb_ref_params* P = &h->p;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double phi = 0, S1 = 0, S2 = 0;
    for (int i = 0; i < h->LF.q; i++) phi += h->f[i * N + n];
    for (int i = 0; i < h->LF.q; i++) S1 += h->h1[i * N + n];
    if (P->scalar_model == CPLB_REF_ONE_SCALAR) {
      /* c = sum h3_i; the phase parts of c at interfacial equilibrium,
         c~1 = Keq c~2 and c = c~1 phi + c~2 (1 - phi) (Sec. II D); the
         effective diffusivity D_eff = D1 Keq phi + D2 (1 - phi) is kept
         in the D_m slot */
      const double c = S1, Keff = k_eff(P, phi);
      const double ct2 = c / Keff;
      h->phi[n] = phi;
      h->Dm[n] = P->D1 * P->Keq * phi + P->D2 * (1.0 - phi);
      h->c1[n] = P->Keq * ct2 * phi;
      h->c2[n] = ct2 * (1.0 - phi);
      h->psi[n] = h->c1[n] + P->Keq * h->c2[n];
      h->ctot[n] = c;
      continue;
    }
    for (int i = 0; i < h->LF.q; i++) S2 += h->h2[i * N + n];
    /* mixed diffusivity, Sec. II C */
    double Dm = P->D1 * P->D2 / (P->Keq * P->D1 * (1.0 - phi) + P->D2 * phi);
    /* c1 = S1 + a [Keq c2 phi - c1 (1-phi)],  c2 = S2 + a [c1 (1-phi) - Keq c2 phi],
     * a = A D_m / 2: a linear 2x2 system in (c1, c2), solved exactly */
    double a = 0.5 * P->A * Dm;
    double a11 = 1.0 + a * (1.0 - phi), a12 = -a * P->Keq * phi;
    double a21 = -a * (1.0 - phi), a22 = 1.0 + a * P->Keq * phi;
    double det = a11 * a22 - a12 * a21;
    double c1 = (S1 * a22 - a12 * S2) / det;
    double c2 = (a11 * S2 - a21 * S1) / det;
    h->phi[n] = phi;
    h->Dm[n] = Dm;
    h->c1[n] = c1;
    h->c2[n] = c2;
    h->psi[n] = c1 + P->Keq * c2;
    h->ctot[n] = c1 + c2;
  }
}

/* -------------------------------------------------------------- pass 2 */

static void pass2(cplb_ref_t* h) {
  const long N = h->N;
  const cplb_ref_params* P = &h->p;
  const lattice_t* L = &h->LG;
  const double beta = 12.0 * P->sigma / P->W;
  const double kappa = 1.5 * P->sigma * P->W;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    long x, y, z;
    coords(h, n, &x, &y, &z);
    const double phi = h->phi[n];
    double gphi[3] = {0, 0, 0}, gpsi[3] = {0, 0, 0}, lap = 0;
    /* isotropic central gradient and Laplacian, Sec. III C */
    for (int i = 1; i < L->q; i++) {
      long m = stencil_index(h, x, y, z, L->c[i]);
      for (int a = 0; a < 3; a++) {
        gphi[a] += L->w[i] * L->c[i][a] * h->phi[m] / L->cs2;
        gpsi[a] += L->w[i] * L->c[i][a] * h->psi[m] / L->cs2;
      }
      lap += 2.0 * L->w[i] * (h->phi[m] - phi) / L->cs2;
    }
    if (P->phase_grad == CPLB_REF_GRAD_LOCAL) {
      /* local scheme after Eq. (39): with C = sum c_i f_i - phi u +
         d_t(phi u) / 2, D = -tau_f cs^2 and B = 4 M phi (1 - phi) / W,
         |grad phi| = (-|C| - B) / D and grad phi = C / (D + B / |grad phi|).
         u and d_t(phi u) need grad phi (through the force), so the previous
         level's u stands in for u, and d_t(phi u) is the backward difference
         (phi - phi_old) u_old.  The direction C / |C| is undefined where C
         vanishes -- at an equilibrium start C is round-off everywhere -- so
         it is regularised like the normal: |C| in the denominator becomes
         sqrt(|C|^2 + (tau_f cs^2 n_eps)^2), the scale of C at a gradient of
         n_eps. */
      const lattice_t* LF = &h->LF;
      const double tau_f = 0.5 + P->M / LF->cs2;
      const double D = -tau_f * LF->cs2, B = 4.0 * P->M * phi * (1.0 - phi) / P->W;
      double C[3] = {0, 0, 0};
      for (int i = 0; i < LF->q; i++)
        for (int a = 0; a < 3; a++) C[a] += LF->c[i][a] * h->f[i * N + n];
      for (int a = 0; a < 3; a++) {
        const double uo = h->u_old[a * N + n];
        C[a] += -phi * uo + 0.5 * (phi - h->phi_old[n]) * uo;
      }
      /* D + B / |grad phi| = D |C| / (|C| + B): the quotient is taken in
         that form, which does not cancel where |C| << B */
      const double cn = sqrt(dot3(C, C)), ec = tau_f * LF->cs2 * P->n_eps;
      for (int a = 0; a < 3; a++) gphi[a] = C[a] * (cn + B) / (D * sqrt(cn * cn + ec * ec));
    }
    /* unit normal n = grad phi / |grad phi|, regularised at n_eps */
    double norm = sqrt(dot3(gphi, gphi) + P->n_eps * P->n_eps);
    double nv[3];
    for (int a = 0; a < 3; a++) nv[a] = gphi[a] / norm;
    /* chemical potential */
    double mu_phi = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap;
    /* density, linear in phi */
    double rho = phi * (P->rho1 - P->rho2) + P->rho2;
    /* total force F = mu_phi grad phi + G,  G = (rho - rho_ref) g */
    double F[3];
    for (int a = 0; a < 3; a++) F[a] = mu_phi * gphi[a] + (rho - P->rho_ref) * P->g[a];
    /* velocity u = [sum c_i g_i + F/2] / rho */
    double m1[3] = {0, 0, 0};
    for (int i = 0; i < L->q; i++)
      for (int a = 0; a < 3; a++) m1[a] += L->c[i][a] * h->g[i * N + n];
    double u[3];
    for (int a = 0; a < 3; a++) u[a] = (m1[a] + 0.5 * F[a]) / rho;
    /* pressure p = cs^2/(1-w0) [sum_{i!=0} g_i + (rho1-rho2) u.grad phi / 2 + rho s_0(u)] */
    double sg = 0;
    for (int i = 1; i < L->q; i++) sg += h->g[i * N + n];
    double pr = L->cs2 / (1.0 - L->w[0]) *
                (sg + 0.5 * (P->rho1 - P->rho2) * dot3(u, gphi) + rho * s_i(L, 0, u));
    if (P->scalar_grad == CPLB_REF_GRAD_LOCAL && P->scalar_model == CPLB_REF_TWO_SCALAR) {
      /* local scheme, Eq. (39): grad c_k from the first moment of h_k,
         with d_t(c_k u) the backward difference against the history */
      const lattice_t* LF = &h->LF;
      const double tau1 = 0.5 + P->D1 / LF->cs2, tau2 = 0.5 + P->D2 / LF->cs2;
      const double c1 = h->c1[n], c2 = h->c2[n];
      double q1[3] = {0, 0, 0}, q2[3] = {0, 0, 0};
      for (int i = 0; i < LF->q; i++)
        for (int a = 0; a < 3; a++) {
          q1[a] += LF->c[i][a] * h->h1[i * N + n];
          q2[a] += LF->c[i][a] * h->h2[i * N + n];
        }
      for (int a = 0; a < 3; a++) {
        const double uo = h->u_old[a * N + n];
        const double dt1 = c1 * u[a] - h->c1_old[n] * uo;
        const double dt2 = c2 * u[a] - h->c2_old[n] * uo;
        const double g1 = (-q1[a] + c1 * u[a] - 0.5 * dt1 +
                           P->D1 * 4.0 * (1.0 - phi) * c1 / P->W * nv[a]) / (tau1 * LF->cs2);
        const double g2 = (-q2[a] + c2 * u[a] - 0.5 * dt2 -
                           P->D2 * 4.0 * phi * c2 / P->W * nv[a]) / (tau2 * LF->cs2);
        gpsi[a] = g1 + P->Keq * g2;
      }
    }
    /* viscosity: linear law, Eq. (1.8), or exponential law, Eq. (4.3) */
    double mu;
    if (P->visc_law == CPLB_REF_VISC_EXP)
      mu = exp(h->c1[n] * log(P->mu1) + h->c2[n] * log(P->mu2));
    else
      mu = phi * (P->mu1 - P->mu2) + P->mu2;
    /* mu = rho (tau_g - 1/2) cs^2 */
    double tau_g = 0.5 + mu / (rho * L->cs2);
    for (int a = 0; a < 3; a++) {
      h->gphi[a * N + n] = gphi[a];
      h->gpsi[a * N + n] = gpsi[a];
      h->nrm[a * N + n] = nv[a];
      h->F[a * N + n] = F[a];
      h->u[a * N + n] = u[a];
    }
    h->lap[n] = lap;
    h->mu_phi[n] = mu_phi;
    h->rho[n] = rho;
    h->pr[n] = pr;
    h->mu[n] = mu;
    h->tau_g[n] = tau_g;
  }
}

static void macros(cplb_ref_t* h) {
  if (h->macros_valid) return;
  pass1(h);
  pass2(h);
  h->macros_valid = 1;
}

/* -------------------------------------------------------------- pass 3 */

static void collide(cplb_ref_t* h) {
  const long N = h->N;
  const cplb_ref_params* P = &h->p;
  const lattice_t* LF = &h->LF;
  const lattice_t* LG = &h->LG;
  /* M = (tau_f - 1/2) cs^2,  D_k = (tau_hk - 1/2) cs^2 */
  const double tau_f = 0.5 + P->M / LF->cs2;
  const double tau_h1 = 0.5 + P->D1 / LF->cs2;
  const double tau_h2 = 0.5 + P->D2 / LF->cs2;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    const double phi = h->phi[n], c1 = h->c1[n], c2 = h->c2[n], Dm = h->Dm[n];
    const double rho = h->rho[n], pr = h->pr[n], tau_g = h->tau_g[n];
    double u[3], gphi[3], gpsi[3], nv[3], F[3], u_old[3];
    for (int a = 0; a < 3; a++) {
      u[a] = h->u[a * N + n];
      gphi[a] = h->gphi[a * N + n];
      gpsi[a] = h->gpsi[a * N + n];
      nv[a] = h->nrm[a * N + n];
      F[a] = h->F[a * N + n];
      u_old[a] = h->u_old[a * N + n];
    }
    /* time derivatives by backward difference over one step */
    double dphiu[3], dc1u[3], dc2u[3];
    for (int a = 0; a < 3; a++) {
      dphiu[a] = phi * u[a] - h->phi_old[n] * u_old[a];
      dc1u[a] = c1 * u[a] - h->c1_old[n] * u_old[a];
      dc2u[a] = c2 * u[a] - h->c2_old[n] * u_old[a];
    }
    /* phase field f: source F_i = w_i [c_i.d_t(phi u)/cs^2 + c_i.n 4 phi (1-phi)/W] */
    for (int i = 0; i < LF->q; i++) {
      const int* c = LF->c[i];
      double feq = f_eq(LF, i, phi, u);
      double Fi = LF->w[i] * (cdot(c, dphiu) / LF->cs2 + cdot(c, nv) * 4.0 * phi * (1.0 - phi) / P->W);
      double fi = h->f[i * N + n];
      h->fs[i * N + n] = fi - (fi - feq) / tau_f + (1.0 - 1.0 / (2.0 * tau_f)) * Fi;
    }
    /* flow g: G_i = w_i [c_i.F/cs^2 + (rho1-rho2)(c_i.u)(c_i.grad phi)/cs^2] */
    for (int i = 0; i < LG->q; i++) {
      const int* c = LG->c[i];
      double geq = g_eq(LG, i, pr, rho, u);
      double Gi = LG->w[i] * (cdot(c, F) / LG->cs2 +
                              (P->rho1 - P->rho2) * cdot(c, u) * cdot(c, gphi) / LG->cs2);
      double gi = h->g[i * N + n];
      h->gs[i * N + n] = gi - (gi - geq) / tau_g + (1.0 - 1.0 / (2.0 * tau_g)) * Gi;
    }
    if (P->scalar_model == CPLB_REF_ONE_SCALAR) {
      /* one-scalar set h3 (Sec. III D): tau_h3 from D_eff = (tau_h3 - 1/2) cs^2,
         source H3_i = w_i c_i.d_t(c u)/cs^2; the history keeps c in the c1 slot */
      const double c = h->ctot[n], Keff = k_eff(P, phi);
      const double tau3 = 0.5 + Dm / LF->cs2;
      double dcu[3];
      for (int a = 0; a < 3; a++) dcu[a] = c * u[a] - h->c1_old[n] * u_old[a];
      for (int i = 0; i < LF->q; i++) {
        const int* cc = LF->c[i];
        double heq = h3_eq(LF, i, c, Keff, u);
        double H3 = LF->w[i] * cdot(cc, dcu) / LF->cs2;
        double a1 = h->h1[i * N + n];
        h->h1s[i * N + n] = a1 - (a1 - heq) / tau3 + (1.0 - 1.0 / (2.0 * tau3)) * H3;
        h->h2s[i * N + n] = 0.0;
      }
      continue;
    }
    /* two-scalar sets h1, h2 with sources H_k and auxiliary sources ~H_k */
    const double M1 = P->A * Dm * (P->Keq * c2 * phi - c1 * (1.0 - phi));
    const double M2 = P->A * Dm * (c1 * (1.0 - phi) - P->Keq * c2 * phi);
    /* D_m grad phi . grad(c1 + Keq c2).  The closure's corrections x1, x2
       of c1, c2 are carried like ~H: h_k loses w_i s_k with (s1, s2) the
       solution of J (s1, s2) = (x1, x2), J the Jacobian of the implicit
       recovery c_k(S1, S2) above, so that the recovered c_k drops by x_k */
    const double aux = Dm * dot3(gphi, gpsi);
    double s1 = 0.0, s2 = 0.0;
    if (h->xs) {
      const double x1 = h->xs[n], x2 = h->xs[N + n];
      const double a = 0.5 * P->A * Dm, den = 1.0 + a * (P->Keq * phi + 1.0 - phi);
      const double J11 = 1.0 - a * (1.0 - phi) / den, J12 = a * P->Keq * phi / den;
      const double J21 = a * (1.0 - phi) / den, J22 = 1.0 - a * P->Keq * phi / den;
      const double det = J11 * J22 - J12 * J21;
      s1 = (J22 * x1 - J12 * x2) / det;
      s2 = (J11 * x2 - J21 * x1) / det;
    }
    for (int i = 0; i < LF->q; i++) {
      const int* c = LF->c[i];
      const double w = LF->w[i];
      double heq1 = h_eq(LF, i, c1, u);
      double heq2 = h_eq(LF, i, c2, u);
      double H1 = w * (cdot(c, dc1u) / LF->cs2 + cdot(c, nv) * 4.0 * (1.0 - phi) * c1 / P->W + M1);
      double H2 = w * (cdot(c, dc2u) / LF->cs2 - cdot(c, nv) * 4.0 * phi * c2 / P->W + M2);
      double Ht1 = -w * aux - w * s1;
      double Ht2 = w * aux - w * s2;
      double a1 = h->h1[i * N + n], a2 = h->h2[i * N + n];
      h->h1s[i * N + n] = a1 - (a1 - heq1) / tau_h1 + (1.0 - 1.0 / (2.0 * tau_h1)) * H1 + Ht1;
      h->h2s[i * N + n] = a2 - (a2 - heq2) / tau_h2 + (1.0 - 1.0 / (2.0 * tau_h2)) * H2 + Ht2;
    }
  }
}

/* -------------------------------------------------------------- pass 4 */

/* X_i(x + c_i, t+1) = X_i*(x, t); a link that leaves through a wall comes
 * back to x in the opposite direction (half-way bounce-back, resting wall).
 * For the scalar sets (k = 0: h1, 1: h2; k = -1: any other set) a Dirichlet
 * face returns -X_i*(x) + 2 w_i c_wall instead (half-way anti-bounce-back). */
static void stream_set(const cplb_ref_t* h, const lattice_t* L, const double* src, double* dst,
                       int k) {
  const long N = h->N;
  const long n3[3] = {h->nx, h->ny, h->nz};
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    long x[3];
    coords(h, n, &x[0], &x[1], &x[2]);
    for (int i = 0; i < L->q; i++) {
      long v[3];
      int face = -1;
      for (int a = 0; a < 3; a++) {
        v[a] = x[a] + L->c[i][a];
        if (v[a] < 0 || v[a] >= n3[a]) {
          if (h->p.periodic[a])
            v[a] = (v[a] + n3[a]) % n3[a];
          else if (face < 0)
            face = 2 * a + (v[a] < 0 ? 0 : 1);
        }
      }
      if (face >= 0) {
        double out = src[i * N + n];
        if (k >= 0 && h->p.scalar_bc[face] == CPLB_REF_DIRICHLET)
          out = -out + 2.0 * L->w[i] * h->p.c_wall[face][k];
        dst[L->opp[i] * N + n] = out;
      } else {
        dst[i * N + v[0] + n3[0] * (v[1] + n3[1] * v[2])] = src[i * N + n];
      }
    }
  }
}

int cplb_ref_set_closure(cplb_ref_t* h, const double* s) {
  if (!h) return CPLB_REF_EINVAL;
  h->xs = s;
  return CPLB_REF_OK;
}

int cplb_ref_step(cplb_ref_t* h, int64_t nsteps) {
  if (!h || nsteps < 0) return CPLB_REF_EINVAL;
  const long N = h->N;
  for (int64_t s = 0; s < nsteps; s++) {
    macros(h);
    collide(h);
    stream_set(h, &h->LF, h->fs, h->f, -1);
    stream_set(h, &h->LG, h->gs, h->g, -1);
    stream_set(h, &h->LF, h->h1s, h->h1, 0);
    stream_set(h, &h->LF, h->h2s, h->h2, 1);
    /* history for the next backward difference */
    memcpy(h->u_old, h->u, 3 * N * sizeof(double));
    memcpy(h->phi_old, h->phi, N * sizeof(double));
    if (h->p.scalar_model == CPLB_REF_ONE_SCALAR) {
      for (long n = 0; n < N; n++) {
        h->c1_old[n] = h->ctot[n];
        h->c2_old[n] = 0.0;
      }
    } else {
      memcpy(h->c1_old, h->c1, N * sizeof(double));
      memcpy(h->c2_old, h->c2, N * sizeof(double));
    }
    h->macros_valid = 0;
    h->step++;
  }
  return CPLB_REF_OK;
}

/* ------------------------------------------------------------ readout */

int cplb_ref_field(cplb_ref_t* h, int field, double* out) {
  if (!h || !out) return CPLB_REF_EINVAL;
  const long N = h->N;
  macros(h);
  const double* src = NULL;
  switch (field) {
    case CPLB_REF_PHI: src = h->phi; break;
    case CPLB_REF_P: src = h->pr; break;
    case CPLB_REF_UX: src = h->u; break;
    case CPLB_REF_UY: src = h->u + N; break;
    case CPLB_REF_UZ: src = h->u + 2 * N; break;
    case CPLB_REF_C1: src = h->c1; break;
    case CPLB_REF_C2: src = h->c2; break;
    case CPLB_REF_MU: src = h->mu; break;
    case CPLB_REF_PSI: src = h->psi; break;
    case CPLB_REF_GPSI_X: src = h->gpsi; break;
    case CPLB_REF_GPSI_Y: src = h->gpsi + N; break;
    case CPLB_REF_GPSI_Z: src = h->gpsi + 2 * N; break;
    default: set_err(h, "unknown field id"); return CPLB_REF_EINVAL;
  }
  memcpy(out, src, N * sizeof(double));
  return CPLB_REF_OK;
}

int cplb_ref_reduce(cplb_ref_t* h, double out[8]) {
  if (!h || !out) return CPLB_REF_EINVAL;
  const long N = h->N;
  macros(h);
  double s_phi = 0, s_c1 = 0, s_c2 = 0, s_c = 0, umax = 0, ke = 0, bad = 0;
  for (long n = 0; n < N; n++) {
    double u2 = h->u[n] * h->u[n] + h->u[N + n] * h->u[N + n] + h->u[2 * N + n] * h->u[2 * N + n];
    int finite = isfinite(h->phi[n]) && isfinite(h->c1[n]) && isfinite(h->c2[n]) && isfinite(u2) &&
                 isfinite(h->pr[n]);
    if (!finite) {
      bad += 1;
      continue;
    }
    s_phi += h->phi[n];
    s_c1 += h->c1[n];
    s_c2 += h->c2[n];
    s_c += h->ctot[n];
    if (sqrt(u2) > umax) umax = sqrt(u2);
    ke += 0.5 * h->rho[n] * u2;
  }
  out[0] = s_phi;
  out[1] = s_c1;
  out[2] = s_c2;
  out[3] = s_c;
  out[4] = umax;
  out[5] = ke;
  out[6] = bad;
  out[7] = (double)h->step;
  return bad > 0 ? CPLB_REF_EUNSTABLE : CPLB_REF_OK;
}

int cplb_ref_get_populations(cplb_ref_t* h, int set, double* out) {
  if (!h || !out) return CPLB_REF_EINVAL;
  const double* src = set == 0 ? h->f : set == 1 ? h->g : set == 2 ? h->h1 : set == 3 ? h->h2 : NULL;
  if (!src) return CPLB_REF_EINVAL;
  memcpy(out, src, (size_t)cplb_ref_population_count(h, set) * h->N * sizeof(double));
  return CPLB_REF_OK;
}

/* ---------------------------------------------------------- checkpoint */

#define REF_MAGIC 0x52454631u /* "REF1" */

typedef struct {
  uint32_t magic;
  uint32_t lattice;
  int64_t nx, ny, nz;
  int64_t step;
  cplb_ref_params prm;
} ref_header_t;

size_t cplb_ref_state_bytes(const cplb_ref_t* h) {
  if (!h) return 0;
  size_t q = (size_t)(3 * h->LF.q + h->LG.q);
  return sizeof(ref_header_t) + (q + 6) * (size_t)h->N * sizeof(double);
}

int cplb_ref_save_state(cplb_ref_t* h, void* dst, size_t bytes) {
  if (!h || !dst || bytes < cplb_ref_state_bytes(h)) return CPLB_REF_EINVAL;
  const size_t N = (size_t)h->N;
  ref_header_t hd;
  memset(&hd, 0, sizeof(hd));
  hd.magic = REF_MAGIC;
  hd.lattice = (uint32_t)h->p.lattice;
  hd.nx = h->nx;
  hd.ny = h->ny;
  hd.nz = h->nz;
  hd.step = h->step;
  hd.prm = h->p;
  char* o = (char*)dst;
  memcpy(o, &hd, sizeof(hd));
  o += sizeof(hd);
  const double* parts[] = {h->f, h->g, h->h1, h->h2, h->u_old, h->phi_old, h->c1_old, h->c2_old};
  const size_t lens[] = {h->LF.q * N, h->LG.q * N, h->LF.q * N, h->LF.q * N, 3 * N, N, N, N};
  for (int k = 0; k < 8; k++) {
    memcpy(o, parts[k], lens[k] * sizeof(double));
    o += lens[k] * sizeof(double);
  }
  return CPLB_REF_OK;
}

int cplb_ref_load_state(cplb_ref_t* h, const void* src, size_t bytes) {
  if (!h || !src || bytes < cplb_ref_state_bytes(h)) return CPLB_REF_EINVAL;
  const size_t N = (size_t)h->N;
  ref_header_t hd;
  memcpy(&hd, src, sizeof(hd));
  if (hd.magic != REF_MAGIC || hd.nx != h->nx || hd.ny != h->ny || hd.nz != h->nz ||
      (int)hd.lattice != h->p.lattice) {
    set_err(h, "checkpoint does not match this lattice");
    return CPLB_REF_ESTATE;
  }
  const char* o = (const char*)src + sizeof(hd);
  double* parts[] = {h->f, h->g, h->h1, h->h2, h->u_old, h->phi_old, h->c1_old, h->c2_old};
  const size_t lens[] = {h->LF.q * N, h->LG.q * N, h->LF.q * N, h->LF.q * N, 3 * N, N, N, N};
  for (int k = 0; k < 8; k++) {
    memcpy(parts[k], o, lens[k] * sizeof(double));
    o += lens[k] * sizeof(double);
  }
  h->step = hd.step;
  h->macros_valid = 0;
  return CPLB_REF_OK;
}
