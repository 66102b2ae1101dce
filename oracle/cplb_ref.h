/*
 * cplb_ref.h -- plain FP64 CPU oracle of the coupled phase-field lattice
 * Boltzmann step (Chen, Zhan, Chai, Shi, arXiv 2402.15752).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this library; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the GPU
 * library: its own lattice tables, its own parameter struct, its own
 * arithmetic, written as plain node loops in the order of Section III.
 *
 * Units: lattice units, dx = dt = 1.  All arrays are host memory, FP64,
 * node index n = x + nx*(y + ny*z) (x fastest).  Vector fields are passed
 * as d consecutive planes of N values (component-major).
 */
#ifndef CPLB_REF_H
#define CPLB_REF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CPLB_REF_D2Q9 = 0, CPLB_REF_D3Q19_D3Q7 = 1 };
enum { CPLB_REF_VISC_LINEAR = 0, CPLB_REF_VISC_EXP = 1 };
/* One-scalar model (Sec. II D, III D): the populations h3 of the total
 * concentration c = c1 + c2 take the place of h1 (h2 stays zero).  Fields
 * c1, c2 read back as the phase parts of c at interfacial equilibrium,
 * c1 = Keq phi c / K_eff, c2 = (1 - phi) c / K_eff, K_eff = Keq phi + 1 - phi;
 * the history keeps c in the c1 slot. */
enum { CPLB_REF_TWO_SCALAR = 0, CPLB_REF_ONE_SCALAR = 1 };
/* Scalar boundary of a wall face (Sec. IV): no flux (half-way bounce-back,
 * the default) or a Dirichlet value (half-way anti-bounce-back of h1, h2:
 * h_opp(i)(x) = -h_i*(x) + 2 w_i c_wall).  f and g bounce back at every
 * wall.  A link leaving through two walls (a corner) takes the boundary of
 * the x face, then of the y face. */
enum { CPLB_REF_NOFLUX = 0, CPLB_REF_DIRICHLET = 1 };
/* Gradient of psi = c1 + Keq c2 in the auxiliary source ~H: the isotropic
 * central stencil (the default), or the local scheme of Eq. (39), which
 * takes grad c_k from the first moment of the node's own h_k:
 *   grad c1 = [-sum c_i h1_i + c1 u - d_t(c1 u)/2 + D1 4 (1-phi) c1 n / W] / (tau_h1 cs^2)
 *   grad c2 = [-sum c_i h2_i + c2 u - d_t(c2 u)/2 - D2 4 phi c2 n / W] / (tau_h2 cs^2)
 * with u and n of the step (n from the central grad phi, which the
 * Laplacian's stencil gives anyway). */
enum { CPLB_REF_GRAD_CENTRAL = 0, CPLB_REF_GRAD_LOCAL = 1 };
enum {
  CPLB_REF_OK = 0,
  CPLB_REF_EINVAL = -1,
  CPLB_REF_ENOMEM = -2,
  CPLB_REF_EUNSTABLE = -4,
  CPLB_REF_ESTATE = -5
};
/* field ids for cplb_ref_field */
enum {
  CPLB_REF_PHI = 0, CPLB_REF_P = 1, CPLB_REF_UX = 2, CPLB_REF_UY = 3,
  CPLB_REF_UZ = 4, CPLB_REF_C1 = 5, CPLB_REF_C2 = 6, CPLB_REF_MU = 7,
  CPLB_REF_PSI = 8,
  /* the grad psi of the last step's auxiliary source (test access) */
  CPLB_REF_GPSI_X = 9, CPLB_REF_GPSI_Y = 10, CPLB_REF_GPSI_Z = 11
};

typedef struct cplb_ref_params {
  int32_t nx, ny, nz;       /* nz = 1 for the 2-D lattice                       */
  int32_t lattice;          /* CPLB_REF_D2Q9 or CPLB_REF_D3Q19_D3Q7             */
  int32_t visc_law;         /* linear law, Eq. (1.8), or exponential, Eq. (4.3) */
  int32_t periodic[3];      /* 1 periodic axis, 0 half-way bounce-back walls    */
  double rho1, rho2;        /* densities of fluid 1 (phi = 1) and fluid 2       */
  double mu1, mu2;          /* dynamic viscosities                              */
  double sigma, W, M;       /* surface tension, interface width, mobility      */
  double D1, D2, Keq, A;    /* diffusivities, partition coefficient, rate A    */
  double g[3];              /* gravity vector; body force G = (rho-rho_ref) g  */
  double rho_ref;
  double n_eps;             /* n = grad phi / sqrt(|grad phi|^2 + n_eps^2), > 0 */
  int32_t scalar_model;     /* CPLB_REF_TWO_SCALAR (h1, h2; Sec. III C) or
                               CPLB_REF_ONE_SCALAR (h3 for c = c1 + c2; Sec. III D) */
  int32_t scalar_bc[6];     /* faces x-, x+, y-, y+, z-, z+ of a walled axis:
                               CPLB_REF_NOFLUX or CPLB_REF_DIRICHLET (h1, h2)   */
  double c_wall[6][2];      /* (c1, c2) imposed at each Dirichlet face          */
  int32_t scalar_grad;      /* grad(c1 + Keq c2) of ~H: CPLB_REF_GRAD_CENTRAL or
                               CPLB_REF_GRAD_LOCAL (two-scalar model)           */
  int32_t phase_grad;       /* grad phi: CPLB_REF_GRAD_CENTRAL or CPLB_REF_GRAD_LOCAL
                               (the local scheme after Eq. (39), Sec. III C)    */
} cplb_ref_params;

typedef struct cplb_ref cplb_ref_t;

int  cplb_ref_create(const cplb_ref_params* prm, cplb_ref_t** out);
void cplb_ref_destroy(cplb_ref_t* h);
const char* cplb_ref_last_error(const cplb_ref_t* h);

/* Initial state from macroscopic fields (host, FP64, N values each; u is
 * d planes or NULL for rest, p NULL for zero).  Populations are set to the
 * equilibria of these fields and the time-derivative history to them. */
int cplb_ref_init_fields(cplb_ref_t* h, const double* phi, const double* c1,
                         const double* c2, const double* u, const double* p);
/* Initial state from a signed-distance field l (host, N values):
 * phi0 = 1/2 + 1/2 tanh(2 l / W) (Sec. II A), c_k = a_k + b_k phi0, u = p = 0. */
int cplb_ref_init_sdf(cplb_ref_t* h, const double* l, double c1_a, double c1_b,
                      double c2_a, double c2_b);

int cplb_ref_step(cplb_ref_t* h, int64_t nsteps);

/* Per-node corrections x1, x2 of c1 and c2 per step (2 N values in node
 * order, the plane of x1 then that of x2, caller-owned, NULL for none),
 * carried like the auxiliary source ~H_k: h_k loses w_i s_k, where (s1, s2)
 * solves J s = x with J the Jacobian of the node's implicit recovery of
 * (c1, c2) from (S1, S2), so that the recovered c_k drops by x_k.  Used to
 * check the learned closure's coupling into the step. */
int cplb_ref_set_closure(cplb_ref_t* h, const double* s);

/* Macroscopic field at the current time level (moments of the current
 * populations, Sec. III): writes N values. */
int cplb_ref_field(cplb_ref_t* h, int field, double* out);
/* out[0..7] = sum phi, sum c1, sum c2, sum (c1+c2), max |u|,
 *             sum rho |u|^2 / 2, count of non-finite nodes, step. */
int cplb_ref_reduce(cplb_ref_t* h, double out[8]);

/* Raw population access for tests: set in {0:f, 1:g, 2:h1, 3:h2};
 * array is Q planes of N values. */
int cplb_ref_get_populations(cplb_ref_t* h, int set, double* out);
int cplb_ref_population_count(const cplb_ref_t* h, int set);

size_t cplb_ref_state_bytes(const cplb_ref_t* h);
int cplb_ref_save_state(cplb_ref_t* h, void* dst, size_t bytes);
int cplb_ref_load_state(cplb_ref_t* h, const void* src, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif
