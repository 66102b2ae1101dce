/*
 * cplb.h -- C-ABI of the MI355X coupled phase-field lattice Boltzmann library
 * (libcplb.so).
 *
 * The library advances, on one GPU, the four coupled population sets of the
 * phase-field LB method of Chen, Zhan, Chai & Shi (arXiv 2402.15752):
 *   f        conservative Allen-Cahn phase field          (Sec. III A)
 *   g        pressure-based incompressible flow           (Sec. III B)
 *   h1, h2   two-scalar concentration / temperature model
 *            with source H_k and auxiliary source ~H_k     (Sec. III C)
 * on D2Q9 (all four sets) or D3Q19 (g and the stencils) + D3Q7 (f, h1, h2).
 *
 * Units are lattice units (dx = dt = 1).  Node index n = x + nx*(y + ny*z),
 * x fastest.  Host arrays are FP64, N = nx*ny*nz values per scalar field and
 * d consecutive planes of N values per vector field.
 *
 * Conventions
 *  - Ownership: the caller owns the device workspace and the HIP stream and
 *    keeps both alive until cplb_destroy.  The library owns the layout of the
 *    workspace and the launch order.  Host arrays passed in are only read
 *    during the call; device destinations are written asynchronously.
 *  - Ordering: every call is ordered on the stream given at create.
 *    cplb_init_*, cplb_reduce, cplb_save_state and cplb_load_state
 *    synchronise that stream before returning.
 *  - Errors: calls never abort and never throw across the ABI; they return
 *    one of the CPLB_* codes below.  cplb_last_error gives the text of the
 *    last failure on a handle.
 *  - Threading: a handle is not thread-safe; any number of handles may exist.
 */
#ifndef CPLB_H
#define CPLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPLB_ABI_VERSION 1

/* return codes */
#define CPLB_OK 0
#define CPLB_EINVAL (-1)    /* bad parameters or arguments                     */
#define CPLB_ENOMEM (-2)    /* workspace or host buffer too small              */
#define CPLB_EHIP (-3)      /* HIP runtime error (text in cplb_last_error)     */
#define CPLB_EUNSTABLE (-4) /* a reduction saw a non-finite field value        */
#define CPLB_ESTATE (-5)    /* checkpoint does not match this lattice          */

/* lattices */
#define CPLB_D2Q9 0       /* D2Q9 for f, g, h1, h2 and the 9-point stencils       */
#define CPLB_D3Q19_D3Q7 1 /* D3Q19 for g and 19-point stencils, D3Q7 for f, h1, h2 */

/* arithmetic and population storage */
#define CPLB_F64 0      /* FP64 compute, FP64 populations                            */
#define CPLB_F32 1      /* FP32 compute, FP32 populations                            */
#define CPLB_F32_S16F 2 /* FP32 compute, populations stored as FP16 of dX_i / w_i     */
#define CPLB_F32_S16B 3 /* FP32 compute, populations stored as BF16 of dX_i / w_i     */

/* viscosity laws */
#define CPLB_VISC_LINEAR 0 /* mu = phi (mu1 - mu2) + mu2, Eq. (1.8)            */
#define CPLB_VISC_EXP 1    /* log mu = c1 log mu1 + c2 log mu2, Eq. (4.3)      */

/* scalar transport models (cplb_params.scalar_model)
 * CPLB_TWO_SCALAR: c1, c2 carried by h1, h2 with the exchange and auxiliary
 *   sources (Sec. II C, III C).
 * CPLB_ONE_SCALAR: the total c = c1 + c2 carried by one set h3 (Sec. II D,
 *   III D): h3_0^eq = c + (w0 - 1) c / K_eff, h3_i^eq = w_i c / K_eff +
 *   w_i c_i.(c u) / cs^2, source w_i c_i.d_t(c u) / cs^2, per-node
 *   tau_h3 = 1/2 + D_eff / cs^2 with D_eff = D1 Keq phi + D2 (1 - phi) and
 *   K_eff = Keq phi + 1 - phi.  CPLB_D2Q9 single lattices only (the batch and
 *   the 3-D lattice take the two-scalar model).  h3 occupies the h1 planes;
 *   the h2 planes are neither read nor written.  Fields c1, c2 read back as
 *   the phase parts of c at interfacial equilibrium, c1 = Keq phi c / K_eff,
 *   c2 = (1 - phi) c / K_eff; init takes c = c1 + c2.  Stable for
 *   K_eff >= 1 - w0 = 5/9 (the rest equilibrium stays non-negative). */
#define CPLB_TWO_SCALAR 0
#define CPLB_ONE_SCALAR 1

/* Scalar boundary of a wall face (cplb_params.scalar_bc, Sec. IV): no flux
 * (half-way bounce-back, the default) or a Dirichlet value (half-way
 * anti-bounce-back of h1, h2: h_opp(i)(x) = -h_i*(x) + 2 w_i c_wall, the
 * value imposed half a node outside the boundary node).  f and g bounce back
 * at every wall.  A link leaving through two walls (a corner) takes the
 * boundary of the x face.  Dirichlet faces need a walled axis, the
 * CPLB_D2Q9 lattice and the two-scalar model. */
#define CPLB_BC_NOFLUX 0
#define CPLB_BC_DIRICHLET 1

/* Gradient of psi = c1 + Keq c2 in the auxiliary source ~H_k
 * (cplb_params.scalar_grad): the isotropic central stencil (Sec. III C, the
 * default), or the local scheme of Eq. (39), which takes grad c_k from the
 * first moment of the node's own h_k,
 *   grad c1 = [-sum c_i h1_i + c1 u - d_t(c1 u)/2 + D1 4 (1-phi) c1 n / W] / (tau_h1 cs^2),
 *   grad c2 = [-sum c_i h2_i + c2 u - d_t(c2 u)/2 - D2 4 phi c2 n / W] / (tau_h2 cs^2),
 * with u and n of the step.  The local scheme needs no psi stencil, so the
 * step reads no h1, h2 of the halo.  The two-scalar model and no-flux
 * scalar walls only; single lattices (not batches). */
#define CPLB_GRAD_CENTRAL 0
#define CPLB_GRAD_LOCAL 1

/* field ids for cplb_read_field */
#define CPLB_FIELD_PHI 0
#define CPLB_FIELD_P 1
#define CPLB_FIELD_UX 2
#define CPLB_FIELD_UY 3
#define CPLB_FIELD_UZ 4
#define CPLB_FIELD_C1 5
#define CPLB_FIELD_C2 6
#define CPLB_FIELD_MU 7
#define CPLB_FIELD_PSI 8 /* c1 + Keq c2 */
#define CPLB_NFIELDS 9

/* destination types for cplb_read_field */
#define CPLB_DTYPE_F32 0
#define CPLB_DTYPE_F64 1

typedef struct cplb_params {
  int32_t nx, ny, nz;    /* grid; nz = 1 on CPLB_D2Q9                            */
  int32_t lattice;       /* CPLB_D2Q9 | CPLB_D3Q19_D3Q7                          */
  int32_t precision;     /* CPLB_F64 | CPLB_F32 | CPLB_F32_S16F | CPLB_F32_S16B  */
  int32_t visc_law;      /* CPLB_VISC_LINEAR | CPLB_VISC_EXP                     */
  int32_t periodic[3];   /* per axis: 1 periodic, 0 half-way bounce-back walls   */
  int32_t scalar_model;  /* CPLB_TWO_SCALAR (0) | CPLB_ONE_SCALAR (1)             */
  double rho1, rho2;     /* densities of fluid 1 (phi = 1) and fluid 2 (Sec. II B) */
  double mu1, mu2;       /* viscosities of the two fluids (or the exp-law bases) */
  double sigma;          /* surface tension: beta = 12 sigma/W, k = 3 sigma W/2  */
  double W;              /* interface width                                      */
  double M;              /* Allen-Cahn mobility, M = (tau_f - 1/2) cs^2          */
  double D1, D2;         /* diffusivities, D_k = (tau_hk - 1/2) cs^2             */
  double Keq;            /* partition (Henry / heat-capacity) coefficient        */
  double A;              /* exchange rate parameter, 1/length^2                  */
  double g[3];           /* gravity; body force G = (rho - rho_ref) g            */
  double rho_ref;        /* reference density of the body force                  */
  double n_eps;          /* normal n = grad phi / sqrt(|grad phi|^2 + n_eps^2)   */
  double ref[4];         /* uniform references of the stored scalar populations:
                            where h1, h2 have no per-node reference (one-scalar
                            model, local gradient scheme) they are held as
                            X_i - w_i ref[k] (k = 2, 3: c1_ref, c2_ref).  f, and
                            h1, h2 otherwise, are held relative to the moments of
                            the node they are stored at, g relative to a pressure
                            bracket, so ref[0] has no effect; ref[1] must be 0 */
  int32_t scalar_bc[6];  /* faces x-, x+, y-, y+, z-, z+ of a walled axis:
                            CPLB_BC_NOFLUX or CPLB_BC_DIRICHLET (h1, h2)          */
  double c_wall[6][2];   /* (c1, c2) imposed at each Dirichlet face              */
  int32_t scalar_grad;   /* grad(c1 + Keq c2) of ~H: CPLB_GRAD_CENTRAL | CPLB_GRAD_LOCAL */
  int32_t phase_grad;    /* grad phi: CPLB_GRAD_CENTRAL (the isotropic stencil) or
                            CPLB_GRAD_LOCAL (the local scheme after Eq. (39), Sec.
                            III C: from the first moment of the node's own f, with
                            the previous step's velocity standing in for this
                            step's, which needs grad phi); the Laplacian is central
                            either way */
} cplb_params;

typedef struct cplb cplb_t; /* opaque handle */

/* Device workspace, in bytes, that cplb_create needs for these parameters.
 * Returns CPLB_EINVAL for invalid parameters (same checks as cplb_create). */
int cplb_workspace_bytes(const cplb_params* prm, size_t* bytes);

/* Validate the parameters and carve the caller's device workspace
 * (dev_workspace, at least cplb_workspace_bytes, 256-byte aligned) into the
 * two population lattices, the time-derivative history, the field buffer and
 * the reduction partials.  hip_stream is a hipStream_t (NULL = null stream).
 * Every relaxation time must exceed 1/2: M, D1, D2 > 0 (Sec. III); rho_k,
 * mu_k, W, Keq, n_eps > 0; sigma, A >= 0; nx, ny, nz >= 1 and >= 2 on a
 * walled axis; on CPLB_D2Q9 nz = 1 and g[2] = 0.
 * Errors: CPLB_EINVAL, CPLB_ENOMEM (workspace too small), CPLB_EHIP. */
int cplb_create(const cplb_params* prm, void* dev_workspace, size_t bytes, void* hip_stream,
                cplb_t** out);

/* Initial state from host fields phi, c1, c2 (N values each), u (d planes of
 * N, or NULL for rest) and p (N values, or NULL for 0): every population is
 * set to its equilibrium (Sec. III A-C) and the time-derivative history to
 * these fields; the step counter restarts at 0.  Synchronises the stream. */
int cplb_init_fields(cplb_t* h, const double* phi, const double* c1, const double* c2,
                     const double* u, const double* p);

/* Initial state from a host signed-distance field l (N values):
 * phi0 = 1/2 + 1/2 tanh(2 l / W) (Sec. II A), c_k = a_k + b_k phi0, u = p = 0.
 * Synchronises the stream. */
int cplb_init_sdf(cplb_t* h, const double* l, double c1_a, double c1_b, double c2_a,
                  double c2_b);

/* Advance nsteps >= 0 time steps (one fused collide-and-stream launch per
 * step: moments, stencils, flow macros, viscosity law, collision of f, g,
 * h1, h2 with F_i, G_i, H_k, ~H_k, streaming with periodic wrap or half-way
 * bounce-back).  Asynchronous on the stream. */
int cplb_step(cplb_t* h, int64_t nsteps);

/* Write macroscopic field `field` (CPLB_FIELD_*) at the current time level --
 * the moments of the current populations, as they enter the next collision
 * -- to dev_dst (device memory, N values of CPLB_DTYPE_F32 or _F64).
 * Asynchronous on the stream. */
int cplb_read_field(cplb_t* h, int field, void* dev_dst, int dtype);

/* FP64 reductions over the current time level, deterministic order:
 * out[0] sum phi, out[1] sum c1, out[2] sum c2, out[3] sum (c1 + c2),
 * out[4] max |u|, out[5] sum rho |u|^2 / 2, out[6] number of nodes with a
 * non-finite phi, c1, c2, u or p, out[7] step counter.
 * Synchronises the stream; returns CPLB_EUNSTABLE if out[6] > 0. */
int cplb_reduce(cplb_t* h, double out[8]);

/* Allocation-free form of cplb_reduce, for callers that cannot allocate or
 * synchronise (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation): the same FP64 values out[0..6], bit for bit, written
 * asynchronously on the stream to dev_out (device memory, caller-owned, at
 * least 7 doubles; dev_out[7] is not written -- the step counter is host
 * state, see cplb_step_count).  The per-block partials go to a fixed array
 * of the library (1024 partials of 8 doubles, 64 KiB per GPU, held until the
 * process ends) instead of the handle's workspace; the call allocates
 * nothing and does not synchronise, and it does not return CPLB_EUNSTABLE
 * (it does not see the values: dev_out[6] counts the non-finite nodes).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (different streams, no ordering between them) race.
 * Errors: CPLB_EINVAL (null handle or dev_out), CPLB_ENOMEM (more partials
 * than the array holds), CPLB_EHIP. */
int cplb_reduce_device(cplb_t* h, double* dev_out);

/* Number of steps taken since the last init or load. */
int64_t cplb_step_count(const cplb_t* h);

/* Checkpoint: raw current populations, history, step counter and a copy of
 * the parameters, into / from a caller-owned host buffer of
 * cplb_state_bytes bytes.  A resumed run is bitwise identical to an
 * uninterrupted one.  Both synchronise the stream.  load returns
 * CPLB_ESTATE if the buffer was written for other parameters. */
size_t cplb_state_bytes(const cplb_t* h);
int cplb_save_state(cplb_t* h, void* host_dst, size_t bytes);
int cplb_load_state(cplb_t* h, const void* host_src, size_t bytes);

/* Learned closure on a D2Q9 lattice: dev_s (device, 2 N FP32 values: the
 * plane of x1 in node order, then that of x2; owned by the caller and kept
 * alive while set) holds per-node corrections of c1 and c2 per step: each
 * step lowers the recovered c_k of the node by x_k.  They are carried like
 * the auxiliary source ~H_k (Sec. III C), h_k losing w_i s_k with (s1, s2)
 * = J^-1 (x1, x2), J the Jacobian of the implicit recovery of c1, c2 at the
 * node (exact where phi and D_m do not change over the step).  x1 = -x2 is
 * a pure exchange (c1 + c2 conserved node by node); in general the total
 * scalar drops by sum (x1 + x2) per step (the network's inference makes it
 * zero per case).  NULL switches it off.  CPLB_EINVAL on a 3-D lattice or
 * with the one-scalar model. */
int cplb_set_closure(cplb_t* h, const float* dev_s);

/* Step-kernel variants (tile shape, non-temporal population traffic).
 * Every variant computes the same step; they differ only in how the work is
 * tiled and how the population streams are hinted to the caches.
 * cplb_tune times each compiled variant for probe_steps launches on the
 * current state and keeps the fastest; the state is left as it was (the
 * probes write only the idle lattice, the history is saved and restored).
 * It synchronises the stream; *ms_per_step (may be NULL) receives the best
 * time per step.  cplb_set_variant returns CPLB_EINVAL for an unknown id. */
int cplb_num_variants(const cplb_t* h);
int cplb_get_variant(const cplb_t* h);
int cplb_set_variant(cplb_t* h, int variant);
const char* cplb_variant_name(const cplb_t* h, int variant);
int cplb_tune(cplb_t* h, int probe_steps, double* ms_per_step);

/* ------------------------------------------------------------------------
 * Batches: many independent 2-D lattices (CPLB_D2Q9), each with its own
 * grid, boundaries and parameters, advanced together -- the parameter
 * sweeps of the paper's transfer studies (Sec. IV) run as one job.  A step
 * runs one kernel launch per size class (cases grouped by nx into
 * CPLB_BATCH_CLASSES classes, each with its own tile-shape variant from
 * the 2-D variant table); each launch covers every tile of every case of
 * its class.  Every case evolves bit-identically to the same case run alone
 * with cplb_create / cplb_step.  All cases share the precision of case 0.
 * The caller owns the workspace and the stream as for a single lattice;
 * icase numbers cases in the order of prm[].  Errors as above.
 */
#define CPLB_BATCH_CLASSES 5 /* size classes: nx <= 64, 96, 128, 192, larger */

typedef struct cplb_batch cplb_batch_t;

/* Device workspace for ncases >= 1 cases with parameters prm[0..ncases).
 * CPLB_EINVAL for an invalid case (the checks of cplb_create, plus:
 * CPLB_D2Q9 and the two-scalar model only, same precision as case 0). */
int cplb_batch_workspace_bytes(const cplb_params* prm, int ncases, size_t* bytes);

/* Validate every case, carve the workspace (256-byte aligned, at least
 * cplb_batch_workspace_bytes) and upload the case tables.  Synchronises. */
int cplb_batch_create(const cplb_params* prm, int ncases, void* dev_workspace, size_t bytes,
                      void* hip_stream, cplb_batch_t** out);

/* Initial state of one case from a host signed-distance field (N values of
 * that case), as cplb_init_sdf.  Synchronises the stream. */
int cplb_batch_init_sdf(cplb_batch_t* b, int icase, const double* l, double c1_a, double c1_b,
                        double c2_a, double c2_b);

/* Initial state of every case from device FP32 planes in the layout of
 * cplb_batch_gather_fields (nplanes planes per case; planes iphi, ic1, ic2
 * hold phi, c1, c2; u = p = 0): equilibria and history as cplb_init_fields.
 * Asynchronous. */
int cplb_batch_init_planes(cplb_batch_t* b, const float* dev_planes, int nplanes, int iphi,
                           int ic1, int ic2);

/* Advance every case nsteps >= 0 steps.  Asynchronous; a caller may capture
 * the launches in a HIP graph.  The size classes run on streams the batch
 * creates for itself (default priority, destroyed with the batch), forked
 * from the caller's stream and joined back into it by events, so the call
 * is ordered on the caller's stream like every other. */
int cplb_batch_step(cplb_batch_t* b, int64_t nsteps);

int cplb_batch_num_cases(const cplb_batch_t* b);
int64_t cplb_batch_step_count(const cplb_batch_t* b);

/* Field of one case at the current level, as cplb_read_field. */
int cplb_batch_read_field(cplb_batch_t* b, int icase, int field, void* dev_dst, int dtype);

/* Reductions of one case, as cplb_reduce (out[7] = batch step counter). */
int cplb_batch_reduce(cplb_batch_t* b, int icase, double out[8]);

/* Nodes of all cases together (the length of a per-node batch buffer). */
int64_t cplb_batch_num_nodes(const cplb_batch_t* b);

/* Learned closure for every case (as cplb_set_closure): dev_s (device, FP32)
 * holds, case after case, each case's s1 plane then its s2 plane (2 x
 * cplb_batch_num_nodes values in all); NULL switches it off.  The buffer
 * stays the caller's; its contents may change between steps.  Synchronises. */
int cplb_batch_set_closure(cplb_batch_t* b, const float* dev_s);

/* Fields fields[0..nf) (CPLB_FIELD_*) of every case at the current level
 * into dev_dst (device, FP32).  Case c owns nplanes >= nf planes of its N
 * values, starting at nplanes times the number of nodes of the cases
 * before it; its first nf planes are written, the others left as they are
 * (room for planes the caller fills once).  Asynchronous. */
int cplb_batch_gather_fields(cplb_batch_t* b, const int* fields, int nf, int nplanes,
                             float* dev_dst);

/* Size classes: number, class of a case, cases in a class, and the 2-D
 * step variant (cplb_variant_name of a D2Q9 lattice names it) each class
 * runs; set_variant returns CPLB_EINVAL for an unknown class or variant. */
int cplb_batch_num_classes(const cplb_batch_t* b);
int cplb_batch_case_class(const cplb_batch_t* b, int icase);
int cplb_batch_class_cases(const cplb_batch_t* b, int cls);
int cplb_batch_get_variant(const cplb_batch_t* b, int cls);
int cplb_batch_set_variant(cplb_batch_t* b, int cls, int variant);

/* Autotuner: class after class, time every variant of the class within the
 * whole sweep (the other classes at their current variants) for
 * probe_steps sweeps on the current state, and keep the fastest (the
 * current variant stays unless another is faster by more than 2%).  The state
 * is left as it was (probes write only the idle lattices and histories).
 * Synchronises; *ms_per_step (may be NULL) receives the time per sweep of
 * the final choice. */
int cplb_batch_tune(cplb_batch_t* b, int probe_steps, double* ms_per_step);

const char* cplb_batch_last_error(const cplb_batch_t* b);

/* Release the batch (not the caller's workspace or stream).  Does not wait:
 * synchronise the stream before freeing or reusing the workspace. */
void cplb_batch_destroy(cplb_batch_t* b);

/* ------------------------------------------------------------------------
 * Closure network: the small CNN that predicts the per-node corrections
 * (s1, s2) of c1 and c2 per step on a coarse grid from its fields (applied
 * through cplb_set_closure / cplb_batch_set_closure).  Fixed architecture:
 * four 3x3 correlations 16 -> 32 -> 32 -> 32 -> 16 channels, leaky-ReLU
 * (slope 0.1) after the first three, outputs = channels 0 and 1 of the
 * last; padding periodic along x, zero outside each sample along y.  BF16
 * MFMA with FP32 accumulation for every convolution, FP32 master
 * parameters, FP64 loss accumulation.  The parameter vector stacks per
 * layer W[co][ci][ky][kx] then b[co] (cplb_cnn_num_params values).
 * Samples are H x W planes; up to `nsamples` are processed at once.
 */
typedef struct cplb_cnn cplb_cnn_t;

int cplb_cnn_num_params(void);
int cplb_cnn_workspace_bytes(int nsamples, int H, int W, size_t* bytes);
int cplb_cnn_create(int nsamples, int H, int W, void* dev_workspace, size_t bytes, void* hip_stream,
                    cplb_cnn_t** out);

/* Parameters: set from / get to a host array of cplb_cnn_num_params FP32
 * values (setting resets the Adam state); init draws He-normal weights
 * (std sqrt(2 / (9 C_in)), a tenth of it on the last layer) and zero biases
 * from a seeded generator.  All synchronise. */
int cplb_cnn_set_params(cplb_cnn_t* c, const float* host_theta);
int cplb_cnn_init_params(cplb_cnn_t* c, uint64_t seed);
int cplb_cnn_get_params(cplb_cnn_t* c, float* host_theta);

/* Input plane k is multiplied by scale[k] before the first layer (host
 * array of 16; default 1).  Synchronises. */
int cplb_cnn_set_input_scale(cplb_cnn_t* c, const float scale[16]);

/* Forward pass of nsamples samples: dev_planes (device) holds
 * [nsamples][cin][H][W] FP32, cin <= 16 (missing planes are zero); dev_out
 * (device, may be NULL) receives [nsamples][2][H][W] FP32: the two output
 * channels times their output scales, then balanced per sample (half the
 * sample's mean of s1 + s2 taken from both planes, so that the corrections
 * add nothing to the sample's total scalar).  Asynchronous. */
int cplb_cnn_forward(cplb_cnn_t* c, int nsamples, const float* dev_planes, int cin, float* dev_out);

/* Inference: the forward pass without the FP32 pre-activations the
 * backward pass needs (activations in BF16 only, the output scaled and
 * written by the last convolution, then balanced).  dev_out (device)
 * receives [nsamples][2][H][W] FP32, bitwise equal to cplb_cnn_forward's
 * output.  A
 * following cplb_cnn_backward needs a cplb_cnn_forward first.  No host
 * synchronisation and no allocation: capturable in a HIP graph.
 * Asynchronous. */
int cplb_cnn_infer(cplb_cnn_t* c, int nsamples, const float* dev_planes, int cin, float* dev_out);

/* Stream of every following call (hip_stream is a hipStream_t); the caller
 * orders it after work already queued on the previous stream. */
int cplb_cnn_set_stream(cplb_cnn_t* c, void* hip_stream);

/* Loss mean((z - target)^2) of the last forward's two output channels z
 * (before output scale and balance) against dev_target ([nsamples][2][H][W]
 * FP32, device), the mean over both channels and every pixel, accumulated
 * in FP64, and the gradient of every parameter (FP32).  *loss (may be NULL)
 * receives the loss; with it the call synchronises. */
int cplb_cnn_backward(cplb_cnn_t* c, const float* dev_target, double* loss);
int cplb_cnn_get_grads(cplb_cnn_t* c, float* host_grad);

/* One Adam step on the last gradients (bias-corrected), then the BF16
 * weight copies are refreshed.  Asynchronous. */
int cplb_cnn_adam(cplb_cnn_t* c, float lr, float beta1, float beta2, float eps);

/* Output channel k (the correction of c_k) is multiplied by scale_k
 * (default 1): the network is trained on targets divided by them. */
int cplb_cnn_set_output_scale(cplb_cnn_t* c, float scale1, float scale2);

/* Block average of nsamples fine planes (H f x W f each, device FP32) onto
 * coarse planes (H x W, device FP32): the restriction of fine-grid fields
 * to the coarse grid.  Asynchronous on hip_stream. */
int cplb_cnn_restrict(void* hip_stream, const float* dev_fine, int nsamples, int H, int W, int f,
                      float* dev_coarse);

const char* cplb_cnn_last_error(const cplb_cnn_t* c);
/* Release the network (not the caller's workspace or stream); does not wait
 * for queued work. */
void cplb_cnn_destroy(cplb_cnn_t* c);

/* Error text of the last failed call on h, and of a return code. */
const char* cplb_last_error(const cplb_t* h);
const char* cplb_strerror(int code);

/* Release the handle (not the caller's workspace or stream).  Does not wait
 * for work queued on the stream: synchronise it before freeing or reusing the
 * workspace. */
void cplb_destroy(cplb_t* h);

#ifdef __cplusplus
}
#endif
#endif
