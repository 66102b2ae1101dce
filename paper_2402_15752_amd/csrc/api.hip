// C-ABI of libcplb.so: parameter validation, workspace layout, launch order.
// The per-step work is entirely in the HIP kernels; this layer only
// validates, carves the caller's workspace and enqueues on the caller's
// stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/cplb.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace pflb;


struct cplb {
  cplb_params prm;
  Geometry G;
  hipStream_t stream;
  char* ws;
  void* lat[2];
  void* hist[2];  // histories, alternating with the lattices: hist[cur] goes with lat[cur]
  void* fields;
  double* partials;
  double* scratch_dev;  // this device's copy of `scratch` (cplb_reduce_device)
  int cur;
  int64_t step;
  int variant;  // compiled step-kernel variant in use
  const float* closure;  // caller's per-node corrections of c1, c2 (2-D), or null
  KParams<double> k64;  // lattice constants (host copies)
  KParams<float> k32;
  KParams<double>* k64_dev;  // the same, in the workspace, read by the step kernels
  KParams<float>* k32_dev;
  char err[512];
};

// Reduction partials of cplb_reduce_device: a fixed array of the library
// instead of the handle's workspace, so that call allocates nothing.  One
// copy per GPU (kReduceBlocks per-block partials of 8 doubles, 64 KiB), held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel -- on the host it only names the symbol -- but the device address
// that hipGetSymbolAddress returns for the current device.
constexpr int kScratchParts = kReduceBlocks;
static __device__ __align__(256) double scratch[8 * kScratchParts];

namespace {

std::mutex scratch_mu;
void* scratch_addr[64];  // device address of `scratch` per device ordinal, once looked up

// address of this device's `scratch`, looked up once per device with that
// device current (cplb_create)
hipError_t scratch_address(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[dev] = p;
  }
  *out = (double*)scratch_addr[dev];
  return hipSuccess;
}

int set_err(cplb_t* h, int code, const char* fmt, const char* a = "") {
  if (h) snprintf(h->err, sizeof(h->err), fmt, a);
  return code;
}

int hip_check(cplb_t* h, hipError_t e, const char* where) {
  if (e == hipSuccess) return CPLB_OK;
  if (h) snprintf(h->err, sizeof(h->err), "%s: %s", where, hipGetErrorString(e));
  return CPLB_EHIP;
}

template <class S, class T>
hipError_t dispatch_step(cplb_t* h, const KParams<T>& K, const KParams<T>* Kdev, int mode) {
  const S* src = (const S*)h->lat[h->cur];
  S* dst = (S*)h->lat[h->cur ^ 1];
  const T* hin = (const T*)h->hist[h->cur];
  T* hout = (T*)h->hist[h->cur ^ 1];
  if (h->G.dim == 2)
    return launch_step2d<S, T>(src, dst, hin, hout, (T*)h->fields, K, Kdev, mode, h->variant,
                               h->closure, h->stream);
  return launch_step3d<S, T>(src, dst, hin, hout, (T*)h->fields, K, Kdev, mode, h->variant,
                             h->stream);
}

int num_variants(const cplb_t* h) { return h->G.dim == 2 ? kVariants2D : kVariants3D; }

// Default step-kernel variant per lattice, storage width and gradient scheme:
// the fastest measured on MI355X for the rising bubble (D2Q9, 256 x 1024 and
// 2048 x 4096) and the rising droplet (256^3) with the skewed plane layout
// (aligned push stores, so non-temporal stores pay off beyond the Infinity
// Cache); cplb_tune re-checks on the caller's own state.
int default_variant(const cplb_params* p) {
  if (p->lattice == CPLB_D2Q9) {
    // 128x4; a lattice beyond the 256 MB Infinity Cache streams faster on
    // 256x4 tiles (runs of 256 nodes per plane stream) with non-temporal
    // stores and cached loads (256x4 nt-st): at 2048 x 4096 FP32 570 us
    // against 599 (128x4 nt-st) and 629 (128x4) for the central stencil,
    // 536 against 555 and 571 for the local scheme; with cached loads the
    // halo re-reads hit L2 (1.00x the algorithmic read bytes against 1.07x
    // and 1.26x with non-temporal loads)
    const int s_pop = p->precision == CPLB_F64 ? 8 : (p->precision == CPLB_F32 ? 4 : 2);
    const double lattice_bytes = (double)p->nx * p->ny * 36.0 * s_pop;
    return lattice_bytes > 256e6 ? 11 : 3;
  }
  // 3-D: non-temporal stores, f, h1, h2 carried from the previous plane.
  // FP32: 128x4 tiles (one 8-wave work-group per CU; rows of 128 nodes, so
  // every plane stream of a tile moves 512-byte runs: 1.23 against 1.29 ms
  // per 256^3 step with 64x4).  16-bit storage: 64x4 tiles, with the central
  // stencil for grad psi the carry in LDS, which takes the flow collision
  // from two to three waves per SIMD (0.89 against 1.01 ms; 128x4 tiles
  // 0.97), with the local scheme in registers (0.78 ms; LDS 0.79, 128x4
  // 0.90).  FP64: 64x4 (its registers do not fit an 8-wave group).  The
  // variant that re-reads f, h1, h2 before their collision is slower, and 41%
  // of its re-reads miss L2 (1.41 x the algorithmic read bytes).
  // (128-wide tiles only where they leave no more idle columns than 64-wide
  // ones: nx a multiple of 128, or more than 64 past one)
  if (p->precision == CPLB_F32 && (p->nx % 128 == 0 || p->nx % 128 > 64)) return 9;
  const bool s16 = p->precision == CPLB_F32_S16F || p->precision == CPLB_F32_S16B;
  return s16 && p->scalar_grad != CPLB_GRAD_LOCAL ? 8 : 4;
}

hipError_t run_kernel(cplb_t* h, int mode) {
  switch (h->prm.precision) {
    case CPLB_F64: return dispatch_step<double, double>(h, h->k64, h->k64_dev, mode);
    case CPLB_F32: return dispatch_step<float, float>(h, h->k32, h->k32_dev, mode);
    case CPLB_F32_S16F: return dispatch_step<__half, float>(h, h->k32, h->k32_dev, mode);
    default: return dispatch_step<__hip_bfloat16, float>(h, h->k32, h->k32_dev, mode);
  }
}

// The field buffer is recomputed from the current populations on every
// read-out: steps may also advance the state from a captured graph, which
// the host does not see, so no host-side flag can tell whether it is stale.
int compute_fields(cplb_t* h) { return hip_check(h, run_kernel(h, kModeMacros), "macros kernel"); }

// host FP64 arrays -> staging area (the idle lattice) -> equilibrium init
int do_init(cplb_t* h, const double* a, const double* c1, const double* c2, const double* u,
            const double* p, int from_sdf, const double (&cab)[4]) {
  const size_t nb = (size_t)h->G.n * sizeof(double);
  const int d = h->G.dim;
  char* stage = (char*)h->lat[1];
  size_t need = nb * (from_sdf ? 1 : (3 + (u ? d : 0) + (p ? 1 : 0)));
  if (need > h->G.lat_bytes) return set_err(h, CPLB_ENOMEM, "staging area too small");
  size_t off = 0;
  auto put = [&](const double* src, size_t bytes) -> const double* {
    if (!src) return nullptr;
    double* dst = (double*)(stage + off);
    off += bytes;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream) != hipSuccess)
      return (const double*)-1;
    return dst;
  };
  const double* da = put(a, nb);
  const double* dc1 = from_sdf ? nullptr : put(c1, nb);
  const double* dc2 = from_sdf ? nullptr : put(c2, nb);
  const double* du = from_sdf ? nullptr : put(u, nb * d);
  const double* dp = from_sdf ? nullptr : put(p, nb);
  const double* bad = (const double*)-1;
  if (da == bad || dc1 == bad || dc2 == bad || du == bad || dp == bad)
    return hip_check(h, hipGetLastError(), "copy of initial fields");
  h->cur = 0;
  const double W = h->prm.W;
  hipError_t e;
  switch (h->prm.precision) {
    case CPLB_F64:
      e = launch_init<double, double>(d, (double*)h->lat[0], (double*)h->hist[0], da, dc1, dc2, du, dp,
                                      from_sdf, W, cab, h->k64, h->stream);
      break;
    case CPLB_F32:
      e = launch_init<float, float>(d, (float*)h->lat[0], (float*)h->hist[0], da, dc1, dc2, du, dp,
                                    from_sdf, W, cab, h->k32, h->stream);
      break;
    case CPLB_F32_S16F:
      e = launch_init<__half, float>(d, (__half*)h->lat[0], (float*)h->hist[0], da, dc1, dc2, du, dp,
                                     from_sdf, W, cab, h->k32, h->stream);
      break;
    default:
      e = launch_init<__hip_bfloat16, float>(d, (__hip_bfloat16*)h->lat[0], (float*)h->hist[0], da,
                                             dc1, dc2, du, dp, from_sdf, W, cab, h->k32, h->stream);
  }
  int rc = hip_check(h, e, "init kernel");
  if (rc) return rc;
  rc = hip_check(h, hipStreamSynchronize(h->stream), "init synchronise");
  if (rc) return rc;
  h->step = 0;
  return CPLB_OK;
}

// "CLP3": lattices with the skewed plane layout of the push streaming, f, h1,
// h2 relative to the history of the node they are stored at
constexpr uint32_t kStateMagic = 0x33504C43u;

struct StateHeader {
  uint32_t magic, abi;
  int64_t step;
  cplb_params prm;
};

}  // namespace

extern "C" {

int cplb_workspace_bytes(const cplb_params* prm, size_t* bytes) {
  char err[256];
  if (!bytes) return CPLB_EINVAL;
  int rc = validate(prm, err, sizeof(err));
  if (rc) return rc;
  *bytes = geometry(prm).total;
  return CPLB_OK;
}

int cplb_create(const cplb_params* prm, void* dev_workspace, size_t bytes, void* hip_stream,
                cplb_t** out) {
  if (!out) return CPLB_EINVAL;
  *out = nullptr;
  char err[256];
  int rc = validate(prm, err, sizeof(err));
  if (rc) return rc;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign)) return CPLB_EINVAL;
  Geometry G = geometry(prm);
  if (bytes < G.total) return CPLB_ENOMEM;
  cplb_t* h = new (std::nothrow) cplb_t();
  if (!h) return CPLB_ENOMEM;
  h->prm = *prm;
  h->G = G;
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char*)dev_workspace;
  size_t off = 0;
  h->lat[0] = h->ws + off;
  off += G.lat_bytes;
  h->lat[1] = h->ws + off;
  off += G.lat_bytes;
  h->hist[0] = h->ws + off;
  off += G.hist_bytes;
  h->hist[1] = h->ws + off;
  off += G.hist_bytes;
  h->fields = h->ws + off;
  off += G.field_bytes;
  h->partials = (double*)(h->ws + off);
  off += G.part_bytes;
  h->k64_dev = (KParams<double>*)(h->ws + off);
  off += align_up(sizeof(KParams<double>), kAlign);
  h->k32_dev = (KParams<float>*)(h->ws + off);
  h->cur = 0;
  h->step = 0;
  h->variant = default_variant(prm);
  h->closure = nullptr;
  h->k64 = make_kparams<double>(prm, G);
  h->k32 = make_kparams<float>(prm, G);
  h->err[0] = 0;
  rc = hip_check(h, scratch_address(&h->scratch_dev), "lookup of the reduction scratch array");
  if (rc) {
    delete h;
    return rc;
  }
  rc = hip_check(h, hipMemcpyAsync(h->k64_dev, &h->k64, sizeof(h->k64), hipMemcpyHostToDevice,
                                   h->stream), "upload of lattice constants");
  if (!rc)
    rc = hip_check(h, hipMemcpyAsync(h->k32_dev, &h->k32, sizeof(h->k32), hipMemcpyHostToDevice,
                                     h->stream), "upload of lattice constants");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "upload of lattice constants");
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return CPLB_OK;
}

void cplb_destroy(cplb_t* h) { delete h; }

int cplb_init_fields(cplb_t* h, const double* phi, const double* c1, const double* c2,
                     const double* u, const double* p) {
  if (!h) return CPLB_EINVAL;
  if (!phi || !c1 || !c2) return set_err(h, CPLB_EINVAL, "phi, c1 and c2 are required");
  const double cab[4] = {0, 0, 0, 0};
  return do_init(h, phi, c1, c2, u, p, 0, cab);
}

int cplb_init_sdf(cplb_t* h, const double* l, double c1_a, double c1_b, double c2_a, double c2_b) {
  if (!h) return CPLB_EINVAL;
  if (!l) return set_err(h, CPLB_EINVAL, "signed distance array is required");
  const double cab[4] = {c1_a, c1_b, c2_a, c2_b};
  return do_init(h, l, nullptr, nullptr, nullptr, nullptr, 1, cab);
}

int cplb_step(cplb_t* h, int64_t nsteps) {
  if (!h) return CPLB_EINVAL;
  if (nsteps < 0) return set_err(h, CPLB_EINVAL, "nsteps must be >= 0");
  for (int64_t s = 0; s < nsteps; ++s) {
    int rc = hip_check(h, run_kernel(h, kModeStep), "step kernel");
    if (rc) return rc;
    h->cur ^= 1;
    h->step++;
  }
  return CPLB_OK;
}

int64_t cplb_step_count(const cplb_t* h) { return h ? h->step : -1; }

int cplb_read_field(cplb_t* h, int field, void* dev_dst, int dtype) {
  if (!h) return CPLB_EINVAL;
  if (field < 0 || field >= CPLB_NFIELDS) return set_err(h, CPLB_EINVAL, "unknown field id");
  if (dtype != CPLB_DTYPE_F32 && dtype != CPLB_DTYPE_F64)
    return set_err(h, CPLB_EINVAL, "unknown destination dtype");
  if (!dev_dst) return set_err(h, CPLB_EINVAL, "null destination");
  int rc = compute_fields(h);
  if (rc) return rc;
  hipError_t e;
  if (h->G.s_cmp == 8)
    e = launch_convert<double>((const double*)h->fields + field * h->G.stride, dev_dst, dtype, h->G.n,
                               h->prm.nx, h->G.px, h->stream);
  else
    e = launch_convert<float>((const float*)h->fields + field * h->G.stride, dev_dst, dtype, h->G.n,
                              h->prm.nx, h->G.px, h->stream);
  return hip_check(h, e, "field conversion");
}

int cplb_reduce(cplb_t* h, double out[8]) {
  if (!h || !out) return CPLB_EINVAL;
  int rc = compute_fields(h);
  if (rc) return rc;
  double* dout = h->partials + 8 * kReduceBlocks;
  const int nparts = h->G.n < (long long)kReduceBlocks * 256 ? (int)((h->G.n + 255) / 256) : kReduceBlocks;
  hipError_t e;
  if (h->G.s_cmp == 8)
    e = launch_reduce<double>((const double*)h->fields, h->G.stride, h->G.n, h->prm.nx, h->G.px,
                              h->prm.rho1, h->prm.rho2, h->partials, nparts, dout, h->stream);
  else
    e = launch_reduce<float>((const float*)h->fields, h->G.stride, h->G.n, h->prm.nx, h->G.px,
                             h->prm.rho1, h->prm.rho2, h->partials, nparts, dout, h->stream);
  rc = hip_check(h, e, "reduction kernels");
  if (rc) return rc;
  double tmp[8];
  rc = hip_check(h, hipMemcpyAsync(tmp, dout, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                 "reduction copy");
  if (rc) return rc;
  rc = hip_check(h, hipStreamSynchronize(h->stream), "reduction synchronise");
  if (rc) return rc;
  for (int k = 0; k < 7; ++k) out[k] = tmp[k];
  out[7] = (double)h->step;
  if (out[6] > 0) return set_err(h, CPLB_EUNSTABLE, "non-finite values in %s fields", "the");
  return CPLB_OK;
}

int cplb_reduce_device(cplb_t* h, double* dev_out) {
  if (!h) return CPLB_EINVAL;
  if (!dev_out) return set_err(h, CPLB_EINVAL, "null device destination%s", "");
  const int nparts = h->G.n < (long long)kReduceBlocks * 256 ? (int)((h->G.n + 255) / 256) : kReduceBlocks;
  if (nparts > kScratchParts)
    return set_err(h, CPLB_ENOMEM, "%s: more reduction partials than the fixed array holds",
                   "cplb_reduce_device");
  if (!h->scratch_dev) return set_err(h, CPLB_EHIP, "reduction scratch array not available%s", "");
  int rc = compute_fields(h);
  if (rc) return rc;
  hipError_t e;
  if (h->G.s_cmp == 8)
    e = launch_reduce<double>((const double*)h->fields, h->G.stride, h->G.n, h->prm.nx, h->G.px,
                              h->prm.rho1, h->prm.rho2, h->scratch_dev, nparts, dev_out, h->stream);
  else
    e = launch_reduce<float>((const float*)h->fields, h->G.stride, h->G.n, h->prm.nx, h->G.px,
                             h->prm.rho1, h->prm.rho2, h->scratch_dev, nparts, dev_out, h->stream);
  return hip_check(h, e, "reduction kernels");
}

size_t cplb_state_bytes(const cplb_t* h) {
  if (!h) return 0;
  return sizeof(StateHeader) + (size_t)h->G.qtot * h->G.cells * h->G.s_pop +
         (size_t)h->G.nhist * h->G.cells * h->G.s_cmp;
}

int cplb_save_state(cplb_t* h, void* host_dst, size_t bytes) {
  if (!h || !host_dst) return CPLB_EINVAL;
  if (bytes < cplb_state_bytes(h)) return set_err(h, CPLB_ENOMEM, "checkpoint buffer too small");
  int rc = hip_check(h, hipStreamSynchronize(h->stream), "checkpoint synchronise");
  if (rc) return rc;
  StateHeader hd{};
  hd.magic = kStateMagic;
  hd.abi = CPLB_ABI_VERSION;
  hd.step = h->step;
  hd.prm = h->prm;
  char* o = (char*)host_dst;
  memcpy(o, &hd, sizeof(hd));
  o += sizeof(hd);
  // whole planes of cells (nodes and row padding), from node 0 of each
  const size_t pb = (size_t)h->G.cells * h->G.s_pop, hb = (size_t)h->G.cells * h->G.s_cmp;
  for (int q = 0; q < h->G.qtot; ++q, o += pb) {
    const long long first = q * h->G.stride + plane_skew_el(h->G.dim, q);  // node 0 of plane q
    rc = hip_check(h, hipMemcpy(o, (char*)h->lat[h->cur] + first * h->G.s_pop, pb,
                                hipMemcpyDeviceToHost), "checkpoint copy");
    if (rc) return rc;
  }
  for (int k = 0; k < h->G.nhist; ++k, o += hb) {
    rc = hip_check(h, hipMemcpy(o, (char*)h->hist[h->cur] + k * h->G.stride * h->G.s_cmp, hb,
                                hipMemcpyDeviceToHost), "checkpoint copy");
    if (rc) return rc;
  }
  return CPLB_OK;
}

int cplb_load_state(cplb_t* h, const void* host_src, size_t bytes) {
  if (!h || !host_src) return CPLB_EINVAL;
  if (bytes < cplb_state_bytes(h)) return set_err(h, CPLB_ESTATE, "checkpoint buffer too small");
  StateHeader hd;
  memcpy(&hd, host_src, sizeof(hd));
  if (hd.magic != kStateMagic || hd.abi != CPLB_ABI_VERSION ||
      !same_params(hd.prm, h->prm))
    return set_err(h, CPLB_ESTATE, "checkpoint was written for other parameters%s", "");
  int rc = hip_check(h, hipStreamSynchronize(h->stream), "restore synchronise");
  if (rc) return rc;
  const char* o = (const char*)host_src + sizeof(hd);
  // whole planes of cells (nodes and row padding), from node 0 of each
  const size_t pb = (size_t)h->G.cells * h->G.s_pop, hb = (size_t)h->G.cells * h->G.s_cmp;
  h->cur = 0;
  for (int q = 0; q < h->G.qtot; ++q, o += pb) {
    const long long first = q * h->G.stride + plane_skew_el(h->G.dim, q);  // node 0 of plane q
    rc = hip_check(h, hipMemcpy((char*)h->lat[0] + first * h->G.s_pop, o, pb,
                                hipMemcpyHostToDevice), "restore copy");
    if (rc) return rc;
  }
  for (int k = 0; k < h->G.nhist; ++k, o += hb) {
    rc = hip_check(h, hipMemcpy((char*)h->hist[0] + k * h->G.stride * h->G.s_cmp, o, hb,
                                hipMemcpyHostToDevice), "restore copy");
    if (rc) return rc;
  }
  h->step = hd.step;
  return CPLB_OK;
}

int cplb_set_closure(cplb_t* h, const float* dev_s) {
  if (!h) return CPLB_EINVAL;
  if (h->G.dim != 2 && dev_s) return set_err(h, CPLB_EINVAL, "a closure applies to D2Q9 lattices%s", "");
  if (h->prm.scalar_model != CPLB_TWO_SCALAR && dev_s)
    return set_err(h, CPLB_EINVAL, "a closure applies to the two-scalar model%s", "");
  h->closure = dev_s;
  return CPLB_OK;
}

int cplb_num_variants(const cplb_t* h) { return h ? num_variants(h) : 0; }

int cplb_get_variant(const cplb_t* h) { return h ? h->variant : -1; }

const char* cplb_variant_name(const cplb_t* h, int v) {
  if (!h) return "?";
  return h->G.dim == 2 ? step2d_variant_name(v) : step3d_variant_name(v);
}

int cplb_set_variant(cplb_t* h, int v) {
  if (!h) return CPLB_EINVAL;
  if (v < 0 || v >= num_variants(h)) return set_err(h, CPLB_EINVAL, "no such kernel variant%s", "");
  h->variant = v;
  return CPLB_OK;
}

int cplb_tune(cplb_t* h, int probe_steps, double* ms_per_step) {
  if (!h) return CPLB_EINVAL;
  if (probe_steps < 1) return set_err(h, CPLB_EINVAL, "probe_steps must be >= 1%s", "");
  // The probes read the current lattice and history and write only the idle
  // ones, which are scratch: the state is left as it was.
  hipEvent_t e0, e1;
  int rc = hip_check(h, hipEventCreate(&e0), "tune: event");
  if (rc) return rc;
  rc = hip_check(h, hipEventCreate(&e1), "tune: event");
  if (rc) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  const int keep = h->variant;
  int best = keep;
  float best_ms = 0;
  for (int v = 0; v < num_variants(h) && rc == CPLB_OK; ++v) {
    h->variant = v;
    rc = hip_check(h, run_kernel(h, kModeStep), "tune: warm-up");  // first launch loads code
    if (rc) break;
    rc = hip_check(h, hipEventRecord(e0, h->stream), "tune: record");
    for (int k = 0; k < probe_steps && rc == CPLB_OK; ++k)
      rc = hip_check(h, run_kernel(h, kModeStep), "tune: probe");
    if (rc) break;
    rc = hip_check(h, hipEventRecord(e1, h->stream), "tune: record");
    if (rc) break;
    rc = hip_check(h, hipEventSynchronize(e1), "tune: wait");
    if (rc) break;
    float ms = 0;
    rc = hip_check(h, hipEventElapsedTime(&ms, e0, e1), "tune: time");
    if (rc) break;
    if (v == 0 || ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->variant = rc == CPLB_OK ? best : keep;
  const int rc2 = hip_check(h, hipStreamSynchronize(h->stream), "tune: synchronise");
  if (rc) return rc;
  if (rc2) return rc2;
  if (ms_per_step) *ms_per_step = best_ms / probe_steps;
  return CPLB_OK;
}

const char* cplb_last_error(const cplb_t* h) { return h ? h->err : "null handle"; }

const char* cplb_strerror(int code) {
  switch (code) {
    case CPLB_OK: return "ok";
    case CPLB_EINVAL: return "invalid parameters or arguments";
    case CPLB_ENOMEM: return "workspace or buffer too small";
    case CPLB_EHIP: return "HIP runtime error";
    case CPLB_EUNSTABLE: return "non-finite values (unstable run)";
    case CPLB_ESTATE: return "checkpoint does not match this lattice";
    default: return "unknown error code";
  }
}

}  // extern "C"
