// C-ABI of the batch: many independent 2-D lattices advanced together.
// Validation, workspace layout, size classes, launch order and the tuner;
// all arithmetic is in the batched kernel (batch2d.hip), the init kernel and
// the read-out / reduction kernels shared with the single-lattice API.
#include <cstdarg>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/cplb.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace pflb;

namespace {

// size classes by nx, matched to the tile widths (32, 64, 128): a class's
// cases fill their last tile column well with one tile shape (64, 3 x 32,
// 128, 3 x 64, 2 x 128 nodes)
constexpr int kBatchClasses = CPLB_BATCH_CLASSES;
constexpr int kClassMaxNx[kBatchClasses] = {64, 96, 128, 192, 1 << 30};

int class_of(int nx) {
  for (int c = 0; c < kBatchClasses; ++c)
    if (nx <= kClassMaxNx[c]) return c;
  return kBatchClasses - 1;
}

// measured on MI355X for lattices of 64..256 a side (the tuner's choice on
// the 512-case sweep: 32x8, 128x4, 128x4, 256x4, 256x4); cplb_batch_tune
// refines
constexpr int kClassDefaultVariant[kBatchClasses] = {1, 3, 3, 10, 10};

struct Region {
  size_t lat, hist, fields;  // offsets in the workspace
};

struct Layout2 {
  std::vector<Region> reg;
  size_t partials, cases, k64, k32, ids, prefix, iota, single, map, total;
};

// entries of the tile maps: one (case, tile of the case) per tile of every
// case in every variant's tiling
long long map_entries(const cplb_params* prm, int n) {
  long long e = 0;
  for (int c = 0; c < n; ++c)
    for (int v = 0; v < kVariants2D; ++v) e += step2d_tiles(prm[c].nx, prm[c].ny, v);
  return e;
}

Layout2 layout(const cplb_params* prm, int n) {
  Layout2 L;
  L.reg.resize(n);
  size_t off = 0;
  for (int c = 0; c < n; ++c) {
    const Geometry G = geometry(&prm[c]);
    L.reg[c].lat = off;
    off += 2 * G.lat_bytes;
    L.reg[c].hist = off;  // two histories, alternating like the lattices
    off += 2 * G.hist_bytes;
    L.reg[c].fields = off;
    off += G.field_bytes;
  }
  L.partials = off;
  off += align_up((size_t)(kReduceBlocks + 1) * 8 * sizeof(double), kAlign);
  L.cases = off;
  off += align_up((size_t)n * sizeof(BatchCase), kAlign);
  L.k64 = off;
  off += align_up((size_t)n * sizeof(KParams<double>), kAlign);
  L.k32 = off;
  off += align_up((size_t)n * sizeof(KParams<float>), kAlign);
  L.ids = off;
  off += align_up((size_t)n * sizeof(int), kAlign);
  L.prefix = off;
  off += align_up((size_t)kBatchClasses * kVariants2D * (n + 1) * sizeof(int), kAlign);
  L.iota = off;
  off += align_up((size_t)n * sizeof(int), kAlign);
  L.single = off;
  off += align_up((size_t)2 * n * sizeof(int), kAlign);
  L.map = off;
  off += align_up((size_t)map_entries(prm, n) * 2 * sizeof(int), kAlign);
  L.total = off;
  return L;
}

int validate_batch(const cplb_params* prm, int n, char* err, size_t errn) {
  if (!prm || n < 1) {
    snprintf(err, errn, "a batch needs at least one case");
    return CPLB_EINVAL;
  }
  for (int c = 0; c < n; ++c) {
    char e[256];
    const int rc = validate(&prm[c], e, sizeof(e));
    if (rc) {
      snprintf(err, errn, "case %d: %s", c, e);
      return rc;
    }
    if (prm[c].lattice != CPLB_D2Q9) {
      snprintf(err, errn, "case %d: batches hold D2Q9 lattices only", c);
      return CPLB_EINVAL;
    }
    if (prm[c].scalar_model != CPLB_TWO_SCALAR) {
      snprintf(err, errn, "case %d: batches run the two-scalar model only", c);
      return CPLB_EINVAL;
    }
    if (prm[c].scalar_grad != CPLB_GRAD_CENTRAL) {
      snprintf(err, errn, "case %d: batches take the central gradient scheme only", c);
      return CPLB_EINVAL;
    }
    for (int f = 0; f < 6; ++f)
      if (prm[c].scalar_bc[f] != CPLB_BC_NOFLUX) {
        snprintf(err, errn, "case %d: batches take no-flux scalar walls only", c);
        return CPLB_EINVAL;
      }
    if (prm[c].precision != prm[0].precision) {
      snprintf(err, errn, "case %d: every case needs the precision of case 0", c);
      return CPLB_EINVAL;
    }
    const Geometry G = geometry(&prm[c]);
    if (!fits_u32_planes(G)) {
      snprintf(err, errn, "case %d: lattice too large for a batch (sets over 4 GiB)", c);
      return CPLB_EINVAL;
    }
  }
  return CPLB_OK;
}

}  // namespace

struct cplb_batch {
  int n;
  int precision;
  long long nodes;  // all nodes of all cases
  long long max_n;  // nodes of the largest case
  std::vector<cplb_params> prm;
  std::vector<Geometry> G;
  std::vector<KParams<double>> k64;
  std::vector<KParams<float>> k32;
  std::vector<BatchCase> cases;  // host copy of the device table
  std::vector<int> ids;          // case ids grouped by class
  std::vector<int> prefix;       // [class][variant][n + 1]
  std::vector<int> map;          // (case, tile) of every tile, per class and variant
  long long map_at[kBatchClasses][kVariants2D];  // first map entry of each
  std::vector<int> iota;         // 0, 1, ..., n - 1: one case as its own work list
  std::vector<int> single;       // per case {0, tiles of the read-out shape}
  std::vector<int> case_cls;
  int cls_first[kBatchClasses], cls_count[kBatchClasses];
  int total[kBatchClasses][kVariants2D];
  int variant[kBatchClasses];
  hipStream_t stream;
  // The size classes step on streams of their own, forked from and joined
  // back into `stream` around every call: their cases are disjoint, so one
  // class's launches fill the tail of another's.  (Library-owned, default
  // priority; null when they could not be created, and the classes then
  // take turns on `stream`.)
  hipStream_t cls_stream[kBatchClasses] = {};
  hipEvent_t fork = nullptr, join[kBatchClasses] = {};
  ~cplb_batch() {
    for (int c = 0; c < kBatchClasses; ++c) {
      if (cls_stream[c]) (void)hipStreamDestroy(cls_stream[c]);
      if (join[c]) (void)hipEventDestroy(join[c]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
  char* ws;
  double* partials;
  BatchCase* d_cases;
  KParams<double>* d_k64;
  KParams<float>* d_k32;
  int* d_ids;
  int* d_prefix;
  int* d_iota;
  int* d_single;
  int* d_map;
  int cur;
  int64_t step;
  char err[512];
};

namespace {

__attribute__((format(printf, 3, 4))) int set_err(cplb_batch_t* b, int code, const char* fmt,
                                                   ...) {
  if (b) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b->err, sizeof(b->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

int hip_check(cplb_batch_t* b, hipError_t e, const char* where) {
  if (e == hipSuccess) return CPLB_OK;
  if (b) snprintf(b->err, sizeof(b->err), "%s: %s", where, hipGetErrorString(e));
  return CPLB_EHIP;
}

size_t prefix_at(const cplb_batch_t* b, int cls, int v) {
  return ((size_t)cls * kVariants2D + v) * (b->n + 1);
}

template <class S, class T>
hipError_t launch_class(cplb_batch_t* b, int cls, int mode, int v, const KParams<T>* kdev,
                        int parity, hipStream_t stream) {
  if (b->cls_count[cls] == 0) return hipSuccess;
  const int pv = mode == kModeMacros ? 0 : v;  // the read-out uses the first tile shape
  return launch_batch2d<S, T>(b->d_cases, b->d_ids + b->cls_first[cls],
                              b->d_prefix + prefix_at(b, cls, pv), b->cls_count[cls],
                              b->d_map + 2 * b->map_at[cls][pv], b->total[cls][pv], kdev, parity,
                              mode, v, stream);
}

// one launch of class cls reading lattice `parity`, on `stream`
hipError_t run_class_on(cplb_batch_t* b, int cls, int mode, int v, int parity, hipStream_t stream) {
  switch (b->precision) {
    case CPLB_F64: return launch_class<double, double>(b, cls, mode, v, b->d_k64, parity, stream);
    case CPLB_F32: return launch_class<float, float>(b, cls, mode, v, b->d_k32, parity, stream);
    case CPLB_F32_S16F: return launch_class<__half, float>(b, cls, mode, v, b->d_k32, parity, stream);
    default: return launch_class<__hip_bfloat16, float>(b, cls, mode, v, b->d_k32, parity, stream);
  }
}

hipError_t run_class(cplb_batch_t* b, int cls, int mode, int v) {
  return run_class_on(b, cls, mode, v, b->cur, b->stream);
}

// nsteps sweeps over every class, class cls with tile variant var[cls].
// advance: the lattices alternate as in stepping (the caller flips `cur`);
// otherwise every sweep reads the current lattice and writes the idle one
// (the tuner's probes).  Each class runs on its own stream, after the work
// already on `stream` (fork) and before any that follows (join); graph
// capture of `stream` takes the class streams in through the events.
int enqueue_sweeps(cplb_batch_t* b, const int* var, int64_t nsteps, bool advance) {
  if (nsteps <= 0) return CPLB_OK;
  if (!b->fork) {
    for (int64_t k = 0; k < nsteps; ++k)
      for (int cls = 0; cls < kBatchClasses; ++cls) {
        const int par = advance ? b->cur ^ (int)(k & 1) : b->cur;
        const int rc = hip_check(b, run_class_on(b, cls, kModeStep, var[cls], par, b->stream),
                                 "batch step kernel");
        if (rc) return rc;
      }
    return CPLB_OK;
  }
  int rc = hip_check(b, hipEventRecord(b->fork, b->stream), "batch step: fork");
  for (int cls = 0; cls < kBatchClasses && !rc; ++cls) {
    if (b->cls_count[cls] == 0) continue;
    hipStream_t s = b->cls_stream[cls];
    rc = hip_check(b, hipStreamWaitEvent(s, b->fork, 0), "batch step: fork");
    for (int64_t k = 0; k < nsteps && !rc; ++k) {
      const int par = advance ? b->cur ^ (int)(k & 1) : b->cur;
      rc = hip_check(b, run_class_on(b, cls, kModeStep, var[cls], par, s), "batch step kernel");
    }
    if (!rc) rc = hip_check(b, hipEventRecord(b->join[cls], s), "batch step: join");
    if (!rc) rc = hip_check(b, hipStreamWaitEvent(b->stream, b->join[cls], 0), "batch step: join");
  }
  return rc;
}

// The field planes of one case, recomputed from its current populations on
// every read-out (a captured graph may have advanced the state unseen): the
// batched kernel in read-out mode over that case alone.
int compute_fields(cplb_batch_t* b, int icase) {
  hipError_t e;
  const int* ids = b->d_iota + icase;
  const int* pre = b->d_single + 2 * icase;
  const int tiles = step2d_tiles(b->prm[icase].nx, b->prm[icase].ny, 0);
  switch (b->precision) {
    case CPLB_F64:
      e = launch_batch2d<double, double>(b->d_cases, ids, pre, 1, nullptr, tiles, b->d_k64, b->cur,
                                         kModeMacros, 0, b->stream);
      break;
    case CPLB_F32:
      e = launch_batch2d<float, float>(b->d_cases, ids, pre, 1, nullptr, tiles, b->d_k32, b->cur,
                                       kModeMacros, 0, b->stream);
      break;
    case CPLB_F32_S16F:
      e = launch_batch2d<__half, float>(b->d_cases, ids, pre, 1, nullptr, tiles, b->d_k32, b->cur,
                                        kModeMacros, 0, b->stream);
      break;
    default:
      e = launch_batch2d<__hip_bfloat16, float>(b->d_cases, ids, pre, 1, nullptr, tiles, b->d_k32, b->cur,
                                                kModeMacros, 0, b->stream);
  }
  return hip_check(b, e, "batch macros kernel");
}

bool valid_case(const cplb_batch_t* b, int icase) { return b && icase >= 0 && icase < b->n; }

}  // namespace

extern "C" {

int cplb_batch_workspace_bytes(const cplb_params* prm, int ncases, size_t* bytes) {
  char err[512];
  if (!bytes) return CPLB_EINVAL;
  const int rc = validate_batch(prm, ncases, err, sizeof(err));
  if (rc) return rc;
  *bytes = layout(prm, ncases).total;
  return CPLB_OK;
}

int cplb_batch_create(const cplb_params* prm, int ncases, void* dev_workspace, size_t bytes,
                      void* hip_stream, cplb_batch_t** out) {
  if (!out) return CPLB_EINVAL;
  *out = nullptr;
  char err[512];
  int rc = validate_batch(prm, ncases, err, sizeof(err));
  if (rc) return rc;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign)) return CPLB_EINVAL;
  const Layout2 L = layout(prm, ncases);
  if (bytes < L.total) return CPLB_ENOMEM;
  cplb_batch_t* b = new (std::nothrow) cplb_batch_t();
  if (!b) return CPLB_ENOMEM;
  b->n = ncases;
  b->nodes = 0;
  b->max_n = 0;
  b->precision = prm[0].precision;
  b->stream = (hipStream_t)hip_stream;
  b->ws = (char*)dev_workspace;
  b->err[0] = 0;
  b->prm.assign(prm, prm + ncases);
  b->G.resize(ncases);
  b->k64.resize(ncases);
  b->k32.resize(ncases);
  b->cases.resize(ncases);
  b->case_cls.resize(ncases);
  for (int c = 0; c < ncases; ++c) {
    const Geometry G = geometry(&prm[c]);
    b->G[c] = G;
    b->k64[c] = make_kparams<double>(&prm[c], G);
    b->k32[c] = make_kparams<float>(&prm[c], G);
    BatchCase& D = b->cases[c];
    D.lat[0] = b->ws + L.reg[c].lat;
    D.lat[1] = b->ws + L.reg[c].lat + G.lat_bytes;
    D.hist[0] = b->ws + L.reg[c].hist;
    D.hist[1] = b->ws + L.reg[c].hist + G.hist_bytes;
    D.fields = b->ws + L.reg[c].fields;
    D.nx = prm[c].nx;
    D.ny = prm[c].ny;
    D.px = G.px;
    D.wall_x = prm[c].periodic[0] ? 0 : 1;
    D.wall_y = prm[c].periodic[1] ? 0 : 1;
    D.sS = (unsigned)(G.stride * G.s_pop);
    D.sT = (unsigned)(G.stride * G.s_cmp);
    D.closure = nullptr;
    D.out_off = b->nodes;
    b->nodes += G.n;
    if (G.n > b->max_n) b->max_n = G.n;
    b->case_cls[c] = class_of(prm[c].nx);
  }
  // cases grouped by class, and every class's tile prefix for every variant
  b->ids.clear();
  b->map.clear();
  b->prefix.assign((size_t)kBatchClasses * kVariants2D * (ncases + 1), 0);
  for (int cls = 0; cls < kBatchClasses; ++cls) {
    b->cls_first[cls] = (int)b->ids.size();
    for (int c = 0; c < ncases; ++c)
      if (b->case_cls[c] == cls) b->ids.push_back(c);
    b->cls_count[cls] = (int)b->ids.size() - b->cls_first[cls];
    b->variant[cls] = kClassDefaultVariant[cls];
    for (int v = 0; v < kVariants2D; ++v) {
      int* p = &b->prefix[prefix_at(b, cls, v)];
      long long acc = 0;
      for (int k = 0; k < b->cls_count[cls]; ++k) {
        p[k] = (int)acc;
        const int c = b->ids[b->cls_first[cls] + k];
        acc += step2d_tiles(prm[c].nx, prm[c].ny, v);
      }
      if (acc > (1ll << 30)) {
        delete b;
        return CPLB_EINVAL;
      }
      p[b->cls_count[cls]] = (int)acc;
      b->total[cls][v] = (int)acc;
      // the tile map: global tile g of this class and variant -> (case, tile)
      b->map_at[cls][v] = (long long)b->map.size() / 2;
      for (int k = 0; k < b->cls_count[cls]; ++k) {
        const int c = b->ids[b->cls_first[cls] + k];
        const int tiles = step2d_tiles(prm[c].nx, prm[c].ny, v);
        for (int t = 0; t < tiles; ++t) {
          b->map.push_back(c);
          b->map.push_back(t);
        }
      }
    }
  }
  b->iota.resize(ncases);
  b->single.resize(2 * (size_t)ncases);
  for (int c = 0; c < ncases; ++c) {
    b->iota[c] = c;
    b->single[2 * c] = 0;
    b->single[2 * c + 1] = step2d_tiles(prm[c].nx, prm[c].ny, 0);
  }
  b->partials = (double*)(b->ws + L.partials);
  b->d_cases = (BatchCase*)(b->ws + L.cases);
  b->d_k64 = (KParams<double>*)(b->ws + L.k64);
  b->d_k32 = (KParams<float>*)(b->ws + L.k32);
  b->d_ids = (int*)(b->ws + L.ids);
  b->d_prefix = (int*)(b->ws + L.prefix);
  b->d_iota = (int*)(b->ws + L.iota);
  b->d_single = (int*)(b->ws + L.single);
  b->d_map = (int*)(b->ws + L.map);
  b->cur = 0;
  b->step = 0;
  struct Up {
    void* dst;
    const void* src;
    size_t n;
  } ups[] = {{b->d_cases, b->cases.data(), ncases * sizeof(BatchCase)},
             {b->d_k64, b->k64.data(), ncases * sizeof(KParams<double>)},
             {b->d_k32, b->k32.data(), ncases * sizeof(KParams<float>)},
             {b->d_ids, b->ids.data(), ncases * sizeof(int)},
             {b->d_prefix, b->prefix.data(), b->prefix.size() * sizeof(int)},
             {b->d_iota, b->iota.data(), ncases * sizeof(int)},
             {b->d_single, b->single.data(), 2 * (size_t)ncases * sizeof(int)},
             {b->d_map, b->map.data(), b->map.size() * sizeof(int)}};
  for (const Up& u : ups) {
    rc = hip_check(b, hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, b->stream),
                   "upload of batch tables");
    if (rc) break;
  }
  if (!rc) rc = hip_check(b, hipStreamSynchronize(b->stream), "upload of batch tables");
  if (rc) {
    delete b;
    return rc;
  }
  // the class streams (optional: without them the classes share `stream`)
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int c = 0; c < kBatchClasses && ok; ++c)
    ok = hipStreamCreateWithFlags(&b->cls_stream[c], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    for (int c = 0; c < kBatchClasses; ++c) {
      if (b->cls_stream[c]) (void)hipStreamDestroy(b->cls_stream[c]);
      if (b->join[c]) (void)hipEventDestroy(b->join[c]);
      b->cls_stream[c] = nullptr;
      b->join[c] = nullptr;
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->fork = nullptr;
  }
  *out = b;
  return CPLB_OK;
}

void cplb_batch_destroy(cplb_batch_t* b) { delete b; }

int cplb_batch_num_cases(const cplb_batch_t* b) { return b ? b->n : 0; }

int64_t cplb_batch_step_count(const cplb_batch_t* b) { return b ? b->step : -1; }

int cplb_batch_init_sdf(cplb_batch_t* b, int icase, const double* l, double c1_a, double c1_b,
                        double c2_a, double c2_b) {
  if (!b) return CPLB_EINVAL;
  if (!valid_case(b, icase)) return set_err(b, CPLB_EINVAL, "no case %d in this batch", icase);
  if (!l) return set_err(b, CPLB_EINVAL, "signed distance array is required");
  const Geometry& G = b->G[icase];
  BatchCase& D = b->cases[icase];
  // stage the FP64 host array in the idle lattice of the case
  double* stage = (double*)D.lat[b->cur ^ 1];
  const size_t nb = (size_t)G.n * sizeof(double);
  int rc = hip_check(b, hipMemcpyAsync(stage, l, nb, hipMemcpyHostToDevice, b->stream),
                     "copy of the signed distance");
  if (rc) return rc;
  const double cab[4] = {c1_a, c1_b, c2_a, c2_b};
  const double W = b->prm[icase].W;
  void* lat = (void*)D.lat[b->cur];
  hipError_t e;
  switch (b->precision) {
    case CPLB_F64:
      e = launch_init<double, double>(2, (double*)lat, (double*)D.hist[b->cur], stage, nullptr, nullptr,
                                      nullptr, nullptr, 1, W, cab, b->k64[icase], b->stream);
      break;
    case CPLB_F32:
      e = launch_init<float, float>(2, (float*)lat, (float*)D.hist[b->cur], stage, nullptr, nullptr, nullptr,
                                    nullptr, 1, W, cab, b->k32[icase], b->stream);
      break;
    case CPLB_F32_S16F:
      e = launch_init<__half, float>(2, (__half*)lat, (float*)D.hist[b->cur], stage, nullptr, nullptr,
                                     nullptr, nullptr, 1, W, cab, b->k32[icase], b->stream);
      break;
    default:
      e = launch_init<__hip_bfloat16, float>(2, (__hip_bfloat16*)lat, (float*)D.hist[b->cur], stage, nullptr,
                                             nullptr, nullptr, nullptr, 1, W, cab, b->k32[icase],
                                             b->stream);
  }
  rc = hip_check(b, e, "init kernel");
  if (rc) return rc;
  rc = hip_check(b, hipStreamSynchronize(b->stream), "init synchronise");
  if (rc) return rc;
  return CPLB_OK;
}

int cplb_batch_init_planes(cplb_batch_t* b, const float* dev_planes, int nplanes, int iphi,
                           int ic1, int ic2) {
  if (!b) return CPLB_EINVAL;
  if (!dev_planes || nplanes < 1 || iphi < 0 || ic1 < 0 || ic2 < 0 || iphi >= nplanes ||
      ic1 >= nplanes || ic2 >= nplanes)
    return set_err(b, CPLB_EINVAL, "invalid plane layout (%d planes)", nplanes);
  const double cab[4] = {0, 0, 0, 0};
  for (int c = 0; c < b->n; ++c) {
    const Geometry& G = b->G[c];
    BatchCase& D = b->cases[c];
    double* stage = (double*)D.lat[b->cur ^ 1];  // idle lattice: 3 N doubles fit
    const float* base = dev_planes + D.out_off * nplanes;
    const int which[3] = {iphi, ic1, ic2};
    for (int k = 0; k < 3; ++k) {
      // compact planes -> compact FP64 staging (row pitch = nx: no padding)
      const int rc = hip_check(b, launch_convert<float>(base + (size_t)which[k] * G.n, stage + k * G.n,
                                                        CPLB_DTYPE_F64, G.n, b->prm[c].nx,
                                                        b->prm[c].nx, b->stream),
                               "init staging");
      if (rc) return rc;
    }
    void* lat = (void*)D.lat[b->cur];
    const double W = b->prm[c].W;
    hipError_t e;
    switch (b->precision) {
      case CPLB_F64:
        e = launch_init<double, double>(2, (double*)lat, (double*)D.hist[b->cur], stage, stage + G.n,
                                        stage + 2 * G.n, nullptr, nullptr, 0, W, cab, b->k64[c],
                                        b->stream);
        break;
      case CPLB_F32:
        e = launch_init<float, float>(2, (float*)lat, (float*)D.hist[b->cur], stage, stage + G.n,
                                      stage + 2 * G.n, nullptr, nullptr, 0, W, cab, b->k32[c],
                                      b->stream);
        break;
      case CPLB_F32_S16F:
        e = launch_init<__half, float>(2, (__half*)lat, (float*)D.hist[b->cur], stage, stage + G.n,
                                       stage + 2 * G.n, nullptr, nullptr, 0, W, cab, b->k32[c],
                                       b->stream);
        break;
      default:
        e = launch_init<__hip_bfloat16, float>(2, (__hip_bfloat16*)lat, (float*)D.hist[b->cur], stage,
                                               stage + G.n, stage + 2 * G.n, nullptr, nullptr, 0, W,
                                               cab, b->k32[c], b->stream);
    }
    const int rc = hip_check(b, e, "init kernel");
    if (rc) return rc;
  }
  return CPLB_OK;
}

int cplb_batch_step(cplb_batch_t* b, int64_t nsteps) {
  if (!b) return CPLB_EINVAL;
  if (nsteps < 0) return set_err(b, CPLB_EINVAL, "nsteps must be >= 0");
  const int rc = enqueue_sweeps(b, b->variant, nsteps, true);
  if (rc) return rc;
  b->cur ^= (int)(nsteps & 1);
  b->step += nsteps;
  return CPLB_OK;
}

int cplb_batch_read_field(cplb_batch_t* b, int icase, int field, void* dev_dst, int dtype) {
  if (!b) return CPLB_EINVAL;
  if (!valid_case(b, icase)) return set_err(b, CPLB_EINVAL, "no case %d in this batch", icase);
  if (field < 0 || field >= CPLB_NFIELDS) return set_err(b, CPLB_EINVAL, "unknown field id");
  if (dtype != CPLB_DTYPE_F32 && dtype != CPLB_DTYPE_F64)
    return set_err(b, CPLB_EINVAL, "unknown destination dtype");
  if (!dev_dst) return set_err(b, CPLB_EINVAL, "null destination");
  int rc = compute_fields(b, icase);
  if (rc) return rc;
  const Geometry& G = b->G[icase];
  const char* f = (const char*)b->cases[icase].fields + (size_t)field * G.stride * G.s_cmp;
  hipError_t e = G.s_cmp == 8
                     ? launch_convert<double>((const double*)f, dev_dst, dtype, G.n, b->prm[icase].nx,
                                              G.px, b->stream)
                     : launch_convert<float>((const float*)f, dev_dst, dtype, G.n, b->prm[icase].nx,
                                             G.px, b->stream);
  return hip_check(b, e, "field conversion");
}

int cplb_batch_reduce(cplb_batch_t* b, int icase, double out[8]) {
  if (!b || !out) return CPLB_EINVAL;
  if (!valid_case(b, icase)) return set_err(b, CPLB_EINVAL, "no case %d in this batch", icase);
  int rc = compute_fields(b, icase);
  if (rc) return rc;
  const Geometry& G = b->G[icase];
  double* dout = b->partials + 8 * kReduceBlocks;
  const int nparts = G.n < (long long)kReduceBlocks * 256 ? (int)((G.n + 255) / 256) : kReduceBlocks;
  const cplb_params& p = b->prm[icase];
  hipError_t e = G.s_cmp == 8
                     ? launch_reduce<double>((const double*)b->cases[icase].fields, G.stride, G.n,
                                             p.nx, G.px, p.rho1, p.rho2, b->partials, nparts, dout,
                                             b->stream)
                     : launch_reduce<float>((const float*)b->cases[icase].fields, G.stride, G.n,
                                            p.nx, G.px, p.rho1, p.rho2, b->partials, nparts, dout,
                                            b->stream);
  rc = hip_check(b, e, "reduction kernels");
  if (rc) return rc;
  double tmp[8];
  rc = hip_check(b, hipMemcpyAsync(tmp, dout, 7 * sizeof(double), hipMemcpyDeviceToHost, b->stream),
                 "reduction copy");
  if (rc) return rc;
  rc = hip_check(b, hipStreamSynchronize(b->stream), "reduction synchronise");
  if (rc) return rc;
  for (int k = 0; k < 7; ++k) out[k] = tmp[k];
  out[7] = (double)b->step;
  if (out[6] > 0) return set_err(b, CPLB_EUNSTABLE, "non-finite values in case %d", icase);
  return CPLB_OK;
}

int cplb_batch_set_closure(cplb_batch_t* b, const float* dev_s) {
  if (!b) return CPLB_EINVAL;
  // case c: its s1 plane then its s2 plane, from twice its node offset on
  for (int c = 0; c < b->n; ++c)
    b->cases[c].closure = dev_s ? dev_s + 2 * b->cases[c].out_off : nullptr;
  int rc = hip_check(b, hipMemcpyAsync(b->d_cases, b->cases.data(), b->n * sizeof(BatchCase),
                                       hipMemcpyHostToDevice, b->stream), "closure table upload");
  if (!rc) rc = hip_check(b, hipStreamSynchronize(b->stream), "closure table synchronise");
  return rc;
}

int64_t cplb_batch_num_nodes(const cplb_batch_t* b) { return b ? b->nodes : -1; }

int cplb_batch_gather_fields(cplb_batch_t* b, const int* fields, int nf, int nplanes,
                             float* dev_dst) {
  if (!b) return CPLB_EINVAL;
  if (!fields || nf < 1 || nf > CPLB_NFIELDS || !dev_dst)
    return set_err(b, CPLB_EINVAL, "gather needs 1..%d field ids and a destination", CPLB_NFIELDS);
  if (nplanes < nf) return set_err(b, CPLB_EINVAL, "nplanes %d below the %d fields", nplanes, nf);
  int ids[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < nf; ++k) {
    if (fields[k] < 0 || fields[k] >= CPLB_NFIELDS)
      return set_err(b, CPLB_EINVAL, "unknown field id %d", fields[k]);
    ids[k] = fields[k];
  }
  bool local = true;  // every field from the node's own moments
  for (int k = 0; k < nf; ++k)
    local = local && (ids[k] == CPLB_FIELD_PHI || ids[k] == CPLB_FIELD_C1 ||
                      ids[k] == CPLB_FIELD_C2 || ids[k] == CPLB_FIELD_PSI);
  if (local) {
    hipError_t e;
    switch (b->precision) {
      case CPLB_F64:
        e = launch_batch_gather_moments<double, double>(b->d_cases, b->d_k64, b->cur, b->n,
                                                        b->max_n, ids, nf, nplanes, dev_dst, b->stream);
        break;
      case CPLB_F32:
        e = launch_batch_gather_moments<float, float>(b->d_cases, b->d_k32, b->cur, b->n, b->max_n,
                                                      ids, nf, nplanes, dev_dst, b->stream);
        break;
      case CPLB_F32_S16F:
        e = launch_batch_gather_moments<__half, float>(b->d_cases, b->d_k32, b->cur, b->n,
                                                       b->max_n, ids, nf, nplanes, dev_dst, b->stream);
        break;
      default:
        e = launch_batch_gather_moments<__hip_bfloat16, float>(b->d_cases, b->d_k32, b->cur, b->n,
                                                               b->max_n, ids, nf, nplanes, dev_dst,
                                                               b->stream);
    }
    return hip_check(b, e, "moment gather");
  }
  for (int cls = 0; cls < kBatchClasses; ++cls) {
    const int rc = hip_check(b, run_class(b, cls, kModeMacros, 0), "batch macros kernel");
    if (rc) return rc;
  }
  const hipError_t e =
      b->precision == CPLB_F64
          ? launch_batch_gather<double>(b->d_cases, b->n, b->max_n, ids, nf, nplanes, dev_dst,
                                        b->stream)
          : launch_batch_gather<float>(b->d_cases, b->n, b->max_n, ids, nf, nplanes, dev_dst,
                                       b->stream);
  return hip_check(b, e, "field gather");
}

int cplb_batch_num_classes(const cplb_batch_t* b) { return b ? kBatchClasses : 0; }

int cplb_batch_case_class(const cplb_batch_t* b, int icase) {
  return valid_case(b, icase) ? b->case_cls[icase] : -1;
}

int cplb_batch_class_cases(const cplb_batch_t* b, int cls) {
  return b && cls >= 0 && cls < kBatchClasses ? b->cls_count[cls] : -1;
}

int cplb_batch_get_variant(const cplb_batch_t* b, int cls) {
  return b && cls >= 0 && cls < kBatchClasses ? b->variant[cls] : -1;
}

int cplb_batch_set_variant(cplb_batch_t* b, int cls, int v) {
  if (!b) return CPLB_EINVAL;
  if (cls < 0 || cls >= kBatchClasses) return set_err(b, CPLB_EINVAL, "no size class %d", cls);
  if (v < 0 || v >= kVariants2D) return set_err(b, CPLB_EINVAL, "no such kernel variant %d", v);
  b->variant[cls] = v;
  return CPLB_OK;
}

int cplb_batch_tune(cplb_batch_t* b, int probe_steps, double* ms_per_step) {
  if (!b) return CPLB_EINVAL;
  if (probe_steps < 1) return set_err(b, CPLB_EINVAL, "probe_steps must be >= 1");
  // Coordinate descent over the classes.  Every probe times the whole sweep
  // -- each class with its current variant but the one being probed --
  // because a class timed alone keeps its lattices in the Infinity Cache and
  // favours variants that lose once the other classes stream beside it.
  // The probes read the current lattices and histories and write only the
  // idle ones, so the state is left as it was.
  hipEvent_t e0, e1;
  int rc = hip_check(b, hipEventCreate(&e0), "tune: event");
  if (rc) return rc;
  rc = hip_check(b, hipEventCreate(&e1), "tune: event");
  if (rc) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  auto sweep = [&](int cls, int v) -> int {
    int var[kBatchClasses];
    for (int c = 0; c < kBatchClasses; ++c) var[c] = c == cls ? v : b->variant[c];
    return enqueue_sweeps(b, var, 1, false);
  };
  float best_ms = -1.f;
  for (int cls = 0; cls < kBatchClasses && rc == CPLB_OK; ++cls) {
    if (b->cls_count[cls] == 0) continue;
    const int keep = b->variant[cls];
    int best = keep;
    float cls_best = -1.f, keep_ms = -1.f;
    for (int v = 0; v < kVariants2D && rc == CPLB_OK; ++v) {
      rc = sweep(cls, v);  // warm-up
      if (!rc) rc = hip_check(b, hipEventRecord(e0, b->stream), "tune: record");
      for (int k = 0; k < probe_steps && rc == CPLB_OK; ++k) rc = sweep(cls, v);
      if (!rc) rc = hip_check(b, hipEventRecord(e1, b->stream), "tune: record");
      if (!rc) rc = hip_check(b, hipEventSynchronize(e1), "tune: wait");
      float ms = 0;
      if (!rc) rc = hip_check(b, hipEventElapsedTime(&ms, e0, e1), "tune: time");
      if (rc) break;
      if (v == keep) keep_ms = ms;
      if (cls_best < 0 || ms < cls_best) {
        cls_best = ms;
        best = v;
      }
    }
    // a class keeps its variant unless another beats it by more than 2%:
    // variants that differ by less than the timing noise of a few probe
    // sweeps would otherwise be picked at random
    if (rc == CPLB_OK && best != keep && keep_ms > 0 && cls_best > 0.98f * keep_ms) {
      best = keep;
      cls_best = keep_ms;
    }
    b->variant[cls] = rc == CPLB_OK ? best : keep;
    best_ms = cls_best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int rc3 = hip_check(b, hipStreamSynchronize(b->stream), "tune: synchronise");
  if (rc) return rc;
  if (rc3) return rc3;
  if (ms_per_step) *ms_per_step = best_ms > 0 ? best_ms / probe_steps : 0.0;
  return CPLB_OK;
}

const char* cplb_batch_last_error(const cplb_batch_t* b) { return b ? b->err : "null batch"; }

}  // extern "C"
