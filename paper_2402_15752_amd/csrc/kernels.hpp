// Launch entry points of the GPU kernels, called by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pflb {

constexpr int kModeStep = 0;    // collide and stream into the other lattice
constexpr int kModeMacros = 1;  // write the macroscopic fields, no update
// compiled scalar-model variants of the 2-D step: the two-scalar model, the
// one-scalar model (Sec. III D), the two-scalar model with Dirichlet faces
constexpr int kModelTwo = 0;
constexpr int kModelOne = 1;
constexpr int kModelTwoDirichlet = 2;
constexpr int kModelTwoLocal = 3;  // the two-scalar model, grad psi by Eq. (39)

// planes of the field buffer (same ids as the CPLB_FIELD_* constants)
constexpr int kFieldPhi = 0, kFieldP = 1, kFieldUx = 2, kFieldUy = 3, kFieldUz = 4, kFieldC1 = 5,
              kFieldC2 = 6, kFieldMu = 7, kFieldPsi = 8, kNumFields = 9;

// Rows of every plane are px >= nx nodes apart (the row pitch; packed,
// px = nx, by measurement); compact index i (x fastest, nx per row) -> index
// in a plane.
__host__ __device__ inline long long pitched(long long i, int nx, int px) {
  const long long r = i / nx;
  return r * px + (i - r * nx);
}

// history planes: u (d of them, stored as 3), phi, c1, c2 of the previous step
constexpr int kHist2D = 5;  // ux, uy, phi, c1, c2
constexpr int kHist3D = 6;  // ux, uy, uz, phi, c1, c2

// step kernels; `variant` picks a compiled tile shape / streaming hint
// (0 is the default; the macros mode always uses variant 0)
constexpr int kVariants2D = 12;
constexpr int kVariants3D = 10;
const char* step2d_variant_name(int v);
const char* step3d_variant_name(int v);

// closure: per-node corrections of c1 and c2 carried like the auxiliary
// scalar source (2 N FP32 values: the plane of s1, then that of s2), or null
// hin: history of the previous level (read), hout: this level's (written)
template <class S, class T>
hipError_t launch_step2d(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                         const KParams<T>* Pdev, int mode, int variant, const float* closure,
                         hipStream_t stream);

// P: host copy of the lattice constants (grid, launch shape); Pdev: the same
// constants in device memory, read by the kernel
template <class S, class T>
hipError_t launch_step3d(const S* src, S* dst, const T* hin, T* hout, T* fields, const KParams<T>& P,
                         const KParams<T>* Pdev, int mode, int variant, hipStream_t stream);

// One case of a batch of independent 2-D lattices, as the batched kernel
// reads it from device memory.
struct BatchCase {
  const void* lat[2];  // the two population lattices (parity 0 reads lat[0])
  void* hist[2];       // the two histories (parity 0 reads hist[0], writes hist[1])
  void* fields;        // field planes
  int nx, ny;
  int px;              // row pitch (nodes between two rows of a plane)
  int wall_x, wall_y;  // 1: half-way bounce-back walls on both faces
  unsigned int sS;     // bytes between two population planes
  unsigned int sT;     // bytes between two history / field planes
  const float* closure;  // per-node corrections (s1 plane, s2 plane) of this case, or null
  long long out_off;     // first value of this case in a gathered field buffer
};

// One step (or the field read-out in kModeMacros) of every case of one size
// class in a single launch: ids[0..ncls) are the class's case ids and
// prefix[0..ncls] the first tile of each in the class's tile list for
// `variant` (prefix[ncls] = total tiles); map (or null) holds (case, tile
// of the case) for every tile of that list, which spares each work-group
// the search over prefix; kps[c] are the constants of case c.  The tile
// shapes are those of the 2-D step variants.
template <class S, class T>
hipError_t launch_batch2d(const BatchCase* cases, const int* ids, const int* prefix, int ncls,
                          const int* map, int total_tiles, const KParams<T>* kps, int parity,
                          int mode, int variant, hipStream_t stream);

// tiles of an nx x ny lattice for a 2-D step variant
int step2d_tiles(int nx, int ny, int variant);

// Copy fields `ids[0..nf)` of every case (its field planes must be current)
// into dst as FP32: case c starts at dst[out_off(c) * nplanes] and holds
// nplanes >= nf planes of its N values, the first nf of them written.
// max_n: the largest N of a case.
// Gather of fields that need only the node's own moments (phi, c1, c2, psi)
// straight from the populations of the current parity.
template <class S, class T>
hipError_t launch_batch_gather_moments(const BatchCase* cases, const KParams<T>* kps, int parity,
                                       int ncases, long long max_n, const int (&ids)[9], int nf,
                                       int nplanes, float* dst, hipStream_t stream);
template <class T>
hipError_t launch_batch_gather(const BatchCase* cases, int ncases, long long max_n,
                               const int (&ids)[9], int nf, int nplanes, float* dst,
                               hipStream_t stream);

// ------------------------------------------------------- closure network
// (cnn.hip) layer l = 0..3 maps C_in = 16, 32, 32, 32 to C_out = 32, 32, 32,
// 16; activations NHWC BF16, P pixels of `rows` rows of width W, samples of
// H rows stacked.  Modes: training forward (Z in FP32 and A = act(Z) in
// BF16; the last layer linear), the adjoint of layer l (dZ of layer l in, dZ
// of layer l - 1 out), inference (A only; the last layer writes
// scale0 * channel 0 and scale1 * channel 1 to Z, which is then the
// [sample][2][H W] output).
enum { kConvForward = 0, kConvAdjoint = 2, kConvInfer = 3, kConvInferOut = 4 };
hipError_t cnn_conv(int layer, int mode, const unsigned short* X, const unsigned short* Wg,
                    const float* bias, float* Z, unsigned short* A, const float* Zprev, int H,
                    int W, int rows, float scale0, float scale1, hipStream_t s);
// weight and bias gradients of layer l over `rows` rows of width W; partial
// and bpart hold cnn_wgrad_parts(W, rows) partial sums of COUT x 9 CIN and
// COUT floats
int cnn_wgrad_parts(int W, long long rows);
hipError_t cnn_wgrad(int layer, const unsigned short* X, const unsigned short* dZ, float* partial,
                     float* bpart, int H, int W, int rows, float* gradW, float* gradb,
                     hipStream_t s);
hipError_t cnn_pack(const float* planes, int cin, const float* scale, long long hw, long long P,
                    unsigned short* X0, hipStream_t s);
// out [sample][2][hw] = scale_c * channel c of Z4, c = 0, 1
hipError_t cnn_output(const float* Z4, long long P, long long hw, float scale0, float scale1,
                      float* out, hipStream_t s);
// per sample: subtract half the mean of out[c=0] + out[c=1] from both planes;
// part holds cnn_balance_parts(nsamples) doubles
int cnn_balance_parts(int nsamples);
hipError_t cnn_balance(float* out, int nsamples, long long hw, double* part, hipStream_t s);
// block average: coarse[s][y][x] = mean of fine[s][f y + j][f x + i], 0 <= i, j < f
hipError_t cnn_restrict(const float* fine, int nsamples, int H, int W, int f, float* coarse,
                        hipStream_t s);
// mean over the two output channels of (Z4 - target)^2, target [sample][2][hw]
hipError_t cnn_loss(const float* Z4, const float* target, long long P, long long hw,
                    unsigned short* dZ4, double* partial, int nparts, double* loss, hipStream_t s);
hipError_t cnn_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float b1,
                    float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t cnn_weights(const float* W, int cin, int cout, unsigned short* Wg, unsigned short* Wf,
                       hipStream_t s);

// equilibrium initialisation from FP64 staging arrays in device memory:
// phi (or the signed distance when from_sdf), c1, c2, u (d planes) and p,
// each N values; u / p may be null.  hist receives the initial (u, phi, c1,
// c2): the history the first step reads, and the references of the stored
// populations.
template <class S, class T>
hipError_t launch_init(int dim, S* lat, T* hist, const double* phi_or_l, const double* c1,
                       const double* c2, const double* u, const double* p, int from_sdf,
                       double W, const double (&cab)[4], const KParams<T>& P, hipStream_t stream);

// convert one field plane to FP32 / FP64
template <class T>
hipError_t launch_convert(const T* src, void* dst, int dtype, long long n, int nx, int px,
                          hipStream_t stream);

// deterministic two-stage FP64 reduction of the field buffer into out[0..6]
template <class T>
hipError_t launch_reduce(const T* fields, long long stride, long long n, int nx, int px,
                         double rho1, double rho2,
                         double* partials, int nparts, double* out, hipStream_t stream);

constexpr int kReduceBlocks = 1024;

}  // namespace pflb
