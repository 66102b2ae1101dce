// Initialisation, field conversion and reductions.
#include "addr.hpp"
#include "kernels.hpp"

namespace pflb {

namespace {

// ------------------------------------------------------------------ init
//
// Populations are set to the equilibria of the initial fields (Sec. III),
// stored as deviations from the reference state, and the time-derivative
// history to the initial (u, phi, c1, c2).  From a
// signed distance l: phi0 = 1/2 + 1/2 tanh(2 l / W) (Sec. II A) and
// c_k = a_k + b_k phi0, u = p = 0.
template <class LF, class LG, class S, class T>
__global__ __launch_bounds__(256) void init_kernel(S* __restrict__ lat, T* __restrict__ hist,
                                                   const double* __restrict__ in_phi,
                                                   const double* __restrict__ in_c1,
                                                   const double* __restrict__ in_c2,
                                                   const double* __restrict__ in_u,
                                                   const double* __restrict__ in_p, int from_sdf,
                                                   double W, double c1a, double c1b, double c2a,
                                                   double c2b, long long n_nodes, KParams<T> P) {
  using Lay = Layout<LF, LG>;
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n_nodes) return;
  double phi, c1, c2;
  if (from_sdf) {
    phi = 0.5 + 0.5 * tanh(2.0 * in_phi[node] / W);
    c1 = c1a + c1b * phi;
    c2 = c2a + c2b * phi;
  } else {
    phi = in_phi[node];
    c1 = in_c1[node];
    c2 = in_c2[node];
  }
  if (P.one_scalar) {
    // one-scalar model: h3 carries c = c1 + c2, the history keeps c in the c1 slot
    c1 += c2;
    c2 = 0.0;
  }
  T u[3] = {0, 0, 0};
  if (in_u)
    for (int a = 0; a < LG::D; ++a) u[a] = T(in_u[a * n_nodes + node]);
  const T p = in_p ? T(in_p[node]) : T(0);
  T f[LF::Q], g[LG::Q], h1[LF::Q], h2[LF::Q];
  equilibria<LF, LG>(P, T(phi), T(c1), T(c2), u, p, f, g, h1, h2);
  // The flow population i at a node is read as coming from the node x - c_i
  // and relative to that node's pressure bracket (the node itself across a
  // wall): store it so.  g[0] is this node's bracket; a neighbour's is formed
  // from its initial p by the same arithmetic, as its own rest slot holds it.
  {
    constexpr T kpi = T((1.0 - LG::w[0]) / LG::cs2);
    const T w0 = T(LG::w[0]), inv_w0 = T(1.0 / LG::w[0]);
    const T pi_own = stored<S, T>(g[0], w0, inv_w0);
    const int n3[3] = {P.nx, P.ny, P.nz};
    const long long xyz[3] = {node % P.nx, (node / P.nx) % P.ny, node / ((long long)P.nx * P.ny)};
#pragma unroll
    for (int i = 1; i < LG::Q; ++i) {
      const int c[3] = {LG::cx[i], LG::cy[i], LG::cz[i]};
      long long src = 0, mul = 1;
      bool back = false;
      for (int a = 0; a < 3; ++a) {
        long long v = xyz[a] - c[a];
        if (v < 0 || v >= n3[a]) {
          if (P.wall[a]) back = true;
          v = v < 0 ? v + n3[a] : v - n3[a];
        }
        src += v * mul;
        mul *= n3[a];
      }
      T pi_src = pi_own;
      if (!back) pi_src = stored<S, T>((in_p ? T(in_p[src]) : T(0)) * kpi, w0, inv_w0);
      g[i] += kp<LG, T>(i) * (g[0] - pi_src);
    }
  }
  const long long st = P.stride;
  const long long pn = pitched(node, P.nx, P.px);  // the node in the planes
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    // plane skew of the push streaming (addr.hpp)
    const long long n = pn + skew_el<LF>(i);
    store_one<LF>(lat, (Lay::F0 + i) * st + n, i, f[i]);
    store_one<LF>(lat, (Lay::H10 + i) * st + n, i, h1[i]);
    store_one<LF>(lat, (Lay::H20 + i) * st + n, i, h2[i]);
  }
#pragma unroll
  for (int i = 0; i < LG::Q; ++i)
    store_one<LG>(lat, (Lay::G0 + i) * st + pn + skew_el<LG>(i), i, g[i]);
  int k = 0;
  for (int a = 0; a < LG::D; ++a) hist[(k++) * st + pn] = u[a];
  hist[(k++) * st + pn] = T(phi);
  hist[(k++) * st + pn] = T(c1);
  hist[(k++) * st + pn] = T(c2);
}

// ------------------------------------------------------------ conversion

// compact dst[i] from a plane of row pitch px
template <class T, class D>
__global__ void convert_kernel(const T* __restrict__ src, D* __restrict__ dst, long long n, int nx,
                               int px) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = D(src[pitched(i, nx, px)]);
}

// ------------------------------------------------------------- reduction
//
// Stage 1: block b reduces the contiguous node range [b*chunk, (b+1)*chunk)
// in a fixed order (per-thread strided partial sums, wavefront shuffles,
// then LDS across the 4 wavefronts) into partials[b][0..6].  Stage 2: one
// block combines the partials the same way.  No atomics: the result does not
// depend on scheduling.
constexpr int kRB = 256;

__device__ inline void wave_reduce(double (&v)[7]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const double o = __shfl_down(v[k], off, 64);
      v[k] = k == 4 ? fmax(v[k], o) : v[k] + o;
    }
  }
}

__device__ inline void block_reduce(double (&v)[7], double* __restrict__ out) {
  __shared__ double red[kRB / 64][7];
  wave_reduce(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 7; ++k) red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 7; ++k) {
      double a = red[0][k];
      for (int w = 1; w < kRB / 64; ++w) a = k == 4 ? fmax(a, red[w][k]) : a + red[w][k];
      out[k] = a;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kRB) void reduce_stage1(const T* __restrict__ fields, long long stride,
                                                     long long n, int nx, int px, double rho1,
                                                     double rho2, double* __restrict__ partials) {
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long ic = lo + threadIdx.x; ic < hi; ic += kRB) {
    const long long i = pitched(ic, nx, px);
    const double phi = fields[kFieldPhi * stride + i];
    const double c1 = fields[kFieldC1 * stride + i];
    const double c2 = fields[kFieldC2 * stride + i];
    const double ux = fields[kFieldUx * stride + i];
    const double uy = fields[kFieldUy * stride + i];
    const double uz = fields[kFieldUz * stride + i];
    const double p = fields[kFieldP * stride + i];
    const double u2 = ux * ux + uy * uy + uz * uz;
    const bool ok = finite_t(phi) && finite_t(c1) && finite_t(c2) && finite_t(u2) && finite_t(p);
    if (!ok) {
      v[6] += 1.0;
      continue;
    }
    v[0] += phi;
    v[1] += c1;
    v[2] += c2;
    v[3] += c1 + c2;
    v[4] = fmax(v[4], sqrt(u2));
    v[5] += 0.5 * (phi * (rho1 - rho2) + rho2) * u2;
  }
  block_reduce(v, partials + 8 * blockIdx.x);
}

__global__ __launch_bounds__(kRB) void reduce_stage2(const double* __restrict__ partials, int nparts,
                                                     double* __restrict__ out) {
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += kRB)
    for (int k = 0; k < 7; ++k) v[k] = k == 4 ? fmax(v[k], partials[8 * b + k]) : v[k] + partials[8 * b + k];
  block_reduce(v, out);
}

}  // namespace

template <class S, class T>
hipError_t launch_init(int dim, S* lat, T* hist, const double* phi_or_l, const double* c1,
                       const double* c2, const double* u, const double* p, int from_sdf, double W,
                       const double (&cab)[4], const KParams<T>& P, hipStream_t stream) {
  const long long n = (long long)P.nx * P.ny * P.nz;
  const int blocks = (int)((n + 255) / 256);
  if (dim == 2)
    hipLaunchKernelGGL((init_kernel<D2Q9, D2Q9, S, T>), dim3(blocks), dim3(256), 0, stream, lat, hist,
                       phi_or_l, c1, c2, u, p, from_sdf, W, cab[0], cab[1], cab[2], cab[3], n, P);
  else
    hipLaunchKernelGGL((init_kernel<D3Q7, D3Q19, S, T>), dim3(blocks), dim3(256), 0, stream, lat,
                       hist, phi_or_l, c1, c2, u, p, from_sdf, W, cab[0], cab[1], cab[2], cab[3], n, P);
  return hipGetLastError();
}

template <class T>
hipError_t launch_convert(const T* src, void* dst, int dtype, long long n, int nx, int px,
                          hipStream_t stream) {
  const int blocks = (int)((n + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL((convert_kernel<T, float>), dim3(blocks), dim3(256), 0, stream, src,
                       (float*)dst, n, nx, px);
  else
    hipLaunchKernelGGL((convert_kernel<T, double>), dim3(blocks), dim3(256), 0, stream, src,
                       (double*)dst, n, nx, px);
  return hipGetLastError();
}

template <class T>
hipError_t launch_reduce(const T* fields, long long stride, long long n, int nx, int px,
                         double rho1, double rho2, double* partials, int nparts, double* out,
                         hipStream_t stream) {
  hipLaunchKernelGGL((reduce_stage1<T>), dim3(nparts), dim3(kRB), 0, stream, fields, stride, n, nx,
                     px, rho1, rho2, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_stage2, dim3(1), dim3(kRB), 0, stream, partials, nparts, out);
  return hipGetLastError();
}

#define CPLB_INST_INIT(S, T)                                                                       \
  template hipError_t launch_init<S, T>(int, S*, T*, const double*, const double*, const double*, \
                                        const double*, const double*, int, double,                  \
                                        const double (&)[4], const KParams<T>&, hipStream_t);
CPLB_INST_INIT(double, double)
CPLB_INST_INIT(float, float)
CPLB_INST_INIT(__half, float)
CPLB_INST_INIT(__hip_bfloat16, float)

template hipError_t launch_convert<double>(const double*, void*, int, long long, int, int,
                                           hipStream_t);
template hipError_t launch_convert<float>(const float*, void*, int, long long, int, int,
                                          hipStream_t);
template hipError_t launch_reduce<double>(const double*, long long, long long, int, int, double,
                                          double, double*, int, double*, hipStream_t);
template hipError_t launch_reduce<float>(const float*, long long, long long, int, int, double,
                                         double, double*, int, double*, hipStream_t);

}  // namespace pflb
