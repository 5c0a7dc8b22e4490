// HIP kernels for the setup of the Chebyshev-accelerated (block-)Jacobi smoother: the
// power iteration that estimates the largest eigenvalue of S A on each level.
//
//   k_weyl        v_i = frac(i g) - 1/2 with g = (sqrt(5) - 1) / 2 (Weyl's equidistributed
//                 sequence; a deterministic start vector with every frequency present)
//   k_sumsq       per-workgroup partial sums of v_i^2 (FP64), re-summed in a fixed order
//                 by launch_finish, as the other reductions of the library
//   k_scale_inv   v = w / *d (device scalar)
//
// The products A v and S (A v) of the iteration reuse the SpMV and first-sweep kernels of
// the cycle (vectors of the cycle precision).
#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kChebThreads = 256;
constexpr double kWeylStep = 0.61803398874989484820;   // (sqrt(5) - 1) / 2, rounded to FP64

template <class X>
__global__ __launch_bounds__(kChebThreads) void k_weyl(int64_t n, X* __restrict__ v) {
  const int64_t i = int64_t(blockIdx.x) * kChebThreads + threadIdx.x;
  if (i >= n) return;
  const double t = double(i) * kWeylStep;
  v[i] = X(t - floor(t) - 0.5);
}

template <class X>
__global__ __launch_bounds__(kRedThreads) void k_sumsq(int64_t n, const X* __restrict__ v,
                                                       double* __restrict__ partials) {
  __shared__ double red[kRedThreads / kWave];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads) {
    const double a = double(v[i]);
    acc += a * a;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRedThreads / kWave; ++w) t += red[w];
    partials[blockIdx.x] = t;
  }
}

template <class X>
__global__ __launch_bounds__(kChebThreads) void k_scale_inv(int64_t n, X* __restrict__ v, const X* __restrict__ w,
                                                            const double* __restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * kChebThreads + threadIdx.x;
  if (i >= n) return;
  v[i] = X(double(w[i]) / *d);
}

unsigned grid_n(int64_t n) { return unsigned((n + kChebThreads - 1) / kChebThreads); }

}  // namespace

hipError_t launch_weyl(int64_t n, void* v, int xk, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (xk == X_F64) hipLaunchKernelGGL(k_weyl<double>, grid_n(n), kChebThreads, 0, s, n, static_cast<double*>(v));
  else hipLaunchKernelGGL(k_weyl<float>, grid_n(n), kChebThreads, 0, s, n, static_cast<float*>(v));
  return hipGetLastError();
}

hipError_t launch_sumsq_partials(int64_t n, const void* v, int xk, double* partials, hipStream_t s) {
  const int g = reduction_grid(n);
  if (xk == X_F64)
    hipLaunchKernelGGL(k_sumsq<double>, g, kRedThreads, 0, s, n, static_cast<const double*>(v), partials);
  else
    hipLaunchKernelGGL(k_sumsq<float>, g, kRedThreads, 0, s, n, static_cast<const float*>(v), partials);
  return hipGetLastError();
}

hipError_t launch_scale_inv(int64_t n, void* v, const void* w, int xk, const double* d, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (xk == X_F64)
    hipLaunchKernelGGL(k_scale_inv<double>, grid_n(n), kChebThreads, 0, s, n, static_cast<double*>(v),
                       static_cast<const double*>(w), d);
  else
    hipLaunchKernelGGL(k_scale_inv<float>, grid_n(n), kChebThreads, 0, s, n, static_cast<float*>(v),
                       static_cast<const float*>(w), d);
  return hipGetLastError();
}

}  // namespace mgq1
