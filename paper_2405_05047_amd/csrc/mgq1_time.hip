// HIP kernels of the time-stepping driver (Algorithm "Nonstationary Linear Problem",
// Sec. 4): the matrices stay on the device for every step, and each step forms its
// right-hand side on the GPU from the previous state by the lumped mass of eq.
// mass_lumping, solves, and maps the free unknowns back to nodal values.
//
//   k_time_rhs    b = R [theta / dt + f ; g], R = [Z H^T M_l | -Z H^T A E_g] (scalar CSR;
//                 the concatenated vector is formed per entry, never stored)
//   k_time_theta  theta = H x, then the Dirichlet values g on the Dirichlet DoFs
//
// Both are one pass over a short-row CSR matrix (1-3 entries per row on uniform meshes,
// a few more next to hanging nodes and the Dirichlet boundary) plus the vectors: a few
// percent of one V-cycle's bytes, so one thread per row with ordinary loads is enough
// (neighbouring rows are neighbours in memory, so a wave's loads share cache lines).
// Entries are summed in their stored (column) order with one rounding per product and
// per sum, as a sequential CSR product does.
#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kTimeThreads = 256;

__global__ __launch_bounds__(kTimeThreads) void k_time_rhs(int32_t n, int32_t n_free, const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ theta,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ g, double dt,
                                                           double* __restrict__ b) {
  const int32_t i = int32_t(blockIdx.x) * kTimeThreads + int32_t(threadIdx.x);
  if (i >= n) return;
  const int32_t k0 = rowptr[i], k1 = rowptr[i + 1];
  double s = 0.0;
  for (int32_t k = k0; k < k1; ++k) {
    const int32_t j = col[k];
    // columns below n_free address theta / dt + f, the others the Dirichlet values
    const double v = j < n_free ? theta[j] / dt + f[j] : g[j - n_free];
    const double p = val[k] * v;
    s = s + p;
  }
  b[i] = s;
}

__global__ __launch_bounds__(kTimeThreads) void k_time_theta(int32_t n, const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val,
                                                             const int32_t* __restrict__ gpos,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ g,
                                                             double* __restrict__ theta) {
  const int32_t i = int32_t(blockIdx.x) * kTimeThreads + int32_t(threadIdx.x);
  if (i >= n) return;
  const int32_t q = gpos[i];
  if (q >= 0) {
    theta[i] = g[q];
    return;
  }
  const int32_t k0 = rowptr[i], k1 = rowptr[i + 1];
  double s = 0.0;
  for (int32_t k = k0; k < k1; ++k) {
    const double p = val[k] * x[col[k]];
    s = s + p;
  }
  theta[i] = s;
}

unsigned grid_rows(int32_t n) { return unsigned((int64_t(n) + kTimeThreads - 1) / kTimeThreads); }

}  // namespace

hipError_t launch_time_rhs(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                           const double* theta, const double* f, const double* g, double dt, double* b,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_rhs, grid_rows(n), kTimeThreads, 0, s, n, n, rowptr, col, val, theta, f, g, dt, b);
  return hipGetLastError();
}

hipError_t launch_time_theta(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                             const int32_t* gpos, const double* x, const double* g, double* theta,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_theta, grid_rows(n), kTimeThreads, 0, s, n, rowptr, col, val, gpos, x, g, theta);
  return hipGetLastError();
}

}  // namespace mgq1
