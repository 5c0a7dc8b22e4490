// HIP kernels of the explicit pressure-correction step (Sec. 5.3, Algorithm "The fully
// discrete solution procedure for the Navier-Stokes equations"):
//
//   k_ns_momentum   Step 1 for every velocity node (one lane per node, its 3 components):
//                   the nodal products u_a u_c of eq. tp are formed from the gathered
//                   neighbour velocities inside the C_a products of eq. multC, the
//                   viscous product K u_c shares the same pass over the 27-entry rows
//                   (K, C_x, C_y, C_z stored together), the pressure term G_c (p + q) is
//                   the second pass of the same lane, then the lumped-mass inverse and the
//                   Dirichlet values: one kernel where the paper runs a custom product
//                   kernel, three SpMVs, a rectangular product and a diagonal scaling.
//   k_ns_divergence D u = sum_a G_a^T u_a per pressure node (pull-style rows of D = G^T,
//                   no atomics; a slice's slot range split over the four waves of a
//                   workgroup, partial sums added in a fixed order), and the Poisson
//                   right-hand side -(1/k) D u (0 on pinned nodes); D u is kept for Step 3.
//   k_ns_pressure   Step 3: p + q - nu D u / m_p.
//
// Matrices are sliced ELL over rows: one slice = 64 rows = one wavefront, slot k of the
// slice holds one entry per row (column col[k*64 + lane], values val[(k*V + v)*64 + lane]
// for the V value arrays), so every index and value load of a wave is one contiguous
// stream; padding entries carry the row's own column and zero values.  All work is
// bandwidth-bound (about 0.1 flop per byte): no matrix cores.
#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kNsThreads = 256;   // 4 slices per workgroup
constexpr int kNsBatch = 8;       // slots whose loads are issued together (one round trip)

__device__ __forceinline__ int64_t slice_of(int lane_block) { return int64_t(blockIdx.x) * (kNsThreads / kWave) + lane_block; }

__global__ __launch_bounds__(kNsThreads) void k_ns_momentum(NsEll V, NsEll G, const double* __restrict__ u,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ q,
                                                             const double* __restrict__ f,
                                                             const double* __restrict__ m_v,
                                                             const uint8_t* __restrict__ dmask,
                                                             const double* __restrict__ dval, double nu, double k,
                                                             double* __restrict__ uo) {
  const int lane = int(threadIdx.x) % kWave;
  const int64_t s = slice_of(int(threadIdx.x) / kWave);
  if (s >= V.nslices) return;
  const int64_t row = s * kWave + lane;
  const bool valid = row < V.nrows;
  double visc[3] = {0.0, 0.0, 0.0}, conv[3] = {0.0, 0.0, 0.0}, pres[3] = {0.0, 0.0, 0.0};
  // viscous and convective terms over the velocity row
  // slots in batches of kNsBatch: the index and value loads of a batch first, then its
  // gathers, then the sums in slot order (the remainder slots one at a time)
  const int32_t v0 = V.sptr[s], v1 = V.sptr[s + 1];
  auto vslot = [&](const double (&m)[4], const double (&uj)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      visc[c] += m[0] * uj[c];
      // eq. tp: the nodal products u_a u_c of neighbour j, inside eq. multC
      const double t0 = m[1] * (uj[0] * uj[c]);
      const double t1 = m[2] * (uj[1] * uj[c]);
      const double t2 = m[3] * (uj[2] * uj[c]);
      conv[c] += t0 + t1 + t2;
    }
  };
  int32_t t = v0;
  for (; t + kNsBatch <= v1; t += kNsBatch) {
    int32_t j[kNsBatch];
    double m[kNsBatch][4], uj[kNsBatch][3];
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) {
      j[b] = V.col[int64_t(t + b) * kWave + lane];
#pragma unroll
      for (int a = 0; a < 4; ++a) m[b][a] = V.val[(int64_t(t + b) * 4 + a) * kWave + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) uj[b][c] = u[int64_t(j[b]) * 3 + c];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) vslot(m[b], uj[b]);
  }
  for (; t < v1; ++t) {
    const int32_t j = V.col[int64_t(t) * kWave + lane];
    double m[4], uj[3];
#pragma unroll
    for (int a = 0; a < 4; ++a) m[a] = V.val[(int64_t(t) * 4 + a) * kWave + lane];
#pragma unroll
    for (int c = 0; c < 3; ++c) uj[c] = u[int64_t(j) * 3 + c];
    vslot(m, uj);
  }
  // pressure term G_c (p + q)
  const int32_t g0 = G.sptr[s], g1 = G.sptr[s + 1];
  t = g0;
  for (; t + kNsBatch <= g1; t += kNsBatch) {
    int32_t j[kNsBatch];
    double g[kNsBatch][3], sv[kNsBatch];
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) {
      j[b] = G.col[int64_t(t + b) * kWave + lane];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[b][c] = G.val[(int64_t(t + b) * 3 + c) * kWave + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) sv[b] = p[j[b]] + q[j[b]];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) pres[c] += g[b][c] * sv[b];
  }
  for (; t < g1; ++t) {
    const int32_t j = G.col[int64_t(t) * kWave + lane];
    const double sv = p[j] + q[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) pres[c] += G.val[(int64_t(t) * 3 + c) * kWave + lane] * sv;
  }
  if (!valid) return;
  const double m = m_v[row];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t d = row * 3 + c;
    if (dmask[d]) {
      uo[d] = dval[d];
    } else {
      const double fc = f ? f[d] : 0.0;
      const double rhs = m * (fc + u[d] / k) - nu * visc[c] + conv[c] + pres[c];
      uo[d] = k * rhs / m;
    }
  }
}

// D has few rows (one per pressure node) of many slots (up to 125 on the Q1-iso-Q2 pair),
// so one workgroup takes one slice: its kNsSplit waves sum consecutive quarters of the
// slot range, and the partial sums are added in wave order (a fixed order, no atomics)
constexpr int kNsSplit = kNsThreads / kWave;

__global__ __launch_bounds__(kNsThreads) void k_ns_divergence(NsEll D, const double* __restrict__ u,
                                                               const uint8_t* __restrict__ pin, double k,
                                                               double* __restrict__ du, double* __restrict__ rhs) {
  __shared__ double part[kNsSplit][kWave];
  const int lane = int(threadIdx.x) % kWave, w = int(threadIdx.x) / kWave;
  const int64_t s = blockIdx.x;
  if (s >= D.nslices) return;                      // whole workgroup: the barrier below is safe
  const int64_t row = s * kWave + lane;
  const int32_t s0 = D.sptr[s], s1 = D.sptr[s + 1];
  const int32_t per = (s1 - s0 + kNsSplit - 1) / kNsSplit;
  const int32_t t0 = std::min(s1, s0 + w * per), t1 = std::min(s1, t0 + per);
  double acc = 0.0;
  int32_t t = t0;
  for (; t + kNsBatch <= t1; t += kNsBatch) {
    int64_t j[kNsBatch];
    double d[kNsBatch][3], uj[kNsBatch][3];
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) {
      j[b] = D.col[int64_t(t + b) * kWave + lane];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[b][c] = D.val[(int64_t(t + b) * 3 + c) * kWave + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) uj[b][c] = u[j[b] * 3 + c];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kNsBatch; ++b) {
      const double a0 = d[b][0] * uj[b][0];
      const double a1 = d[b][1] * uj[b][1];
      const double a2 = d[b][2] * uj[b][2];
      acc += a0 + a1 + a2;
    }
  }
  for (; t < t1; ++t) {
    const int64_t e = int64_t(t) * kWave + lane;
    const int64_t j = D.col[e];
    const double a0 = D.val[(int64_t(t) * 3 + 0) * kWave + lane] * u[j * 3 + 0];
    const double a1 = D.val[(int64_t(t) * 3 + 1) * kWave + lane] * u[j * 3 + 1];
    const double a2 = D.val[(int64_t(t) * 3 + 2) * kWave + lane] * u[j * 3 + 2];
    acc += a0 + a1 + a2;
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w != 0 || row >= D.nrows) return;
  double sum = part[0][lane];
#pragma unroll
  for (int q = 1; q < kNsSplit; ++q) sum += part[q][lane];
  du[row] = sum;
  rhs[row] = pin[row] ? 0.0 : -sum / k;
}

__global__ __launch_bounds__(kNsThreads) void k_ns_pressure(int64_t n, double* __restrict__ p,
                                                             const double* __restrict__ q,
                                                             const double* __restrict__ du,
                                                             const double* __restrict__ m_p, double nu) {
  const int64_t i = int64_t(blockIdx.x) * kNsThreads + threadIdx.x;
  if (i < n) p[i] = p[i] + q[i] - nu * du[i] / m_p[i];
}

unsigned slices_grid(int64_t nslices) { return unsigned((nslices + kNsThreads / kWave - 1) / (kNsThreads / kWave)); }

}  // namespace

hipError_t launch_ns_momentum(const NsEll& V, const NsEll& G, const double* u, const double* p, const double* q,
                              const double* f, const double* m_v, const uint8_t* dmask, const double* dval, double nu,
                              double k, double* uo, hipStream_t s) {
  if (V.nslices == 0) return hipSuccess;
  if (G.nslices != V.nslices || G.nrows != V.nrows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ns_momentum, slices_grid(V.nslices), kNsThreads, 0, s, V, G, u, p, q, f, m_v, dmask, dval, nu, k,
                     uo);
  return hipGetLastError();
}

hipError_t launch_ns_divergence(const NsEll& D, const double* u, const uint8_t* pin, double k, double* du, double* rhs,
                                hipStream_t s) {
  if (D.nslices == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ns_divergence, unsigned(D.nslices), kNsThreads, 0, s, D, u, pin, k, du, rhs);
  return hipGetLastError();
}

hipError_t launch_ns_pressure(int64_t n, double* p, const double* q, const double* du, const double* m_p, double nu,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ns_pressure, unsigned((n + kNsThreads - 1) / kNsThreads), kNsThreads, 0, s, n, p, q, du, m_p, nu);
  return hipGetLastError();
}

}  // namespace mgq1
