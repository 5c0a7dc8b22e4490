// HIP kernels of the GPU-side assembly of the constrained Q1 operators on adaptive
// meshes: A = Z (H^T A_full H) Z + I_C (Sec. 2.2: hanging nodes through the
// interpolation H; Dirichlet and hanging DoFs eliminated), the assembly the paper leaves
// on the CPU ("init", Sec. 5.1 and Sec. 6).
//
//   k_asm_table   the element matrices of every distinct cell size: Q1 on a box from
//                 tensor products of the 1D P1 stiffness, mass and derivative matrices
//                 (exact for constant coefficients): Laplace, transport-diffusion with
//                 the streamline-stabilisation term, linear elasticity, plus a lumped-mass
//                 term c m_i (eq. mass_lumping)
//   k_asm_gather  one thread per stored block (i, j): the sums over its precomputed
//                 contributions w K_e[a][b] (cell size class, corners a, b, w = the
//                 product of the two hanging-node weights, a power of two), in a fixed
//                 order, then the constraint rows and columns; no atomics, so repeated
//                 assemblies are bitwise identical
//
// The contribution lists (which cell corners reach which stored block through H) are
// built once on the host from the mesh; only the coefficients change between numeric
// assemblies.
#include <cmath>

#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kAsmThreads = 256;

__device__ __forceinline__ double k1(int i, int j, double s) { return (i == j ? 1.0 : -1.0) / s; }
__device__ __forceinline__ double m1(int i, int j, double s) { return (i == j ? 2.0 : 1.0) * s / 6.0; }
__device__ __forceinline__ double g1(int i, int j) { return j ? 0.5 : -0.5; }   // int phi_i phi_j'

// int d_k phi_a d_m phi_b over a box of side s
__device__ double dd(int dim, int k, int m, int a, int b, double s) {
  double v = 1.0;
  for (int ax = 0; ax < dim; ++ax) {
    const int ia = (a >> ax) & 1, ib = (b >> ax) & 1;
    double f;
    if (ax == k && ax == m) f = k1(ia, ib, s);
    else if (ax == k) f = g1(ib, ia);
    else if (ax == m) f = g1(ia, ib);
    else f = m1(ia, ib, s);
    v = v * f;
  }
  return v;
}

// int phi_a d_k phi_b
__device__ double gradtrial(int dim, int k, int a, int b, double s) {
  double v = 1.0;
  for (int ax = 0; ax < dim; ++ax) {
    const int ia = (a >> ax) & 1, ib = (b >> ax) & 1;
    const double f = ax == k ? g1(ia, ib) : m1(ia, ib, s);
    v = v * f;
  }
  return v;
}

// streamline-stabilisation parameter tau_K = h_K / (2 |b|) (coth Pe - 1 / Pe),
// Pe = |b| h_K / (2 eps), h_K = s |b| / max_k |b_k| (the cell's length along b)
__device__ double supg_tau(const AsmCoef& c, int dim, double s) {
  double nb2 = 0.0, mx = 0.0;
  for (int k = 0; k < dim; ++k) {
    nb2 += c.bvec[k] * c.bvec[k];
    mx = fmax(mx, fabs(c.bvec[k]));
  }
  const double nb = sqrt(nb2);
  if (nb == 0.0 || !c.supg) return 0.0;
  const double hk = s * nb / mx;
  const double pe = nb * hk / (2.0 * c.eps);
  double l;
  if (pe < 1e-2) l = pe / 3.0 - pe * pe * pe / 45.0 + 2.0 * pow(pe, 5.0) / 945.0;
  else l = 1.0 / tanh(pe) - 1.0 / pe;
  return hk / (2.0 * nb) * l;
}

// table[((d * nb + a) * nb + b) * B * B + ci * B + cj]: element matrix entry of corner a's
// row, corner b's column, components (ci, cj), for cell size class d
__global__ __launch_bounds__(kAsmThreads) void k_asm_table(AsmCoef c, int dim, int B, int nd,
                                                           const double* __restrict__ sizes,
                                                           double* __restrict__ table) {
  const int nb = 1 << dim;
  const int t = int(blockIdx.x) * kAsmThreads + int(threadIdx.x);
  if (t >= nd * nb * nb) return;
  const int d = t / (nb * nb), a = (t / nb) % nb, b = t % nb;
  const double s = sizes[d];
  double* out = table + int64_t(t) * B * B;
  for (int z = 0; z < B * B; ++z) out[z] = 0.0;
  if (c.pde == kAsmPoisson || c.pde == kAsmTD) {
    double lap = 0.0;
    for (int k = 0; k < dim; ++k) lap += dd(dim, k, k, a, b, s);
    double v = lap;
    if (c.pde == kAsmTD) {
      const double tau = supg_tau(c, dim, s);
      double conv = 0.0, stab = 0.0;
      for (int k = 0; k < dim; ++k) conv += c.bvec[k] * gradtrial(dim, k, a, b, s);
      for (int k = 0; k < dim; ++k)
        for (int m = 0; m < dim; ++m) stab += c.bvec[k] * c.bvec[m] * dd(dim, m, k, a, b, s);
      v = c.eps * lap + conv + tau * stab;
    }
    out[0] = v;
  } else {
    double lap = 0.0;
    for (int k = 0; k < dim; ++k) lap += dd(dim, k, k, a, b, s);
    for (int ci = 0; ci < dim; ++ci)
      for (int cj = 0; cj < dim; ++cj) {
        double v = c.mu * dd(dim, cj, ci, a, b, s) + c.lam * dd(dim, ci, cj, a, b, s);
        if (ci == cj) v += c.mu * lap;
        out[ci * B + cj] = v;
      }
  }
  if (c.mass_coef != 0.0 && a == b) {
    const double vol = dim == 3 ? s * s * s : s * s;
    for (int ci = 0; ci < B; ++ci) out[ci * B + ci] += c.mass_coef * vol / double(nb);
  }
}

// code = d | a << 5 | b << 8 | k << 11: cell size class, corners, weight 2^-k.  One
// thread per stored block: it reads the block's contribution list once, kAsmBatch codes
// at a time (the codes first, then their element-table rows), and sums the B^2 entries
// w K_e[a][b] in list order; then the constraint rows and columns.  LT: the workgroup first
// copies the element table (tn doubles) into LDS, where the lanes' scattered row reads
// cost far less than as cached global gathers (1.5x on the 129^3 elasticity level).  The
// block's values are staged in LDS so that each store instruction of a wave writes 64
// consecutive values of the value stream.
constexpr int kAsmBatch = 4;
constexpr int kAsmLdsBytes = 64 << 10;   // LDS of one workgroup: staging + table

template <int B, bool LT>
__global__ __launch_bounds__(kAsmThreads) void k_asm_gather(int64_t nnzb, int dim, int tn,
                                                            const int32_t* __restrict__ brow,
                                                            const int32_t* __restrict__ bcol,
                                                            const uint32_t* __restrict__ cptr,
                                                            const uint16_t* __restrict__ code,
                                                            const double* __restrict__ table,
                                                            const uint8_t* __restrict__ mask,
                                                            double* __restrict__ val) {
  constexpr int BB = B * B;
  __shared__ double stage[kAsmThreads * BB];
  extern __shared__ double ltab[];
  if constexpr (LT) {
    for (int e = int(threadIdx.x); e < tn; e += kAsmThreads) ltab[e] = table[e];
    __syncthreads();
  }
  const double* tb = LT ? ltab : table;
  const int64_t k = int64_t(blockIdx.x) * kAsmThreads + threadIdx.x;
  const int nb = 1 << dim;
  double acc[BB];
#pragma unroll
  for (int z = 0; z < BB; ++z) acc[z] = 0.0;
  if (k < nnzb) {
    const uint32_t t0 = cptr[k], t1 = cptr[k + 1];
    const int64_t i = brow[k], j = bcol[k];
    uint8_t mi[B], mj[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      mi[c] = mask[i * B + c];
      mj[c] = mask[j * B + c];
    }
    for (uint32_t u = t0; u < t1; u += kAsmBatch) {
      uint32_t cd[kAsmBatch];
#pragma unroll
      for (int q = 0; q < kAsmBatch; ++q) cd[q] = u + q < t1 ? uint32_t(code[u + q]) : 0u;
#pragma unroll
      for (int q = 0; q < kAsmBatch; ++q) {
        if (u + q < t1) {
          const int d = int(cd[q] & 31u), a = int((cd[q] >> 5) & 7u), b = int((cd[q] >> 8) & 7u);
          const int e = int((cd[q] >> 11) & 7u);
          const double w = ldexp(1.0, -e);
          const double* row = tb + int64_t((d * nb + a) * nb + b) * BB;
#pragma unroll
          for (int z = 0; z < BB; ++z) {
            const double p = w * row[z];
            acc[z] = acc[z] + p;
          }
        }
      }
    }
#pragma unroll
    for (int ci = 0; ci < B; ++ci)
#pragma unroll
      for (int cj = 0; cj < B; ++cj)
        if (mi[ci] || mj[cj]) acc[ci * B + cj] = (i == j && ci == cj) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int z = 0; z < BB; ++z) stage[threadIdx.x * BB + z] = acc[z];
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kAsmThreads * BB, total = nnzb * BB;
#pragma unroll
  for (int r = 0; r < BB; ++r) {
    const int e = r * kAsmThreads + int(threadIdx.x);
    if (base + e < total) val[base + e] = stage[e];
  }
}

template <int B>
void asm_gather_b(unsigned g, int64_t nnzb, int dim, int nd, const int32_t* brow, const int32_t* bcol,
                  const uint32_t* cptr, const uint16_t* code, const double* table, const uint8_t* mask, double* val,
                  hipStream_t s) {
  const int tn = nd * (1 << dim) * (1 << dim) * B * B;
  const size_t lds = size_t(tn) * sizeof(double);
  if (lds + size_t(kAsmThreads) * B * B * sizeof(double) <= size_t(kAsmLdsBytes))
    hipLaunchKernelGGL((k_asm_gather<B, true>), g, kAsmThreads, lds, s, nnzb, dim, tn, brow, bcol, cptr, code,
                       table, mask, val);
  else
    hipLaunchKernelGGL((k_asm_gather<B, false>), g, kAsmThreads, 0, s, nnzb, dim, tn, brow, bcol, cptr, code,
                       table, mask, val);
}

}  // namespace

hipError_t launch_asm_table(const AsmCoef& c, int dim, int B, int nd, const double* sizes, double* table,
                            hipStream_t s) {
  const int n = nd * (1 << dim) * (1 << dim);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_asm_table, unsigned((n + kAsmThreads - 1) / kAsmThreads), kAsmThreads, 0, s, c, dim, B, nd,
                     sizes, table);
  return hipGetLastError();
}

hipError_t launch_asm_gather(int64_t nnzb, int dim, int B, int nd, const int32_t* brow, const int32_t* bcol,
                             const uint32_t* cptr, const uint16_t* code, const double* table, const uint8_t* mask,
                             double* val, hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  const unsigned g = unsigned((nnzb + kAsmThreads - 1) / kAsmThreads);
  switch (B) {
    case 1: asm_gather_b<1>(g, nnzb, dim, nd, brow, bcol, cptr, code, table, mask, val, s); break;
    case 2: asm_gather_b<2>(g, nnzb, dim, nd, brow, bcol, cptr, code, table, mask, val, s); break;
    case 3: asm_gather_b<3>(g, nnzb, dim, nd, brow, bcol, cptr, code, table, mask, val, s); break;
    case 4: asm_gather_b<4>(g, nnzb, dim, nd, brow, bcol, cptr, code, table, mask, val, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mgq1
