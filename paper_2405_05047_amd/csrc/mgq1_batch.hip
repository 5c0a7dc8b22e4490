// HIP kernels of the batched form: every V-cycle step and Krylov vector operation of many
// independent problems (1 or 8 right-hand sides each) in one launch.  The per-slice
// bodies are those of the single-problem kernels; a block finds its problem entry with
// one wave-wide compare of 64 entries, and segmented reductions keep one partial per
// block and right-hand side, re-summed in a fixed order by the consumer kernel.
#include "mgq1_device.h"

namespace mgq1 {

// ======================================================================== batched form
namespace {

// the entry of block blk: the largest e with E[e].first <= blk (entries are sorted by
// first and E[0].first = 0).  Called by the whole first wave: each lane tests one entry, so
// 64 entries cost one round trip instead of a chain of dependent loads.
__device__ __forceinline__ int find_entry_wave(const BEntry* __restrict__ E, int n, int blk) {
  const int lane = threadIdx.x % kWave;
  int cnt = 0;
  for (int e0 = 0; e0 < n; e0 += kWave) {
    const int e = e0 + lane;
    const bool le = e < n && E[e].first <= blk;
    cnt += __popcll(__ballot(le));
    if (cnt < e0 + kWave) break;           // this chunk holds the first entry past blk
  }
  return cnt - 1;
}

__device__ __forceinline__ void block_entry(const BEntry* __restrict__ E, int n, int& se) {
  if (threadIdx.x < kWave) {
    const int e = find_entry_wave(E, n, blockIdx.x);
    if (threadIdx.x == 0) se = e;
  }
  __syncthreads();
}

// V-cycle steps on slices (sweep0, sweep, masked defect) for every problem of the batch
template <int B, int NR, int K, class X, class T, int KIND, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_bsell(const BEntry* __restrict__ E, int ne, T omega,
                                                    const int* __restrict__ active) {
  __shared__ int se;
  block_entry(E, ne, se);
  const BEntry& e = E[se];
  if (active && !active[e.prob]) return;
  const SliceLane s = slice_lane<B, NR>(e.A, (blockIdx.x - e.first) * kSliceWaves + threadIdx.x / kWave,
                                        threadIdx.x % kWave);
  if (KIND == BK_SWEEP0)
    sweep0_slice<B, NR, X, T>(static_cast<const X*>(e.S), static_cast<const X*>(e.in0), static_cast<X*>(e.out),
                              omega, s);
  else if (KIND == BK_SWEEP)
    sweep_slice<B, NR, K, X, T, KB, C16, 1>(e.A, static_cast<const X*>(e.S), static_cast<const X*>(e.in0),
                                    static_cast<const X*>(e.in1), static_cast<X*>(e.out), omega, s);
  else
    spmv_slice<B, NR, K, X, X, T, 2, KB, C16, 1>(e.A, static_cast<const X*>(e.in0), static_cast<const X*>(e.in1),
                                         static_cast<X*>(e.out), e.mask, s);
}

// fixed-order sum over the block of values that belong to rhs q = tid % NR; thread q of
// the result gets the sum for q
__device__ __forceinline__ double block_sum_rhs(double v, int NR, double* lds) {
  // inside each wave a fixed shuffle tree combines the lanes of equal lane % NR, then
  // thread q adds the per-wave results in wave order
  for (int o = kWave / 2; o >= NR; o >>= 1) v += __shfl_down(v, o, kWave);
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  if (ln < NR) lds[wv * NR + ln] = v;
  __syncthreads();
  double t = 0.0;
  if (int(threadIdx.x) < NR)
    for (int k = 0; k < int(blockDim.x) / kWave; ++k) t += lds[k * NR + threadIdx.x];
  __syncthreads();
  return t;
}

// outer-loop products with the FP64 operator: w = A z (KIND SPMV64) or r = b - A x with
// partial sums of squares per (block, rhs) (KIND DEFECT64)
template <int B, int NR, class XI, int KIND, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_bsell64(const BEntry* __restrict__ E, int ne,
                                                      const int* __restrict__ active, double* __restrict__ partials) {
  __shared__ int se;
  __shared__ double lds[kThreads];
  block_entry(E, ne, se);
  const BEntry& e = E[se];
  const bool on = !(active && !active[e.prob]);
  double out = 0.0, other = 0.0;
  if (on) {
    const SliceLane s = slice_lane<B, NR>(e.A, (blockIdx.x - e.first) * kSliceWaves + threadIdx.x / kWave,
                                          threadIdx.x % kWave);
    if (KIND == BK_SPMV64) {
      out = spmv_slice<B, NR, VK_F64, XI, double, double, 0, KB, C16, 1>(e.A, nullptr, static_cast<const XI*>(e.in1),
                                                                 static_cast<double*>(e.out), nullptr, s);
    } else {
      out = spmv_slice<B, NR, VK_F64, double, double, double, 1, KB, C16, 1>(e.A, static_cast<const double*>(e.in0),
                                                                     static_cast<const double*>(e.in1),
                                                                     static_cast<double*>(e.out), nullptr, s);
      other = out;
    }
  }
  if (KIND == BK_DEFECT64) {               // lane % NR is the right-hand side
    const double t = block_sum_rhs(out * other, NR, lds);
    if (threadIdx.x < NR) partials[int64_t(blockIdx.x) * NR + threadIdx.x] = t;
  }
}

template <int B, int NR, class X, class T, int KIND>
__global__ __launch_bounds__(kThreads) void k_belem(const BEntry* __restrict__ E, int ne,
                                                    const int* __restrict__ active) {
  __shared__ int se;
  block_entry(E, ne, se);
  const BEntry& e = E[se];
  if (active && !active[e.prob]) return;
  const int64_t t = int64_t(blockIdx.x - e.first) * kThreads + threadIdx.x;
  if (t < int64_t(e.A.n) * B * NR) static_cast<X*>(e.out)[t] = X(0);   // BK_FILL0
}

// restriction (rows = coarse nodes, row mask M_c) and prolongation + correction (rows =
// fine nodes, row mask M_f, column mask M_c) of every problem with the sliced transfers
template <int B, int NR, class X, class T, int KIND>
__global__ __launch_bounds__(kThreads) void k_btsell(const BEntry* __restrict__ E, int ne,
                                                     const int* __restrict__ active) {
  __shared__ int se;
  block_entry(E, ne, se);
  const BEntry& e = E[se];
  if (active && !active[e.prob]) return;
  const int slice = (blockIdx.x - e.first) * kSliceWaves + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const X* in = static_cast<const X*>(e.in0);
  X* out = static_cast<X*>(e.out);
  if (KIND == BK_RESTRICT) {
    if (e.Ts.f32) tsell_lane<B, NR, X, T, float, false, 0>(e.Ts, slice, lane, in, out, e.mask_c, nullptr);
    else tsell_lane<B, NR, X, T, double, false, 0>(e.Ts, slice, lane, in, out, e.mask_c, nullptr);
  } else {
    if (e.Ts.f32) tsell_lane<B, NR, X, T, float, true, 1>(e.Ts, slice, lane, in, out, e.mask, e.mask_c);
    else tsell_lane<B, NR, X, T, double, true, 1>(e.Ts, slice, lane, in, out, e.mask, e.mask_c);
  }
}

// coarse solve x = Ainv b for NR right-hand sides, one wavefront per row
template <int NR, class X>
__global__ __launch_bounds__(kThreads) void k_bcoarse(const BEntry* __restrict__ E, int ne,
                                                      const int* __restrict__ active) {
  __shared__ int se;
  block_entry(E, ne, se);
  const BEntry& e = E[se];
  if (active && !active[e.prob]) return;
  const int i = (blockIdx.x - e.first) * kSliceWaves + threadIdx.x / kWave;
  if (i >= e.n0) return;
  const int lane = threadIdx.x % kWave, q = lane % NR;
  const X* b = static_cast<const X*>(e.in0);
  constexpr int U = 8;
  double acc = 0.0;
  const double* row = e.Ainv + int64_t(i) * e.n0;
  for (int k0 = lane / NR; k0 < e.n0; k0 += (kWave / NR) * U) {
    double av[U];
    X bv[U];                                 // widened when used (no wait per element)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * (kWave / NR);
      av[u] = k < e.n0 ? row[k] : 0.0;
      bv[u] = k < e.n0 ? b[int64_t(k) * NR + q] : X(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += av[u] * double(bv[u]);
  }
#pragma unroll
  for (int o = kWave / 2; o >= NR; o >>= 1) acc += __shfl_down(acc, o, kWave);
  if (lane < NR) static_cast<X*>(e.out)[int64_t(i) * NR + lane] = X(acc);
}

// ---- segmented vector kernels: block -> problem segment, thread keeps rhs q = tid % NR
struct SegPos {
  int p, lb, nb, first;
  int64_t off, len;
  bool on;                                 // the problem takes part in this launch
};

__device__ __forceinline__ SegPos seg_pos(const BSegs& g) {
  SegPos s;
  s.p = g.blk_prob[blockIdx.x];
  s.first = g.vfirst[s.p];
  s.lb = blockIdx.x - s.first;
  s.nb = g.vcount[s.p];
  s.off = g.off[s.p];
  s.len = g.len[s.p];
  s.on = !g.on || g.on[s.p];
  return s;
}

// every block of problem p computes the per-rhs sums of the problem's partials
__device__ __forceinline__ void seg_sums(const double* __restrict__ pin, const SegPos& sp, int NR, double* lds,
                                         double* out) {
  constexpr int U = 8;                     // partial loads issued together
  double t = 0.0;
  const int q = threadIdx.x % NR;
  const int step = int(blockDim.x) / NR;
  const int first = sp.first, nb = sp.nb;
  for (int b0 = threadIdx.x / NR; b0 < nb; b0 += step * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * step;
      v[u] = b < nb ? pin[int64_t(first + b) * NR + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
  }
  const double r = block_sum_rhs(t, NR, lds);
  if (int(threadIdx.x) < NR) out[threadIdx.x] = r;
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_bdot(BSegs g, const double* __restrict__ a,
                                                   const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double lds[kThreads];
  const SegPos sp = seg_pos(g);
  if (!sp.on) return;                      // uniform over the block
  constexpr int U = 4;
  double t = 0.0;
  const int64_t stride = int64_t(sp.nb) * blockDim.x;
  for (int64_t i0 = int64_t(sp.lb) * blockDim.x + threadIdx.x; i0 < sp.len; i0 += stride * U) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      av[u] = i < sp.len ? a[sp.off + i] : 0.0;
      bv[u] = (b && i < sp.len) ? b[sp.off + i] : av[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) t += av[u] * bv[u];
  }
  const double r = block_sum_rhs(t, g.NR, lds);
  if (int(threadIdx.x) < g.NR) out[int64_t(blockIdx.x) * g.NR + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void k_bmgs_step(BSegs g, double* __restrict__ w, const double* __restrict__ vi,
                                                        const double* __restrict__ vnext, const double* __restrict__ pin,
                                                        double* __restrict__ pout, double* __restrict__ H,
                                                        int64_t hstride) {
  __shared__ double lds[kThreads];
  __shared__ double hq[64];
  const SegPos sp = seg_pos(g);
  if (!sp.on) return;                      // uniform over the block
  constexpr int U = 4;
  const int64_t stride = int64_t(sp.nb) * blockDim.x;
  double wv[U], vv[U], nv[U];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      const bool ok = i < sp.len;
      wv[u] = ok ? w[sp.off + i] : 0.0;
      vv[u] = ok ? vi[sp.off + i] : 0.0;
      nv[u] = (ok && vnext) ? vnext[sp.off + i] : 0.0;
    }
  };
  const int64_t first = int64_t(sp.lb) * blockDim.x + threadIdx.x;
  load(first);                             // independent of h: overlaps the partial sums
  seg_sums(pin, sp, g.NR, lds, hq);
  if (sp.lb == 0 && int(threadIdx.x) < g.NR) H[int64_t(sp.p * g.NR + threadIdx.x) * hstride] = hq[threadIdx.x];
  const double h = hq[threadIdx.x % g.NR];
  double t = 0.0;
  for (int64_t i0 = first; i0 < sp.len; i0 += stride * U) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      const double v = wv[u] - h * vv[u];
      if (i < sp.len) w[sp.off + i] = v;
      t += v * (vnext ? nv[u] : v);
    }
  }
  const double r = block_sum_rhs(t, g.NR, lds);
  if (int(threadIdx.x) < g.NR) pout[int64_t(blockIdx.x) * g.NR + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void k_bmgs_normalize(BSegs g, double* __restrict__ w,
                                                             const double* __restrict__ pin, double* __restrict__ H,
                                                             int64_t hstride, float* __restrict__ wc) {
  __shared__ double lds[kThreads];
  __shared__ double hq[64];
  const SegPos sp = seg_pos(g);
  if (!sp.on) return;                      // uniform over the block
  constexpr int U = 4;
  const int64_t stride = int64_t(sp.nb) * blockDim.x;
  double wv[U];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      wv[u] = i < sp.len ? w[sp.off + i] : 0.0;
    }
  };
  const int64_t first = int64_t(sp.lb) * blockDim.x + threadIdx.x;
  load(first);                             // independent of the norm (latency overlap)
  seg_sums(pin, sp, g.NR, lds, hq);
  if (int(threadIdx.x) < g.NR) hq[threadIdx.x] = sqrt(hq[threadIdx.x]);
  __syncthreads();
  if (sp.lb == 0 && int(threadIdx.x) < g.NR) H[int64_t(sp.p * g.NR + threadIdx.x) * hstride] = hq[threadIdx.x];
  const double nrm = hq[threadIdx.x % g.NR];
  if (nrm == 0.0) {
    if (wc)
      for (int64_t i = first; i < sp.len; i += stride) wc[sp.off + i] = float(w[sp.off + i]);
    return;
  }
  for (int64_t i0 = first; i0 < sp.len; i0 += stride * U) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < sp.len) {
        const double v = wv[u] / nrm;
        w[sp.off + i] = v;
        if (wc) wc[sp.off + i] = float(v);
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_bscale(BSegs g, double* __restrict__ y, const double* __restrict__ x,
                                                     const double* __restrict__ beta, const int* __restrict__ iact,
                                                     float* __restrict__ yc) {
  const SegPos sp = seg_pos(g);
  if (!sp.on) return;                      // uniform over the block
  const int inst = sp.p * g.NR + threadIdx.x % g.NR;
  const double bt = beta[inst];
  const bool on = iact[inst] && bt != 0.0;
  const int64_t stride = int64_t(sp.nb) * blockDim.x;
  for (int64_t i = int64_t(sp.lb) * blockDim.x + threadIdx.x; i < sp.len; i += stride) {
    const double v = on ? x[sp.off + i] / bt : 0.0;
    y[sp.off + i] = v;
    if (yc) yc[sp.off + i] = float(v);
  }
}

template <class Z>
__global__ __launch_bounds__(kThreads) void k_bupdate(BSegs g, double* __restrict__ x, const Z* __restrict__ Zm,
                                                      int64_t ldz, const double* __restrict__ yv, int m,
                                                      const int* __restrict__ kk) {
  const SegPos sp = seg_pos(g);
  if (!sp.on) return;                      // uniform over the block
  const int inst = sp.p * g.NR + threadIdx.x % g.NR;
  const int k = kk[inst];
  if (k == 0) return;
  const double* y = yv + int64_t(inst) * m;
  const int64_t stride = int64_t(sp.nb) * blockDim.x;
  for (int64_t i = int64_t(sp.lb) * blockDim.x + threadIdx.x; i < sp.len; i += stride) {
    const int64_t e = sp.off + i;
    double acc = x[e];
    for (int c = 0; c < k; ++c) acc += y[c] * double(Zm[int64_t(c) * ldz + e]);
    x[e] = acc;
  }
}

__global__ __launch_bounds__(kThreads) void k_bfinish(const double* __restrict__ p, const int* __restrict__ pfirst,
                                                      const int* __restrict__ pcount, int NR, double* out, int sq) {
  __shared__ double lds[kMaxWaves + 1];
  const int inst = blockIdx.x, pr = inst / NR, q = inst % NR;
  double t = 0.0;
  for (int b = threadIdx.x; b < pcount[pr]; b += blockDim.x) t += p[int64_t(pfirst[pr] + b) * NR + q];
  const double s = block_allsum(t, lds);
  if (threadIdx.x == 0) out[inst] = sq ? sqrt(s) : s;
}

__global__ void k_bgivens(int j, int m, int n_inst, double* H, double* cs, double* sn, double* g, double* st,
                          const double* __restrict__ tol, int* kk, const int* __restrict__ iact) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  // rotations after the instance's cycle has closed are never used
  if (inst >= n_inst || !iact[inst] || kk[inst] != 0) return;
  const int ld = m + 1;
  double* h = H + int64_t(inst) * ld * m + int64_t(j) * ld;
  double* c = cs + int64_t(inst) * m;
  double* s = sn + int64_t(inst) * m;
  double* gg = g + int64_t(inst) * ld;
  const bool breakdown = h[j + 1] == 0.0;
  for (int i = 0; i < j; ++i) {
    const double t = c[i] * h[i] + s[i] * h[i + 1];
    h[i + 1] = -s[i] * h[i] + c[i] * h[i + 1];
    h[i] = t;
  }
  const double den = hypot(h[j], h[j + 1]);
  c[j] = h[j] / den;
  s[j] = h[j + 1] / den;
  h[j] = den;
  h[j + 1] = 0.0;
  gg[j + 1] = -s[j] * gg[j];
  gg[j] = c[j] * gg[j];
  st[2 * inst] = fabs(gg[j + 1]);
  st[2 * inst + 1] = breakdown ? 1.0 : 0.0;
  // closes on breakdown, on the tolerance, or on a non-finite estimate (!(x > tol))
  if (kk[inst] == 0 && (breakdown || !(fabs(gg[j + 1]) > tol[inst]))) kk[inst] = j + 1;
}

__global__ void k_bbacksolve(int m, int n_inst, const double* H, const double* g, double* yv, const int* kk) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  const int k = kk[inst];
  const int ld = m + 1;
  const double* Hh = H + int64_t(inst) * ld * m;
  const double* gg = g + int64_t(inst) * ld;
  double* y = yv + int64_t(inst) * m;
  for (int i = k - 1; i >= 0; --i) {
    double t = gg[i];
    for (int c = i + 1; c < k; ++c) t -= Hh[int64_t(c) * ld + i] * y[c];
    y[i] = t / Hh[int64_t(i) * ld + i];
  }
}

__global__ void k_binit(int m, int n_inst, double* g, const double* beta, int* kk) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  double* gg = g + int64_t(inst) * (m + 1);
  gg[0] = beta[inst];
  for (int i = 1; i <= m; ++i) gg[i] = 0.0;
  kk[inst] = 0;
}

__global__ void k_bclose(int j, int n_inst, int* kk, const int* iact) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst < n_inst && iact[inst] && kk[inst] == 0) kk[inst] = j + 1;
}

template <int B, int NR, int K, class X, class T, int KB, bool C16>
hipError_t batched_sell(int kind, const BEntry* E, int ne, int nb, double omega, const int* active,
                        double* partials, hipStream_t s) {
  switch (kind) {
    case BK_SWEEP: hipLaunchKernelGGL((k_bsell<B, NR, K, X, T, BK_SWEEP, KB, C16>), nb, kThreads, 0, s, E, ne, T(omega), active); break;
    case BK_DEFECT: hipLaunchKernelGGL((k_bsell<B, NR, K, X, T, BK_DEFECT, KB, C16>), nb, kThreads, 0, s, E, ne, T(omega), active); break;
    case BK_SPMV64: hipLaunchKernelGGL((k_bsell64<B, NR, X, BK_SPMV64, KB, C16>), nb, kThreads, 0, s, E, ne, active, partials); break;
    case BK_DEFECT64: hipLaunchKernelGGL((k_bsell64<B, NR, double, BK_DEFECT64, KB, C16>), nb, kThreads, 0, s, E, ne, active, partials); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int B, int NR, int K, class X, class T>
hipError_t batched_t(int kind, const BEntry* E, int ne, int nb, double omega, const int* active, double* partials,
                     int kb, hipStream_t s) {
  switch (kind) {
    case BK_SWEEP: case BK_DEFECT: case BK_SPMV64: case BK_DEFECT64:
      // kb < 0 selects the 16-bit column format (every entry of the launch has it)
      if (kb < 0) {
        if (-kb == kb_alt<B>()) return batched_sell<B, NR, K, X, T, kb_alt<B>(), true>(kind, E, ne, nb, omega, active, partials, s);
        return batched_sell<B, NR, K, X, T, kb_default<B>(), true>(kind, E, ne, nb, omega, active, partials, s);
      }
      if (kb == kb_alt<B>()) return batched_sell<B, NR, K, X, T, kb_alt<B>(), false>(kind, E, ne, nb, omega, active, partials, s);
      return batched_sell<B, NR, K, X, T, kb_default<B>(), false>(kind, E, ne, nb, omega, active, partials, s);
    case BK_SWEEP0: hipLaunchKernelGGL((k_bsell<B, NR, K, X, T, BK_SWEEP0, kb_default<B>(), false>), nb, kThreads, 0, s, E, ne, T(omega), active); break;
    case BK_RESTRICT: hipLaunchKernelGGL((k_btsell<B, NR, X, T, BK_RESTRICT>), nb, kThreads, 0, s, E, ne, active); break;
    case BK_PROLONG: hipLaunchKernelGGL((k_btsell<B, NR, X, T, BK_PROLONG>), nb, kThreads, 0, s, E, ne, active); break;
    case BK_FILL0: hipLaunchKernelGGL((k_belem<B, NR, X, T, BK_FILL0>), nb, kThreads, 0, s, E, ne, active); break;
    case BK_COARSE: hipLaunchKernelGGL((k_bcoarse<NR, X>), nb, kThreads, 0, s, E, ne, active); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int B, int NR>
hipError_t batched_bn(int kind, const BEntry* E, int ne, int nb, int vkind, int xk, double omega, const int* active,
                      double* partials, int kb, hipStream_t s) {
  if (xk == X_F64) {
    if (vkind != VK_F64) return hipErrorInvalidValue;
    return batched_t<B, NR, VK_F64, double, double>(kind, E, ne, nb, omega, active, partials, kb, s);
  }
  switch (vkind) {
    case VK_F32: return batched_t<B, NR, VK_F32, float, float>(kind, E, ne, nb, omega, active, partials, kb, s);
    case VK_F16: return batched_t<B, NR, VK_F16, float, float>(kind, E, ne, nb, omega, active, partials, kb, s);
    case VK_BF16: return batched_t<B, NR, VK_BF16, float, float>(kind, E, ne, nb, omega, active, partials, kb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int batched_blocks(int kind, const SellDev& A, const TSellDev& Ts, int n0, int NR) {
  switch (kind) {
    case BK_SWEEP0: case BK_SWEEP: case BK_DEFECT: case BK_SPMV64: case BK_DEFECT64:
      return int(slice_grid(A.nslices));
    case BK_RESTRICT: case BK_PROLONG:
      return int(slice_grid(Ts.nslices));
    case BK_FILL0:
      return int(grid_for(int64_t(A.n) * A.B * NR, kThreads));
    case BK_COARSE:
      return int(grid_for(n0, kSliceWaves));
    default:
      return 0;
  }
}

hipError_t launch_batched(int kind, const BEntry* E, int ne, int nb, int B, int NR, int vkind, int xk, double omega,
                          const int* active, double* partials, int kb, hipStream_t s) {
  if (nb == 0 || ne == 0) return hipSuccess;
  if (NR == 1) {
    switch (B) {
      case 1: return batched_bn<1, 1>(kind, E, ne, nb, vkind, xk, omega, active, partials, kb, s);
      case 3: return batched_bn<3, 1>(kind, E, ne, nb, vkind, xk, omega, active, partials, kb, s);
      case 4: return batched_bn<4, 1>(kind, E, ne, nb, vkind, xk, omega, active, partials, kb, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (NR == 8) {
    switch (B) {
      case 1: return batched_bn<1, 8>(kind, E, ne, nb, vkind, xk, omega, active, partials, kb, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bdot(const BSegs& g, const double* a, const double* b, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_bdot, g.n_blocks, kThreads, 0, s, g, a, b, partials);
  return hipGetLastError();
}

hipError_t launch_bfinish(const double* partials, const int* pfirst, const int* pcount, int n_inst, int NR,
                          double* out, int sqrt_out, hipStream_t s) {
  hipLaunchKernelGGL(k_bfinish, n_inst, kThreads, 0, s, partials, pfirst, pcount, NR, out, sqrt_out);
  return hipGetLastError();
}

hipError_t launch_bmgs_step(const BSegs& g, double* w, const double* vi, const double* vnext, const double* pin,
                            double* pout, double* H, int64_t hstride, hipStream_t s) {
  hipLaunchKernelGGL(k_bmgs_step, g.n_blocks, kThreads, 0, s, g, w, vi, vnext, pin, pout, H, hstride);
  return hipGetLastError();
}

hipError_t launch_bmgs_normalize(const BSegs& g, double* w, const double* pin, double* H, int64_t hstride,
                                 hipStream_t s, float* wc) {
  hipLaunchKernelGGL(k_bmgs_normalize, g.n_blocks, kThreads, 0, s, g, w, pin, H, hstride, wc);
  return hipGetLastError();
}

hipError_t launch_bscale(const BSegs& g, double* y, const double* x, const double* beta, const int* iact,
                         hipStream_t s, float* yc) {
  hipLaunchKernelGGL(k_bscale, g.n_blocks, kThreads, 0, s, g, y, x, beta, iact, yc);
  return hipGetLastError();
}

hipError_t launch_bupdate(const BSegs& g, double* x, const void* Z, int zk, int64_t ldz, const double* yv, int m,
                          const int* kk, hipStream_t s) {
  if (zk == X_F64)
    hipLaunchKernelGGL(k_bupdate<double>, g.n_blocks, kThreads, 0, s, g, x, static_cast<const double*>(Z), ldz, yv, m, kk);
  else
    hipLaunchKernelGGL(k_bupdate<float>, g.n_blocks, kThreads, 0, s, g, x, static_cast<const float*>(Z), ldz, yv, m, kk);
  return hipGetLastError();
}

hipError_t launch_bgivens(int j, int m, int n_inst, double* H, double* cs, double* sn, double* g, double* st,
                          const double* tol, int* kk, const int* iact, hipStream_t s) {
  hipLaunchKernelGGL(k_bgivens, grid_for(n_inst, 64), 64, 0, s, j, m, n_inst, H, cs, sn, g, st, tol, kk, iact);
  return hipGetLastError();
}

hipError_t launch_bbacksolve(int m, int n_inst, const double* H, const double* g, double* yv, const int* kk,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_bbacksolve, grid_for(n_inst, 64), 64, 0, s, m, n_inst, H, g, yv, kk);
  return hipGetLastError();
}

hipError_t launch_binit(int m, int n_inst, double* g, const double* beta, int* kk, hipStream_t s) {
  hipLaunchKernelGGL(k_binit, grid_for(n_inst, 64), 64, 0, s, m, n_inst, g, beta, kk);
  return hipGetLastError();
}

hipError_t launch_bclose(int j, int n_inst, int* kk, const int* iact, hipStream_t s) {
  hipLaunchKernelGGL(k_bclose, grid_for(n_inst, 64), 64, 0, s, j, n_inst, kk, iact);
  return hipGetLastError();
}

}  // namespace mgq1
