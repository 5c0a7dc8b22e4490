// HIP kernels of the multigrid hot path for gfx950 (MI355X).
//
// Every kernel here streams sparse data and is bound by HBM bandwidth (about 0.1-0.25
// flop per byte in FP64), so there is no matrix-core work: the design goals are coalesced
// value / index streams, cached gathers of x, one pass over A per smoothing sweep, short
// chains of dependent loads on small levels, and deterministic reductions (no atomics).
//
//   SELL slice kernels (defect / SpMV, smoothing sweep): one wavefront per slice of
//   64/(B*NR) nodes; lane = (node*B + component)*NR + rhs owns one scalar row of one
//   right-hand side.  Block slots are consumed in batches of KB (chosen per level by the
//   setup's autotuner): column indices and values of a batch are loaded first, then the x
//   gathers, then the FMAs in slot order, as straight-line code between scheduling
//   barriers, so a row of 9 (2D) or 27 (3D) blocks costs a few memory round trips instead
//   of one per block.  Each value load of a wave is one contiguous stream.  For block
//   operators each lane gathers only its own component of a neighbour node and takes the
//   others from the node's lanes by wave shuffles; the smoother exchanges the B residual
//   components of a node the same way and applies the stored block inverse.  Column
//   indices are 16-bit offsets from a per-slot base, except in slices whose columns span
//   2^16 or more (a per-slice bit selects the 32-bit indices there).  Uniform-width levels
//   compute a slice's slot range instead of loading it; block rows may be sorted by
//   length inside windows of slices (a permutation maps each row position to its node).
//   Workgroup ids are remapped so that each XCD (round-robin dispatch over 8 XCDs) walks a
//   contiguous range of slices and keeps its own L2 warm.
//
//   Transfers: the scalar P~ and R = P~^T in the same sliced layout over node rows, applied
//   per component with the constraint masks (pull-style, no atomics).
//
//   Reductions: every block writes one partial sum; the consumer (the next kernel in the
//   chain) re-sums all partials in a fixed order in every block, so the result is
//   deterministic, identical in all blocks and needs no atomics (same-address atomics
//   serialise at roughly 30 ns each).
//
//   Tail kernel (optional, off by default): the levels below a size threshold and the
//   coarse solve as one single-workgroup launch with barriers between the steps.
//
//   Batched form (mgq1_batch.hip): the same slice bodies over the entries of many problems
//   per launch, and segmented Krylov kernels (each block belongs to one problem's vector
//   segment).  The shared device code is in mgq1_device.h.
//
// Paper correspondence: smoother x + omega S (b - A x), transfers P and R = P^T and the
// coarse solve (Sec. 4.1 "Geometric Multigrid CUDA", Algorithm "Geometric multigrid
// solver"); GMRES building blocks with modified Gram-Schmidt (Sec. 4.2).
#include "mgq1_device.h"

namespace mgq1 {
namespace {

// ------------------------------------------------------------------ grid kernels
// NORM: per-block partial sums of out * out, or of out * dotv[row] when dotv is given
template <int B, int K, class XI, class XO, class T, int MODE, bool NORM, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_spmv(SellDev A, const XO* __restrict__ b, const XI* __restrict__ x,
                                                   XO* __restrict__ y, const uint8_t* __restrict__ mask,
                                                   double* __restrict__ partials, const double* __restrict__ dotv) {
  dict_stage<K>(A);
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const SliceLane s = slice_lane<B, 1>(A, bid * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave);
  const T out = spmv_slice<B, 1, K, XI, XO, T, MODE, KB, C16>(A, b, x, y, mask, s);
  if (NORM) {
    __shared__ double lds[kMaxWaves + 1];
    const double p = block_allsum(double(out) * (dotv ? (s.valid ? dotv[s.dof] : 0.0) : double(out)), lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = p;
  }
}

template <int B, int K, class X, class T, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_sweep(SellDev A, const X* __restrict__ S, const X* __restrict__ b,
                                                    const X* __restrict__ x, X* __restrict__ xo, T omega,
                                                    T beta, int pmode) {
  dict_stage<K>(A);
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const SliceLane s = slice_lane<B, 1>(A, bid * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave);
  sweep_slice<B, 1, K, X, T, KB, C16>(A, S, b, x, xo, omega, s, beta, pmode);
}

// two smoothing sweeps from x = 0 in one pass, one component per node:
// x1 = omega S b (formed per column on the fly), x2 = x1 + omega S (b - A x1)
template <int K, class X, class T, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_sweep2z(SellDev A, const X* __restrict__ S, const X* __restrict__ b,
                                                      X* __restrict__ xo, T omega) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int slice = bid * kSliceWaves + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int64_t i = int64_t(slice) * kWave + lane;
  if (slice >= A.nslices || i >= A.n) return;
  const X si = S[i], bi = b[i];              // issued with the slice bounds
  const int su = __builtin_amdgcn_readfirstlane(slice);
  int k, k1;
  slot_range(A, su, k, k1);
  T acc = T(0);
  const int node = int(i);
  const bool wide = C16 && is_wide(A, su);
  if (A.nt) {
    if (wide) sell_loop_z<KB, K, X, T, false, true>(k, k1, A, lane, node, S, b, omega, acc);
    else sell_loop_z<KB, K, X, T, C16, true>(k, k1, A, lane, node, S, b, omega, acc);
  } else {
    if (wide) sell_loop_z<KB, K, X, T, false, false>(k, k1, A, lane, node, S, b, omega, acc);
    else sell_loop_z<KB, K, X, T, C16, false>(k, k1, A, lane, node, S, b, omega, acc);
  }
  if (K == VK_F16 || K == VK_BF16) acc *= T(ldexpf(1.0f, A.rexp[int64_t(slice) * kWave + lane]));
  const X x1 = X(omega * (T(0) + T(si) * T(bi)));
  const T res = T(bi) - acc;
  const T upd = T(0) + T(si) * res;
  xo[i] = X(T(x1) + omega * upd);
}

template <int B, class X, class T>
__global__ __launch_bounds__(kThreads) void k_sweep0(SellDev A, const X* __restrict__ S, const X* __restrict__ b,
                                                     X* __restrict__ xo, T omega) {
  const SliceLane s = slice_lane<B, 1>(A, blockIdx.x * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave);
  sweep0_slice<B, 1, X, T>(S, b, xo, omega, s);
}


// x = Ainv b, one wavefront per row (Ainv row-major, FP64)
// U row chunks of 64 elements have their loads issued together; every lane sums its
// elements in increasing column order whatever U is, so U does not change the result
template <class XI, class XO, int U = 8>
__device__ __forceinline__ void gemv_row(int n, const double* __restrict__ Ainv, const XI* __restrict__ b,
                                         XO* __restrict__ x, int i, int lane) {
  double acc = 0.0;
  const double* row = Ainv + int64_t(i) * n;
  for (int k0 = lane; k0 < n; k0 += kWave * U) {
    double av[U];
    XI bv[U];                                // widened only when used: a conditional load
#pragma unroll                               // converted in place would wait per element
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kWave;
      av[u] = k < n ? row[k] : 0.0;
      bv[u] = k < n ? b[k] : XI(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += av[u] * double(bv[u]);
  }
  acc = wave_sum(acc);
  if (lane == 0) x[i] = XO(acc);
}

template <class XI, class XO>
__global__ __launch_bounds__(kThreads) void k_coarse_gemv(int n, const double* __restrict__ Ainv,
                                                          const XI* __restrict__ b, XO* __restrict__ x) {
  const int i = blockIdx.x * kSliceWaves + threadIdx.x / kWave;
  if (i < n) gemv_row<XI, XO, 32>(n, Ainv, b, x, i, threadIdx.x % kWave);   // rows up to 2048 in one pass
}

// ------------------------------------------------------------------ tail kernel
template <int B, int K, class X, class T>
__device__ void tail_sweep(const TailLevel& L, const X* b, const X* x, X* xo, T omega) {
  const int nw = blockDim.x / kWave, w = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  for (int sl = w; sl < L.A.nslices; sl += nw)
    sweep_slice<B, 1, K, X, T, kb_default<B>(), false, 2>(L.A, static_cast<const X*>(L.S), b, x, xo, omega,
                                                          slice_lane<B, 1>(L.A, sl, ln));
  __syncthreads();
}

// Levels top .. 1 and the coarse solve of one V-cycle in a single workgroup.  Level top
// reads its right-hand side from lv[top].b and leaves its result in lv[top].x, exactly
// like the grid-kernel path of the host driver (same ping-pong order).
template <int B, int K, class X, class T>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailLevel* __restrict__ lv, TailParams p) {
  const int nw = blockDim.x / kWave, w = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const T omega = T(p.omega);
  const int pre_pp = p.nu1 >= 1 ? p.nu1 - 1 : 0;
  const int pp = pre_pp + p.nu2;
  // descent
  for (int l = p.top; l >= 1; --l) {
    const TailLevel& L = lv[l];
    X* own = static_cast<X*>(L.x);
    X* tmp = static_cast<X*>(L.t);
    X* cur = (pp % 2 == 0) ? own : tmp;
    X* oth = (pp % 2 == 0) ? tmp : own;
    const X* b = static_cast<const X*>(L.b);
    if (p.nu1 >= 1) {
      for (int sl = w; sl < L.A.nslices; sl += nw)
        sweep0_slice<B, 1, X, T>(static_cast<const X*>(L.S), b, cur, omega, slice_lane<B, 1>(L.A, sl, ln));
      __syncthreads();
      for (int q = 1; q < p.nu1; ++q) {
        tail_sweep<B, K, X, T>(L, b, cur, oth, omega);
        X* t = cur; cur = oth; oth = t;
      }
    } else {
      for (int64_t t = threadIdx.x; t < int64_t(L.A.n) * B; t += blockDim.x) cur[t] = X(0);
      __syncthreads();
    }
    for (int sl = w; sl < L.A.nslices; sl += nw)
      spmv_slice<B, 1, K, X, X, T, 2, kb_default<B>(), false, 2>(L.A, b, cur, static_cast<X*>(L.r), L.mask,
                                                                 slice_lane<B, 1>(L.A, sl, ln));
    __syncthreads();
    const TailLevel& C = lv[l - 1];
    for (int64_t t = threadIdx.x; t < int64_t(C.A.n) * B; t += blockDim.x)
      restrict_dof<B, 1, X, T>(L.R, static_cast<const X*>(L.r), static_cast<X*>(C.b), C.mask, nullptr, t);
    __syncthreads();
  }
  // coarse solve on level 0
  {
    const TailLevel& C = lv[0];
    X* x0 = static_cast<X*>(C.x);
    const X* b0 = static_cast<const X*>(C.b);
    if (p.coarse_mode == 0) {
      for (int i = w; i < p.n0; i += nw) gemv_row<X, X>(p.n0, p.Ainv, b0, x0, i, ln);
      __syncthreads();
    } else {
      const int k = p.coarse_sweeps > 1 ? p.coarse_sweeps : 1;
      X* tmp = static_cast<X*>(C.t);
      X* cur = ((k - 1) % 2 == 0) ? x0 : tmp;
      X* oth = ((k - 1) % 2 == 0) ? tmp : x0;
      for (int sl = w; sl < C.A.nslices; sl += nw)
        sweep0_slice<B, 1, X, T>(static_cast<const X*>(C.S), b0, cur, omega, slice_lane<B, 1>(C.A, sl, ln));
      __syncthreads();
      for (int q = 1; q < k; ++q) {
        tail_sweep<B, K, X, T>(C, b0, cur, oth, omega);
        X* t = cur; cur = oth; oth = t;
      }
    }
  }
  // ascent
  for (int l = 1; l <= p.top; ++l) {
    const TailLevel& L = lv[l];
    const TailLevel& C = lv[l - 1];
    X* own = static_cast<X*>(L.x);
    X* tmp = static_cast<X*>(L.t);
    X* cur = (pp % 2 == 0) ? own : tmp;
    X* oth = (pp % 2 == 0) ? tmp : own;
    if (pre_pp % 2 == 1) { X* t = cur; cur = oth; oth = t; }
    for (int64_t t = threadIdx.x; t < int64_t(L.A.n) * B; t += blockDim.x)
      prolong_dof<B, 1, X, T>(L.P, static_cast<const X*>(C.x), cur, L.mask, C.mask, t);
    __syncthreads();
    for (int q = 0; q < p.nu2; ++q) {
      tail_sweep<B, K, X, T>(L, static_cast<const X*>(L.b), cur, oth, omega);
      X* t = cur; cur = oth; oth = t;
    }
  }
}

// ------------------------------------------------------------------ setup kernels
// Gauss-Jordan step k, part 1 (one workgroup): pivot search in column k, row swap,
// pivot row scaled to 1 and copied to pivbuf.
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int k, double* M, double* pivbuf, int* flag) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  __shared__ double spv;
  const int w = 2 * n;
  double best = -1.0;
  int arg = k;
  for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(M[int64_t(i) * w + k]);
    if (a > best) { best = a; arg = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int p = bi[0];
  if (bv[0] <= 0.0) {
    if (threadIdx.x == 0) *flag = 1;
    return;
  }
  if (threadIdx.x == 0) spv = M[int64_t(p) * w + k];
  __syncthreads();
  const double pv = spv;
  for (int c = threadIdx.x; c < w; c += blockDim.x) {
    const double a = M[int64_t(k) * w + c], b = M[int64_t(p) * w + c];
    pivbuf[c] = b / pv;
    M[int64_t(p) * w + c] = a;        // old row k moves to row p (no-op when p == k)
  }
  __syncthreads();
  for (int c = threadIdx.x; c < w; c += blockDim.x) M[int64_t(k) * w + c] = pivbuf[c];
}

// Gauss-Jordan step k, part 2: eliminate column k from every other row
__global__ __launch_bounds__(256) void k_gj_elim(int n, int k, double* M, const double* pivbuf, const int* flag) {
  if (*flag) return;
  const int w = 2 * n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * w) return;
  const int i = int(t / w), c = int(t % w);
  if (i == k || c == k) return;         // column k is cleared by k_gj_clear
  M[t] -= M[int64_t(i) * w + k] * pivbuf[c];
}

__global__ __launch_bounds__(256) void k_gj_clear(int n, int k, double* M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && i != k) M[int64_t(i) * 2 * n + k] = 0.0;
}

__global__ __launch_bounds__(256) void k_gj_extract(int n, const double* M, double* Ainv) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int i = int(t / n), j = int(t % n);
  Ainv[t] = M[int64_t(i) * 2 * n + n + j];
}

template <int B, int NR, class ST>
__global__ __launch_bounds__(256) void k_block_invert(SellDev A, ST* __restrict__ S, int* flag) {
  constexpr int R = kWave / (B * NR);
  constexpr int W = kWave / NR;
  const int pos = blockIdx.x * blockDim.x + threadIdx.x;   // row position; S in lane layout
  if (pos >= A.n) return;
  const int node = A.perm ? A.perm[pos] : pos;
  const int slice = pos / R, r = pos % R;
  const double* val = static_cast<const double*>(A.val);
  int kd = -1;
  for (int k = A.sptr[slice]; k < A.sptr[slice + 1]; ++k)
    if (A.col[int64_t(k) * R + r] == node) { kd = k; break; }
  if (kd < 0) { *flag = 1; return; }
  double m[B][2 * B];
  for (int c = 0; c < B; ++c)
    for (int cc = 0; cc < B; ++cc) {
      m[c][cc] = val[(int64_t(kd) * B + cc) * W + r * B + c];
      m[c][B + cc] = (c == cc) ? 1.0 : 0.0;
    }
  for (int k = 0; k < B; ++k) {
    int p = k;
    for (int i = k + 1; i < B; ++i)
      if (fabs(m[i][k]) > fabs(m[p][k])) p = i;
    if (m[p][k] == 0.0) { *flag = 1; return; }
    if (p != k)
      for (int c = 0; c < 2 * B; ++c) { const double t = m[k][c]; m[k][c] = m[p][c]; m[p][c] = t; }
    const double inv = 1.0 / m[k][k];
    for (int c = 0; c < 2 * B; ++c) m[k][c] *= inv;
    for (int i = 0; i < B; ++i) {
      if (i == k) continue;
      const double f = m[i][k];
      for (int c = 0; c < 2 * B; ++c) m[i][c] -= f * m[k][c];
    }
  }
  for (int c = 0; c < B; ++c)
    for (int cc = 0; cc < B; ++cc) S[(int64_t(slice) * B + cc) * W + r * B + c] = ST(m[c][B + cc]);
}

// ------------------------------------------------------------------ vector kernels
template <class Y>
__global__ void k_fill(int64_t n, Y* y, double v) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = Y(v);
}

template <class X, class Y>
__global__ void k_convert(int64_t n, const X* __restrict__ x, Y* __restrict__ y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = Y(x[t]);
}

template <class Y, class X>
__global__ void k_axpy(int64_t n, Y* __restrict__ y, const X* __restrict__ x, double sign,
                       const double* __restrict__ alpha) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = Y(double(y[t]) + sign * (*alpha) * double(x[t]));
}

__global__ void k_scale_div(int64_t n, double* __restrict__ y, const double* __restrict__ x,
                            const double* __restrict__ denom, float* __restrict__ yc) {
  const double d = *denom;
  if (d == 0.0) return;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) {
    const double v = x[t] / d;
    y[t] = v;
    if (yc) yc[t] = float(v);
  }
}

// partial sums of a.b (b == nullptr: a.a), one per block
__global__ __launch_bounds__(kRedThreads) void k_dot_partials(int64_t n, const double* __restrict__ a,
                                                              const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double lds[kMaxWaves + 1];
  constexpr int U = 4;                     // elements per thread and round, loads first
  double t = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < n; i0 += stride * U) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      av[u] = i < n ? a[i] : 0.0;
      bv[u] = (b && i < n) ? b[i] : av[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) t += av[u] * bv[u];
  }
  const double s = block_allsum(t, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// out = sum (or sqrt of the sum) of partials, one workgroup
__global__ __launch_bounds__(1024) void k_finish(const double* __restrict__ p, int g, double* out, int sq) {
  __shared__ double lds[kMaxWaves + 1];
  const double s = sum_partials(p, g, lds);
  if (threadIdx.x == 0) *out = sq ? sqrt(s) : s;
}

// modified Gram-Schmidt step: h = sum(pin) (= (w, v_i)), stored by block 0;
// w -= h v_i; partial sums of (w, vnext) or, for vnext == nullptr, of (w, w)
__global__ __launch_bounds__(kRedThreads) void k_mgs_step(int64_t n, double* __restrict__ w,
                                                          const double* __restrict__ vi,
                                                          const double* __restrict__ vnext,
                                                          const double* __restrict__ pin, int gin,
                                                          double* __restrict__ pout, double* __restrict__ hout) {
  __shared__ double lds[kMaxWaves + 1];
  constexpr int U = 4;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  double wv[U], vv[U], nv[U];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      const bool ok = i < n;
      wv[u] = ok ? w[i] : 0.0;
      vv[u] = ok ? vi[i] : 0.0;
      nv[u] = (ok && vnext) ? vnext[i] : 0.0;
    }
  };
  // the first chunk's loads do not depend on h: issue them before the partial sums are
  // combined, so the two latencies overlap
  const int64_t first = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  load(first);
  const double h = sum_partials(pin, gin, lds);
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = h;
  double t = 0.0;
  for (int64_t i0 = first; i0 < n; i0 += stride * U) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      const double v = wv[u] - h * vv[u];
      if (i < n) w[i] = v;
      t += v * (vnext ? nv[u] : v);
    }
  }
  const double s = block_allsum(t, lds);
  if (threadIdx.x == 0) pout[blockIdx.x] = s;
}

// Givens rotation j of the Hessenberg column j (applies the previous rotations, forms the
// new one, rotates g); st receives |g_{j+1}| and the breakdown flag
__device__ __forceinline__ void givens_column(int j, int m, double* H, double* cs, double* sn, double* g,
                                              double* st) {
  const int ld = m + 1;
  double* h = H + int64_t(j) * ld;
  const bool breakdown = h[j + 1] == 0.0;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * h[i] + sn[i] * h[i + 1];
    h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
    h[i] = t;
  }
  const double den = hypot(h[j], h[j + 1]);
  cs[j] = h[j] / den;
  sn[j] = h[j + 1] / den;
  h[j] = den;
  h[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  st[0] = fabs(g[j + 1]);
  st[1] = breakdown ? 1.0 : 0.0;
  __threadfence_system();                  // st may be host memory read after the step
}

// nrm = sqrt(sum(pin)), stored by block 0; w /= nrm (unless nrm == 0).  With gv given,
// block 0 then applies Givens rotation gv->j to the finished Hessenberg column; with wc
// given, the normalised vector is also written in FP32 (the next V-cycle's input).
struct GivensArgs {
  int j, m;
  double *H, *cs, *sn, *g, *st;
};

// hout is the Hessenberg entry (j+1, j) that the Givens step reads back through gv.H: it
// must not be declared non-aliasing
__global__ __launch_bounds__(kRedThreads) void k_mgs_normalize(int64_t n, double* __restrict__ w,
                                                               const double* __restrict__ pin, int gin,
                                                               double* hout, GivensArgs gv,
                                                               float* __restrict__ wc) {
  __shared__ double lds[kMaxWaves + 1];
  constexpr int U = 4;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  double wv[U];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      wv[u] = i < n ? w[i] : 0.0;
    }
  };
  const int64_t first = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  load(first);                             // independent of the norm (latency overlap)
  const double nrm = sqrt(sum_partials(pin, gin, lds));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *hout = nrm;
    if (gv.H) givens_column(gv.j, gv.m, gv.H, gv.cs, gv.sn, gv.g, gv.st);
  }
  if (nrm == 0.0) {
    if (wc)
      for (int64_t i = first; i < n; i += stride) wc[i] = float(w[i]);
    return;
  }
  for (int64_t i0 = first; i0 < n; i0 += stride * U) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
        const double v = wv[u] / nrm;
        w[i] = v;
        if (wc) wc[i] = float(v);
      }
    }
  }
}

template <class Z>
__global__ void k_update_x(int64_t n, double* __restrict__ x, const Z* __restrict__ Zm, int64_t ldz,
                           const double* __restrict__ y, int k) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double acc = x[t];
  for (int i = 0; i < k; ++i) acc += y[i] * double(Zm[int64_t(i) * ldz + t]);
  x[t] = acc;
}



__global__ void k_backsolve(int k, int m, const double* H, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int ld = m + 1;
  for (int i = k - 1; i >= 0; --i) {
    double t = g[i];
    for (int c = i + 1; c < k; ++c) t -= H[int64_t(c) * ld + i] * y[c];
    y[i] = t / H[int64_t(i) * ld + i];
  }
}

__global__ void k_init_g(int m, double* g, const double* beta) {
  const int t = threadIdx.x;
  if (t <= m) g[t] = (t == 0) ? *beta : 0.0;
}

// ------------------------------------------------------------------ launch helpers

template <int B, int K, class XI, class XO, class T>
hipError_t spmv_t(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask, int mode,
                  double* partials, const double* dotv, hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  const XO* bb = static_cast<const XO*>(b);
  const XI* xx = static_cast<const XI*>(x);
  XO* yy = static_cast<XO*>(y);
  // slot batch and column format are runtime properties of the operator
#define MGQ1_SPMV4(MODE, NORM, KB, C16)                                                                     \
  hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, MODE, NORM, KB, C16>), g, kThreads, dict_lds_bytes<K>(A), s, A, bb, xx, yy, mask, partials, \
                     dotv)
#define MGQ1_SPMV(MODE, NORM)                                                             \
  if (A.col16) {                                                                          \
    if (A.kb == kb_alt<B>()) MGQ1_SPMV4(MODE, NORM, kb_alt<B>(), true);                   \
    else MGQ1_SPMV4(MODE, NORM, kb_default<B>(), true);                                   \
  } else {                                                                                \
    if (A.kb == kb_alt<B>()) MGQ1_SPMV4(MODE, NORM, kb_alt<B>(), false);                  \
    else MGQ1_SPMV4(MODE, NORM, kb_default<B>(), false);                                  \
  }
  // the combinations the library uses: y = Ax, b - Ax with or without norm partials,
  // masked defect
  if (mode == 0 && !partials) MGQ1_SPMV(0, false)
  else if (mode == 0 && dotv) MGQ1_SPMV(0, true)
  else if (mode == 1 && partials && !dotv) MGQ1_SPMV(1, true)
  else if (mode == 1) MGQ1_SPMV(1, false)
  else if (mode == 2 && !partials) MGQ1_SPMV(2, false)
  else return hipErrorInvalidValue;
#undef MGQ1_SPMV4
#undef MGQ1_SPMV
  return hipGetLastError();
}

template <int B>
hipError_t spmv_b(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask, int xk, int yk,
                  int mode, double* partials, const double* dotv, hipStream_t s) {
  if (A.kind == VK_DICT) {
    if (xk == X_F64 && yk == X_F64) return spmv_t<B, VK_DICT, double, double, double>(A, b, x, y, mask, mode, partials, dotv, s);
    return hipErrorInvalidValue;
  }
  if (A.kind == VK_F64) {
    if (xk == X_F64 && yk == X_F64) return spmv_t<B, VK_F64, double, double, double>(A, b, x, y, mask, mode, partials, dotv, s);
    if (xk == X_F32 && yk == X_F64) return spmv_t<B, VK_F64, float, double, double>(A, b, x, y, mask, mode, partials, dotv, s);
    return hipErrorInvalidValue;
  }
  if (xk != X_F32 || yk != X_F32) return hipErrorInvalidValue;
  switch (A.kind) {
    case VK_F32: return spmv_t<B, VK_F32, float, float, float>(A, b, x, y, mask, mode, partials, dotv, s);
    case VK_F16: return spmv_t<B, VK_F16, float, float, float>(A, b, x, y, mask, mode, partials, dotv, s);
    case VK_BF16: return spmv_t<B, VK_BF16, float, float, float>(A, b, x, y, mask, mode, partials, dotv, s);
    default: return hipErrorInvalidValue;
  }
}

template <int B, class X, class T>
hipError_t sweep_t(const SellDev& A, const void* S, const void* b, const void* x, void* xo, double omega,
                   double beta, int pmode, hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  const X* SS = static_cast<const X*>(S);
  const X* bb = static_cast<const X*>(b);
  const X* xx = static_cast<const X*>(x);
  X* oo = static_cast<X*>(xo);
#define MGQ1_SWEEP4(KIND, KB, C16) \
  hipLaunchKernelGGL((k_sweep<B, KIND, X, T, KB, C16>), g, kThreads, dict_lds_bytes<KIND>(A), s, A, SS, bb, xx, oo, T(omega), T(beta), pmode)
#define MGQ1_SWEEP(KIND)                                                   \
  if (A.col16) {                                                           \
    if (A.kb == kb_alt<B>()) MGQ1_SWEEP4(KIND, kb_alt<B>(), true);         \
    else MGQ1_SWEEP4(KIND, kb_default<B>(), true);                         \
  } else {                                                                 \
    if (A.kb == kb_alt<B>()) MGQ1_SWEEP4(KIND, kb_alt<B>(), false);        \
    else MGQ1_SWEEP4(KIND, kb_default<B>(), false);                        \
  }
  // FP64 vectors go with FP64 values only; FP32 vectors with the reduced formats
  if constexpr (sizeof(X) == 8) {
    if (A.kind == VK_DICT) {
      MGQ1_SWEEP(VK_DICT);
    } else {
      if (A.kind != VK_F64) return hipErrorInvalidValue;
      MGQ1_SWEEP(VK_F64);
    }
  } else {
    switch (A.kind) {
      case VK_F32: MGQ1_SWEEP(VK_F32); break;
      case VK_F16: MGQ1_SWEEP(VK_F16); break;
      case VK_BF16: MGQ1_SWEEP(VK_BF16); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef MGQ1_SWEEP
#undef MGQ1_SWEEP4
  return hipGetLastError();
}

template <int B, int K, class X, class T>
hipError_t tail_t(const TailLevel* lv, const TailParams& p, hipStream_t s) {
  hipLaunchKernelGGL((k_tail<B, K, X, T>), 1, kTailThreads, 0, s, lv, p);
  return hipGetLastError();
}

template <int B>
hipError_t tail_b(const TailLevel* lv, int kind, int xk, const TailParams& p, hipStream_t s) {
  if (xk == X_F64) {
    if (kind != VK_F64) return hipErrorInvalidValue;
    return tail_t<B, VK_F64, double, double>(lv, p, s);
  }
  switch (kind) {
    case VK_F32: return tail_t<B, VK_F32, float, float>(lv, p, s);
    case VK_F16: return tail_t<B, VK_F16, float, float>(lv, p, s);
    case VK_BF16: return tail_t<B, VK_BF16, float, float>(lv, p, s);
    default: return hipErrorInvalidValue;
  }
}

inline unsigned vec_grid(int64_t n) {
  unsigned g = grid_for(n, int64_t(kRedThreads) * 4);   // 4 elements per thread and round
  if (g > unsigned(kMaxRedBlocks)) g = kMaxRedBlocks;
  return g ? g : 1;
}

}  // namespace

int reduction_grid(int64_t n) { return int(vec_grid(n)); }

void slot_batch_choices(int B, int* kb_def, int* kb_other) {
  switch (B) {
    case 1: *kb_def = kb_default<1>(); *kb_other = kb_alt<1>(); break;
    case 2: *kb_def = kb_default<2>(); *kb_other = kb_alt<2>(); break;
    case 3: *kb_def = kb_default<3>(); *kb_other = kb_alt<3>(); break;
    default: *kb_def = kb_default<4>(); *kb_other = kb_alt<4>(); break;
  }
}
int spmv_grid(const SellDev& A) { return int(slice_grid(A.nslices)); }

hipError_t launch_spmv(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask, int xk, int yk,
                       int mode, double* partials, hipStream_t s, const double* dotv) {
  switch (A.B) {
    case 1: return spmv_b<1>(A, b, x, y, mask, xk, yk, mode, partials, dotv, s);
    case 2: return spmv_b<2>(A, b, x, y, mask, xk, yk, mode, partials, dotv, s);
    case 3: return spmv_b<3>(A, b, x, y, mask, xk, yk, mode, partials, dotv, s);
    case 4: return spmv_b<4>(A, b, x, y, mask, xk, yk, mode, partials, dotv, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep(const SellDev& A, const void* S, const void* b, const void* x, void* xo, double omega,
                        int xk, hipStream_t s, double beta, int pmode) {
  if (xk == X_F64) {
    switch (A.B) {
      case 1: return sweep_t<1, double, double>(A, S, b, x, xo, omega, beta, pmode, s);
      case 2: return sweep_t<2, double, double>(A, S, b, x, xo, omega, beta, pmode, s);
      case 3: return sweep_t<3, double, double>(A, S, b, x, xo, omega, beta, pmode, s);
      case 4: return sweep_t<4, double, double>(A, S, b, x, xo, omega, beta, pmode, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (A.B) {
    case 1: return sweep_t<1, float, float>(A, S, b, x, xo, omega, beta, pmode, s);
    case 2: return sweep_t<2, float, float>(A, S, b, x, xo, omega, beta, pmode, s);
    case 3: return sweep_t<3, float, float>(A, S, b, x, xo, omega, beta, pmode, s);
    case 4: return sweep_t<4, float, float>(A, S, b, x, xo, omega, beta, pmode, s);
    default: return hipErrorInvalidValue;
  }
}

template <int B>
static hipError_t sweep0_b(const SellDev& A, const void* S, const void* b, void* xo, double omega, int xk,
                           hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  if (xk == X_F64)
    hipLaunchKernelGGL((k_sweep0<B, double, double>), g, kThreads, 0, s, A, static_cast<const double*>(S),
                       static_cast<const double*>(b), static_cast<double*>(xo), omega);
  else
    hipLaunchKernelGGL((k_sweep0<B, float, float>), g, kThreads, 0, s, A, static_cast<const float*>(S),
                       static_cast<const float*>(b), static_cast<float*>(xo), float(omega));
  return hipGetLastError();
}

hipError_t launch_sweep2z(const SellDev& A, const void* S, const void* b, void* xo, double omega, int xk,
                          hipStream_t s) {
  if (A.B != 1 || A.perm != nullptr) return hipErrorInvalidValue;   // node order = lane order
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
#define MGQ1_S2Z4(KIND, X, T, KB, C16)                                                              \
  hipLaunchKernelGGL((k_sweep2z<KIND, X, T, KB, C16>), g, kThreads, 0, s, A, static_cast<const X*>(S), \
                     static_cast<const X*>(b), static_cast<X*>(xo), T(omega))
#define MGQ1_S2Z(KIND, X, T)                                                     \
  if (A.col16) {                                                                 \
    if (A.kb == kb_alt<1>()) MGQ1_S2Z4(KIND, X, T, kb_alt<1>(), true);           \
    else MGQ1_S2Z4(KIND, X, T, kb_default<1>(), true);                           \
  } else {                                                                       \
    if (A.kb == kb_alt<1>()) MGQ1_S2Z4(KIND, X, T, kb_alt<1>(), false);          \
    else MGQ1_S2Z4(KIND, X, T, kb_default<1>(), false);                          \
  }
  if (xk == X_F64) {
    if (A.kind != VK_F64) return hipErrorInvalidValue;
    MGQ1_S2Z(VK_F64, double, double);
  } else {
    switch (A.kind) {
      case VK_F32: MGQ1_S2Z(VK_F32, float, float); break;
      case VK_F16: MGQ1_S2Z(VK_F16, float, float); break;
      case VK_BF16: MGQ1_S2Z(VK_BF16, float, float); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef MGQ1_S2Z
#undef MGQ1_S2Z4
  return hipGetLastError();
}

hipError_t launch_sweep0(const SellDev& A, const void* S, const void* b, void* xo, double omega, int xk,
                         hipStream_t s) {
  switch (A.B) {
    case 1: return sweep0_b<1>(A, S, b, xo, omega, xk, s);
    case 2: return sweep0_b<2>(A, S, b, xo, omega, xk, s);
    case 3: return sweep0_b<3>(A, S, b, xo, omega, xk, s);
    case 4: return sweep0_b<4>(A, S, b, xo, omega, xk, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int B, class X, class T, class WT>
hipError_t tsell_w(int mode, const TSellDev& M, const void* in, void* out, const uint8_t* mrow,
                   const uint8_t* mcol, hipStream_t s) {
  const unsigned g = slice_grid(M.nslices);
  if (g == 0) return hipSuccess;
  const X* ii = static_cast<const X*>(in);
  X* oo = static_cast<X*>(out);
  if (mode == 0) {
    if (mcol) hipLaunchKernelGGL((k_tsell<B, 1, X, T, WT, true, 0>), g, kThreads, 0, s, M, ii, oo, mrow, mcol);
    else hipLaunchKernelGGL((k_tsell<B, 1, X, T, WT, false, 0>), g, kThreads, 0, s, M, ii, oo, mrow, mcol);
  } else {
    hipLaunchKernelGGL((k_tsell<B, 1, X, T, WT, true, 1>), g, kThreads, 0, s, M, ii, oo, mrow, mcol);
  }
  return hipGetLastError();
}

template <int B>
hipError_t tsell_b(int mode, const TSellDev& M, const void* in, void* out, const uint8_t* mrow,
                   const uint8_t* mcol, int xk, hipStream_t s) {
  if (xk == X_F64)
    return M.f32 ? tsell_w<B, double, double, float>(mode, M, in, out, mrow, mcol, s)
                 : tsell_w<B, double, double, double>(mode, M, in, out, mrow, mcol, s);
  return M.f32 ? tsell_w<B, float, float, float>(mode, M, in, out, mrow, mcol, s)
               : tsell_w<B, float, float, double>(mode, M, in, out, mrow, mcol, s);
}

template <int B, class X>
hipError_t tnode_x(int mode, const TSellDev& M, const void* in, void* out, bool mc, hipStream_t s) {
  const unsigned g = slice_grid(M.nslices);
  if (g == 0) return hipSuccess;
  const X* ii = static_cast<const X*>(in);
  X* oo = static_cast<X*>(out);
  if (mode == 1) hipLaunchKernelGGL((k_tnode<B, X, X, true, 1>), g, kThreads, 0, s, M, ii, oo);
  else if (mc) hipLaunchKernelGGL((k_tnode<B, X, X, true, 0>), g, kThreads, 0, s, M, ii, oo);
  else hipLaunchKernelGGL((k_tnode<B, X, X, false, 0>), g, kThreads, 0, s, M, ii, oo);
  return hipGetLastError();
}

template <int B>
hipError_t tnode_b(int mode, const TSellDev& M, const void* in, void* out, bool mc, int xk, hipStream_t s) {
  return xk == X_F64 ? tnode_x<B, double>(mode, M, in, out, mc, s) : tnode_x<B, float>(mode, M, in, out, mc, s);
}

// node form: the row and column masks are the ones built into the layout (the levels' own
// masks); mcol only says whether the column mask applies
hipError_t tnode_launch(int mode, const TSellDev& M, int B, const void* in, void* out, const uint8_t* mcol, int xk,
                        hipStream_t s) {
  if (M.R != kWave) return hipErrorInvalidValue;
  switch (B) {
    case 1: return tnode_b<1>(mode, M, in, out, mcol != nullptr, xk, s);
    case 2: return tnode_b<2>(mode, M, in, out, mcol != nullptr, xk, s);
    case 3: return tnode_b<3>(mode, M, in, out, mcol != nullptr, xk, s);
    case 4: return tnode_b<4>(mode, M, in, out, mcol != nullptr, xk, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t tsell_launch(int mode, const TSellDev& M, int B, const void* in, void* out, const uint8_t* mrow,
                        const uint8_t* mcol, int xk, hipStream_t s) {
  if (M.node) return tnode_launch(mode, M, B, in, out, mcol, xk, s);
  if (M.R != kWave / B) return hipErrorInvalidValue;     // single right-hand-side layout
  switch (B) {
    case 1: return tsell_b<1>(mode, M, in, out, mrow, mcol, xk, s);
    case 2: return tsell_b<2>(mode, M, in, out, mrow, mcol, xk, s);
    case 3: return tsell_b<3>(mode, M, in, out, mrow, mcol, xk, s);
    case 4: return tsell_b<4>(mode, M, in, out, mrow, mcol, xk, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_restrict_s(const TSellDev& R, int B, const void* r, void* d, const uint8_t* mask_c,
                             const uint8_t* mask_f, int xk, hipStream_t s) {
  return tsell_launch(0, R, B, r, d, mask_c, mask_f, xk, s);
}

hipError_t launch_prolong_s(const TSellDev& P, int B, const void* y, void* x, const uint8_t* mask_f,
                            const uint8_t* mask_c, int xk, hipStream_t s) {
  return tsell_launch(1, P, B, y, x, mask_f, mask_c, xk, s);
}


hipError_t launch_tail(const TailLevel* lv, int B, int kind, int xk, const TailParams& p, hipStream_t s) {
  switch (B) {
    case 1: return tail_b<1>(lv, kind, xk, p, s);
    case 2: return tail_b<2>(lv, kind, xk, p, s);
    case 3: return tail_b<3>(lv, kind, xk, p, s);
    case 4: return tail_b<4>(lv, kind, xk, p, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarse_gemv(int n, const double* Ainv, const void* b, void* x, int xk, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, kSliceWaves);
  if (xk == X_F64)
    hipLaunchKernelGGL((k_coarse_gemv<double, double>), g, kThreads, 0, s, n, Ainv, static_cast<const double*>(b),
                       static_cast<double*>(x));
  else
    hipLaunchKernelGGL((k_coarse_gemv<float, float>), g, kThreads, 0, s, n, Ainv, static_cast<const float*>(b),
                       static_cast<float*>(x));
  return hipGetLastError();
}

hipError_t launch_coarse_invert(int n, double* M, double* Ainv, double* pivbuf, int* flag, hipStream_t s) {
  const int64_t tot = int64_t(n) * 2 * n;
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, 1, 1024, 0, s, n, k, M, pivbuf, flag);
    hipLaunchKernelGGL(k_gj_elim, grid_for(tot, 256), 256, 0, s, n, k, M, pivbuf, flag);
    hipLaunchKernelGGL(k_gj_clear, grid_for(n, 256), 256, 0, s, n, k, M);
  }
  hipLaunchKernelGGL(k_gj_extract, grid_for(int64_t(n) * n, 256), 256, 0, s, n, M, Ainv);
  return hipGetLastError();
}

hipError_t launch_block_invert(const SellDev& A, void* S, int sk, int* flag, int NR, hipStream_t s) {
  const unsigned g = grid_for(A.n, 256);
  if (g == 0) return hipSuccess;
#define MGQ1_BI(BB, NN)                                                                                           \
  if (sk == X_F64) hipLaunchKernelGGL((k_block_invert<BB, NN, double>), g, 256, 0, s, A, static_cast<double*>(S), flag); \
  else hipLaunchKernelGGL((k_block_invert<BB, NN, float>), g, 256, 0, s, A, static_cast<float*>(S), flag);
  if (NR == 8) {
    if (A.B != 1) return hipErrorInvalidValue;
    MGQ1_BI(1, 8)
    return hipGetLastError();
  }
  switch (A.B) {
    case 1: MGQ1_BI(1, 1) break;
    case 2: MGQ1_BI(2, 1) break;
    case 3: MGQ1_BI(3, 1) break;
    case 4: MGQ1_BI(4, 1) break;
    default: return hipErrorInvalidValue;
  }
#undef MGQ1_BI
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, void* y, int yk, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (yk == X_F64) hipLaunchKernelGGL(k_fill<double>, grid_for(n, 256), 256, 0, s, n, static_cast<double*>(y), v);
  else hipLaunchKernelGGL(k_fill<float>, grid_for(n, 256), 256, 0, s, n, static_cast<float*>(y), v);
  return hipGetLastError();
}

hipError_t launch_convert(int64_t n, const void* x, int xk, void* y, int yk, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (xk == X_F64 && yk == X_F32)
    hipLaunchKernelGGL((k_convert<double, float>), g, 256, 0, s, n, static_cast<const double*>(x), static_cast<float*>(y));
  else if (xk == X_F32 && yk == X_F64)
    hipLaunchKernelGGL((k_convert<float, double>), g, 256, 0, s, n, static_cast<const float*>(x), static_cast<double*>(y));
  else if (xk == X_F64 && yk == X_F64)
    hipLaunchKernelGGL((k_convert<double, double>), g, 256, 0, s, n, static_cast<const double*>(x), static_cast<double*>(y));
  else
    hipLaunchKernelGGL((k_convert<float, float>), g, 256, 0, s, n, static_cast<const float*>(x), static_cast<float*>(y));
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, void* y, int yk, const void* x, int xk, double sign, const double* alpha,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (yk == X_F64 && xk == X_F64)
    hipLaunchKernelGGL((k_axpy<double, double>), g, 256, 0, s, n, static_cast<double*>(y), static_cast<const double*>(x), sign, alpha);
  else if (yk == X_F64 && xk == X_F32)
    hipLaunchKernelGGL((k_axpy<double, float>), g, 256, 0, s, n, static_cast<double*>(y), static_cast<const float*>(x), sign, alpha);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_scale_div(int64_t n, double* y, const double* x, const double* denom, hipStream_t s, float* yc) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_div, grid_for(n, 256), 256, 0, s, n, y, x, denom, yc);
  return hipGetLastError();
}

hipError_t launch_dot_partials(int64_t n, const double* a, const double* b, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, vec_grid(n), kRedThreads, 0, s, n, a, b, partials);
  return hipGetLastError();
}

hipError_t launch_finish(const double* partials, int g, double* out, int sqrt_out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, 1, 1024, 0, s, partials, g, out, sqrt_out);
  return hipGetLastError();
}

hipError_t launch_mgs_step(int64_t n, double* w, const double* vi, const double* vnext, const double* pin,
                           double* pout, double* hout, hipStream_t s, int gin) {
  const unsigned g = vec_grid(n);
  hipLaunchKernelGGL(k_mgs_step, g, kRedThreads, 0, s, n, w, vi, vnext, pin, gin > 0 ? gin : int(g), pout, hout);
  return hipGetLastError();
}

hipError_t launch_mgs_normalize(int64_t n, double* w, const double* pin, double* hout, hipStream_t s, int gj,
                                int gm, double* H, double* cs, double* sn, double* gg, double* st, float* wc) {
  const unsigned g = vec_grid(n);
  GivensArgs gv{gj, gm, H, cs, sn, gg, st};
  hipLaunchKernelGGL(k_mgs_normalize, g, kRedThreads, 0, s, n, w, pin, int(g), hout, gv, wc);
  return hipGetLastError();
}

hipError_t launch_update_x(int64_t n, double* x, const void* Z, int zk, int64_t ldz, const double* y, int k,
                           hipStream_t s) {
  if (n == 0 || k == 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (zk == X_F64)
    hipLaunchKernelGGL(k_update_x<double>, g, 256, 0, s, n, x, static_cast<const double*>(Z), ldz, y, k);
  else
    hipLaunchKernelGGL(k_update_x<float>, g, 256, 0, s, n, x, static_cast<const float*>(Z), ldz, y, k);
  return hipGetLastError();
}

hipError_t launch_backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, 1, 64, 0, s, k, m, H, g, y);
  return hipGetLastError();
}

hipError_t launch_init_g(int m, double* g, const double* beta, hipStream_t s) {
  hipLaunchKernelGGL(k_init_g, 1, 128, 0, s, m, g, beta);
  return hipGetLastError();
}

}  // namespace mgq1
