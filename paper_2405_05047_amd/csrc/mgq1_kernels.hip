// HIP kernels of the multigrid hot path for gfx950 (MI355X).
//
// Every kernel here streams sparse data and is bound by HBM bandwidth (about 0.1-0.25
// flop per byte in FP64), so there is no matrix-core work: the design goals are coalesced
// value / index streams, cached gathers of x, one pass over A per smoothing sweep and
// deterministic reductions (no floating-point atomics).
//
//   SELL slice kernels (defect / SpMV, smoothing sweep): one wavefront per slice of
//   64/B nodes; lane = node*B + component owns one scalar row.  For every block slot the
//   wave issues B fully coalesced 512-byte value loads and one load of the R column
//   indices, gathers x[col*B + cc] (L2 / MALL hits: neighbouring slices share columns),
//   and accumulates in registers.  The smoother exchanges the B residual components of a
//   node across its lanes with wave shuffles and applies the stored block inverse.
//   Workgroup ids are remapped so that each XCD (round-robin dispatch over 8 XCDs) walks
//   a contiguous range of slices and keeps its own L2 warm.
//
// Paper correspondence: smoother x + omega S (b - A x) and transfers P, R = P^T
// (Sec. 4.1 "Geometric Multigrid CUDA"); GMRES building blocks (Sec. 4.2).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kThreads = kWave * kSliceWaves;   // 256

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  // hardware dispatch sends workgroup w to XCD w % 8; give XCD x a contiguous range
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + (x < r ? x : r) + k;
}

template <int K> struct Val;
template <> struct Val<VK_F64> {
  using T = double;
  __device__ __forceinline__ static double get(const void* p, int64_t i, float) {
    return __builtin_nontemporal_load(static_cast<const double*>(p) + i);
  }
};
template <> struct Val<VK_F32> {
  using T = float;
  __device__ __forceinline__ static float get(const void* p, int64_t i, float) {
    return __builtin_nontemporal_load(static_cast<const float*>(p) + i);
  }
};
template <> struct Val<VK_F16> {
  using T = float;
  __device__ __forceinline__ static float get(const void* p, int64_t i, float sc) {
    const unsigned short u = __builtin_nontemporal_load(static_cast<const unsigned short*>(p) + i);
    return sc * __half2float(__ushort_as_half(u));
  }
};
template <> struct Val<VK_BF16> {
  using T = float;
  __device__ __forceinline__ static float get(const void* p, int64_t i, float sc) {
    const unsigned short u = __builtin_nontemporal_load(static_cast<const unsigned short*>(p) + i);
    return sc * __uint_as_float(static_cast<uint32_t>(u) << 16);
  }
};

// per-lane row dot product of a slice: sum_k sum_cc a(k, cc) x[col_k * B + cc]
template <int B, int K, class XI, class T>
__device__ __forceinline__ T sell_dot(const SellDev& A, int slice, int lane, bool valid,
                                      const XI* __restrict__ x) {
  constexpr int R = kWave / B;
  T acc = T(0);
  if (!valid) return acc;
  float sc = 1.0f;
  if (K == VK_F16 || K == VK_BF16) sc = ldexpf(1.0f, A.rexp[int64_t(slice) * kWave + lane]);
  const int r = lane / B;
  const int k0 = A.sptr[slice], k1 = A.sptr[slice + 1];
  const int32_t* colp = A.col + int64_t(k0) * R + r;
  int64_t vb = int64_t(k0) * B * kWave + lane;
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const int j = __builtin_nontemporal_load(colp);
    colp += R;
    const XI* xj = x + int64_t(j) * B;
#pragma unroll
    for (int cc = 0; cc < B; ++cc) acc += T(Val<K>::get(A.val, vb + cc * kWave, sc)) * T(xj[cc]);
    vb += B * kWave;
  }
  return acc;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}

// block sum (256 threads) -> thread 0
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  if (ln == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < int(blockDim.x / kWave); ++q) t += lds[q];
  __syncthreads();
  return t;
}

// store this block's partial; the last block to arrive sums all partials in block order
__device__ void finish_reduction(double part, const RedDev& red, double* lds) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    red.partials[blockIdx.x] = part;
    __threadfence();
    const unsigned prev = atomicAdd(red.counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double t = 0.0;
  for (int q = threadIdx.x; q < int(gridDim.x); q += blockDim.x)
    t += __hip_atomic_load(red.partials + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t = block_sum(t, lds);
  if (threadIdx.x == 0) {
    *red.out = red.sqrt_out ? sqrt(t) : t;
    *red.counter = 0u;
  }
}

template <int B, int K, class XI, class XO, class T, int MODE, bool NORM>
__global__ __launch_bounds__(kThreads) void k_spmv(SellDev A, const XO* __restrict__ b,
                                                   const XI* __restrict__ x, XO* __restrict__ y,
                                                   const uint8_t* __restrict__ mask, RedDev red) {
  constexpr int R = kWave / B;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int slice = bid * kSliceWaves + wave;
  const int node = slice * R + lane / B;
  const bool valid = slice < A.nslices && lane < R * B && node < A.n;
  const T acc = sell_dot<B, K, XI, T>(A, slice, lane, valid, x);
  const int64_t dof = int64_t(slice) * R * B + lane;
  T out = T(0);
  if (valid) {
    if (MODE == 0) {
      out = acc;
    } else {
      out = T(b[dof]) - acc;
      if (MODE == 2 && mask[dof]) out = T(0);
    }
    y[dof] = XO(out);
  }
  if (NORM) {
    __shared__ double lds[kSliceWaves];
    const double p = block_sum(double(out) * double(out), lds);
    // keep the partial index in dispatch order: reductions stay deterministic
    finish_reduction(p, red, lds);
  }
}

template <int B, int K, class X, class T>
__global__ __launch_bounds__(kThreads) void k_sweep(SellDev A, const X* __restrict__ S,
                                                    const X* __restrict__ b, const X* __restrict__ x,
                                                    X* __restrict__ xo, T omega) {
  constexpr int R = kWave / B;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int slice = bid * kSliceWaves + wave;
  const int node = slice * R + lane / B;
  const bool valid = slice < A.nslices && lane < R * B && node < A.n;
  const T acc = sell_dot<B, K, X, T>(A, slice, lane, valid, x);
  const int64_t dof = int64_t(slice) * R * B + lane;
  const T res = valid ? T(b[dof]) - acc : T(0);
  const int base = (lane / B) * B;
  T upd = T(0);
#pragma unroll
  for (int cc = 0; cc < B; ++cc) {
    const T rc = __shfl(res, (base + cc) & (kWave - 1), kWave);
    if (valid) upd += T(S[(int64_t(slice) * B + cc) * kWave + lane]) * rc;
  }
  if (valid) xo[dof] = X(T(x[dof]) + omega * upd);
}

template <int B, class X, class T>
__global__ __launch_bounds__(kThreads) void k_sweep0(int n, int nslices, const X* __restrict__ S,
                                                     const X* __restrict__ b, X* __restrict__ xo,
                                                     T omega) {
  constexpr int R = kWave / B;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int slice = blockIdx.x * kSliceWaves + wave;
  const int node = slice * R + lane / B;
  if (!(slice < nslices && lane < R * B && node < n)) return;
  const int64_t dof = int64_t(slice) * R * B + lane;
  T upd = T(0);
#pragma unroll
  for (int cc = 0; cc < B; ++cc)
    upd += T(S[(int64_t(slice) * B + cc) * kWave + lane]) * T(b[int64_t(node) * B + cc]);
  xo[dof] = X(omega * upd);
}

template <int B, class X, class T, class W>
__global__ __launch_bounds__(kThreads) void k_restrict(int nc, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ rc,
                                                       const W* __restrict__ rv,
                                                       const X* __restrict__ r, X* __restrict__ d,
                                                       const uint8_t* __restrict__ mask_c,
                                                       const uint8_t* __restrict__ mask_f) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nc) * B) return;
  const int j = int(t / B), c = int(t % B);
  T acc = T(0);
  if (!mask_c[t]) {
    for (int k = rp[j]; k < rp[j + 1]; ++k) {
      const int64_t q = int64_t(rc[k]) * B + c;
      if (mask_f == nullptr || !mask_f[q]) acc += T(rv[k]) * T(r[q]);
    }
  }
  d[t] = X(acc);
}

template <int B, class X, class T, class W>
__global__ __launch_bounds__(kThreads) void k_prolong(int nf, const int32_t* __restrict__ pp,
                                                      const int32_t* __restrict__ pc,
                                                      const W* __restrict__ pv,
                                                      const X* __restrict__ y, X* __restrict__ x,
                                                      const uint8_t* __restrict__ mask_f,
                                                      const uint8_t* __restrict__ mask_c) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nf) * B) return;
  if (mask_f[t]) return;
  const int i = int(t / B), c = int(t % B);
  T acc = T(0);
  for (int k = pp[i]; k < pp[i + 1]; ++k) {
    const int64_t q = int64_t(pc[k]) * B + c;
    if (!mask_c[q]) acc += T(pv[k]) * T(y[q]);
  }
  x[t] = X(T(x[t]) + acc);
}

template <class XI, class XO>
__global__ __launch_bounds__(kThreads) void k_coarse_gemv(int n, const double* __restrict__ AinvT,
                                                          const XI* __restrict__ b, XO* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc += AinvT[int64_t(k) * n + i] * double(b[k]);
  x[i] = XO(acc);
}

// Gauss-Jordan step k, part 1 (one workgroup): pivot search in column k, row swap,
// pivot row scaled to 1 and copied to pivbuf.
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int k, double* M, double* pivbuf, int* flag) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
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
  __shared__ double spv;
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
__global__ __launch_bounds__(256) void k_gj_elim(int n, int k, double* M, const double* pivbuf,
                                                 const int* flag) {
  if (*flag) return;
  const int w = 2 * n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * w) return;
  const int i = int(t / w), c = int(t % w);
  if (i == k) return;
  const double f = M[int64_t(i) * w + k];
  if (c == k) return;                   // column k cleared after the row is done
  M[t] -= f * pivbuf[c];
}

__global__ __launch_bounds__(256) void k_gj_clear(int n, int k, double* M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && i != k) M[int64_t(i) * 2 * n + k] = 0.0;
}

__global__ __launch_bounds__(256) void k_gj_extract(int n, const double* M, double* AinvT) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int i = int(t / n), j = int(t % n);          // inverse entry (i, j)
  AinvT[int64_t(j) * n + i] = M[int64_t(i) * 2 * n + n + j];
}

template <int B, class ST>
__global__ __launch_bounds__(256) void k_block_invert(SellDev A, ST* __restrict__ S, int* flag) {
  constexpr int R = kWave / B;
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= A.n) return;
  const int slice = node / R, r = node % R;
  const double* val = static_cast<const double*>(A.val);
  int kd = -1;
  for (int k = A.sptr[slice]; k < A.sptr[slice + 1]; ++k)
    if (A.col[int64_t(k) * R + r] == node) { kd = k; break; }
  if (kd < 0) { *flag = 1; return; }
  double m[B][2 * B];
  for (int c = 0; c < B; ++c)
    for (int cc = 0; cc < B; ++cc) {
      m[c][cc] = val[(int64_t(kd) * B + cc) * kWave + r * B + c];
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
    for (int cc = 0; cc < B; ++cc) S[(int64_t(slice) * B + cc) * kWave + r * B + c] = ST(m[c][B + cc]);
}

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
                            const double* __restrict__ denom) {
  const double d = *denom;
  if (d == 0.0) return;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t] / d;
}

__global__ __launch_bounds__(kRedThreads) void k_dot(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, RedDev red) {
  __shared__ double lds[kRedThreads / kWave];
  double t = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    t += a[i] * (b ? b[i] : a[i]);
  const double p = block_sum(t, lds);
  finish_reduction(p, red, lds);
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

__global__ void k_givens(int j, int m, double* H, double* cs, double* sn, double* g, double* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
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

inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }
inline unsigned slice_grid(int nslices) { return unsigned((nslices + kSliceWaves - 1) / kSliceWaves); }

inline RedDev null_red() { return RedDev{}; }

template <int B, int K, class XI, class XO, class T>
hipError_t spmv_t(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask,
                  int mode, const RedDev* red, hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  const XO* bb = static_cast<const XO*>(b);
  const XI* xx = static_cast<const XI*>(x);
  XO* yy = static_cast<XO*>(y);
  const RedDev rd = red ? *red : null_red();
  if (red) {
    if (mode == 0) hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 0, true>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
    else if (mode == 1) hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 1, true>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
    else hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 2, true>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
  } else {
    if (mode == 0) hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 0, false>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
    else if (mode == 1) hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 1, false>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
    else hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, 2, false>), g, kThreads, 0, s, A, bb, xx, yy, mask, rd);
  }
  return hipGetLastError();
}

template <int B>
hipError_t spmv_b(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask, int xk,
                  int yk, int mode, const RedDev* red, hipStream_t s) {
  if (A.kind == VK_F64) {
    if (xk == X_F64 && yk == X_F64) return spmv_t<B, VK_F64, double, double, double>(A, b, x, y, mask, mode, red, s);
    if (xk == X_F32 && yk == X_F64) return spmv_t<B, VK_F64, float, double, double>(A, b, x, y, mask, mode, red, s);
    return hipErrorInvalidValue;
  }
  if (xk != X_F32 || yk != X_F32) return hipErrorInvalidValue;
  switch (A.kind) {
    case VK_F32: return spmv_t<B, VK_F32, float, float, float>(A, b, x, y, mask, mode, red, s);
    case VK_F16: return spmv_t<B, VK_F16, float, float, float>(A, b, x, y, mask, mode, red, s);
    case VK_BF16: return spmv_t<B, VK_BF16, float, float, float>(A, b, x, y, mask, mode, red, s);
    default: return hipErrorInvalidValue;
  }
}

template <int B, class X, class T>
hipError_t sweep_t(const SellDev& A, const void* S, const void* b, const void* x, void* xo, double omega,
                   hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  const X* SS = static_cast<const X*>(S);
  const X* bb = static_cast<const X*>(b);
  const X* xx = static_cast<const X*>(x);
  X* oo = static_cast<X*>(xo);
  switch (A.kind) {
    case VK_F64: hipLaunchKernelGGL((k_sweep<B, VK_F64, X, T>), g, kThreads, 0, s, A, SS, bb, xx, oo, T(omega)); break;
    case VK_F32: hipLaunchKernelGGL((k_sweep<B, VK_F32, X, T>), g, kThreads, 0, s, A, SS, bb, xx, oo, T(omega)); break;
    case VK_F16: hipLaunchKernelGGL((k_sweep<B, VK_F16, X, T>), g, kThreads, 0, s, A, SS, bb, xx, oo, T(omega)); break;
    case VK_BF16: hipLaunchKernelGGL((k_sweep<B, VK_BF16, X, T>), g, kThreads, 0, s, A, SS, bb, xx, oo, T(omega)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int B, class X, class T, class W>
hipError_t transfer_t(bool restrict_op, const CsrDev& M, const void* in, void* out, const uint8_t* m1,
                      const uint8_t* m2, hipStream_t s) {
  const int64_t n = int64_t(M.nrows) * B;
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, kThreads);
  const W* w = static_cast<const W*>(M.val);
  if (restrict_op)
    hipLaunchKernelGGL((k_restrict<B, X, T, W>), g, kThreads, 0, s, M.nrows, M.rowptr, M.col, w,
                       static_cast<const X*>(in), static_cast<X*>(out), m1, m2);
  else
    hipLaunchKernelGGL((k_prolong<B, X, T, W>), g, kThreads, 0, s, M.nrows, M.rowptr, M.col, w,
                       static_cast<const X*>(in), static_cast<X*>(out), m1, m2);
  return hipGetLastError();
}

template <int B>
hipError_t transfer_b(bool restrict_op, const CsrDev& M, const void* in, void* out, const uint8_t* m1,
                      const uint8_t* m2, int xk, hipStream_t s) {
  if (xk == X_F64)
    return M.f32 ? transfer_t<B, double, double, float>(restrict_op, M, in, out, m1, m2, s)
                 : transfer_t<B, double, double, double>(restrict_op, M, in, out, m1, m2, s);
  return M.f32 ? transfer_t<B, float, float, float>(restrict_op, M, in, out, m1, m2, s)
               : transfer_t<B, float, float, double>(restrict_op, M, in, out, m1, m2, s);
}

#define MGQ1_DISPATCH_B(B, CALL)                       \
  switch (B) {                                         \
    case 1: return CALL<1>;                            \
    case 2: return CALL<2>;                            \
    case 3: return CALL<3>;                            \
    case 4: return CALL<4>;                            \
    default: return hipErrorInvalidValue;              \
  }

}  // namespace

hipError_t launch_spmv(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask, int xk,
                       int yk, int mode, const RedDev* red, hipStream_t s) {
  switch (A.B) {
    case 1: return spmv_b<1>(A, b, x, y, mask, xk, yk, mode, red, s);
    case 2: return spmv_b<2>(A, b, x, y, mask, xk, yk, mode, red, s);
    case 3: return spmv_b<3>(A, b, x, y, mask, xk, yk, mode, red, s);
    case 4: return spmv_b<4>(A, b, x, y, mask, xk, yk, mode, red, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep(const SellDev& A, const void* S, const void* b, const void* x, void* xo, double omega,
                        int xk, hipStream_t s) {
  if (xk == X_F64) {
    switch (A.B) {
      case 1: return sweep_t<1, double, double>(A, S, b, x, xo, omega, s);
      case 2: return sweep_t<2, double, double>(A, S, b, x, xo, omega, s);
      case 3: return sweep_t<3, double, double>(A, S, b, x, xo, omega, s);
      case 4: return sweep_t<4, double, double>(A, S, b, x, xo, omega, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (A.B) {
    case 1: return sweep_t<1, float, float>(A, S, b, x, xo, omega, s);
    case 2: return sweep_t<2, float, float>(A, S, b, x, xo, omega, s);
    case 3: return sweep_t<3, float, float>(A, S, b, x, xo, omega, s);
    case 4: return sweep_t<4, float, float>(A, S, b, x, xo, omega, s);
    default: return hipErrorInvalidValue;
  }
}

template <int B>
static hipError_t sweep0_b(const SellDev& A, const void* S, const void* b, void* xo, double omega, int xk,
                           hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  if (xk == X_F64)
    hipLaunchKernelGGL((k_sweep0<B, double, double>), g, kThreads, 0, s, A.n, A.nslices,
                       static_cast<const double*>(S), static_cast<const double*>(b), static_cast<double*>(xo), omega);
  else
    hipLaunchKernelGGL((k_sweep0<B, float, float>), g, kThreads, 0, s, A.n, A.nslices,
                       static_cast<const float*>(S), static_cast<const float*>(b), static_cast<float*>(xo),
                       float(omega));
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

hipError_t launch_restrict(const CsrDev& R, int B, const void* r, void* d, const uint8_t* mask_c,
                           const uint8_t* mask_f, int xk, hipStream_t s) {
  switch (B) {
    case 1: return transfer_b<1>(true, R, r, d, mask_c, mask_f, xk, s);
    case 2: return transfer_b<2>(true, R, r, d, mask_c, mask_f, xk, s);
    case 3: return transfer_b<3>(true, R, r, d, mask_c, mask_f, xk, s);
    case 4: return transfer_b<4>(true, R, r, d, mask_c, mask_f, xk, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prolong(const CsrDev& P, int B, const void* y, void* x, const uint8_t* mask_f,
                          const uint8_t* mask_c, int xk, hipStream_t s) {
  switch (B) {
    case 1: return transfer_b<1>(false, P, y, x, mask_f, mask_c, xk, s);
    case 2: return transfer_b<2>(false, P, y, x, mask_f, mask_c, xk, s);
    case 3: return transfer_b<3>(false, P, y, x, mask_f, mask_c, xk, s);
    case 4: return transfer_b<4>(false, P, y, x, mask_f, mask_c, xk, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarse_gemv(int n, const double* AinvT, const void* b, void* x, int xk, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, kThreads);
  if (xk == X_F64)
    hipLaunchKernelGGL((k_coarse_gemv<double, double>), g, kThreads, 0, s, n, AinvT,
                       static_cast<const double*>(b), static_cast<double*>(x));
  else
    hipLaunchKernelGGL((k_coarse_gemv<float, float>), g, kThreads, 0, s, n, AinvT,
                       static_cast<const float*>(b), static_cast<float*>(x));
  return hipGetLastError();
}

hipError_t launch_coarse_invert(int n, double* M, double* AinvT, double* pivbuf, int* flag, hipStream_t s) {
  const int64_t tot = int64_t(n) * 2 * n;
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, 1, 1024, 0, s, n, k, M, pivbuf, flag);
    hipLaunchKernelGGL(k_gj_elim, grid_for(tot, 256), 256, 0, s, n, k, M, pivbuf, flag);
    hipLaunchKernelGGL(k_gj_clear, grid_for(n, 256), 256, 0, s, n, k, M);
  }
  hipLaunchKernelGGL(k_gj_extract, grid_for(int64_t(n) * n, 256), 256, 0, s, n, M, AinvT);
  return hipGetLastError();
}

hipError_t launch_block_invert(const SellDev& A, void* S, int sk, int* flag, hipStream_t s) {
  const unsigned g = grid_for(A.n, 256);
  if (g == 0) return hipSuccess;
#define MGQ1_BI(BB)                                                                                          \
  if (sk == X_F64) hipLaunchKernelGGL((k_block_invert<BB, double>), g, 256, 0, s, A, static_cast<double*>(S), flag); \
  else hipLaunchKernelGGL((k_block_invert<BB, float>), g, 256, 0, s, A, static_cast<float*>(S), flag);
  switch (A.B) {
    case 1: MGQ1_BI(1) break;
    case 2: MGQ1_BI(2) break;
    case 3: MGQ1_BI(3) break;
    case 4: MGQ1_BI(4) break;
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

hipError_t launch_scale_div(int64_t n, double* y, const double* x, const double* denom, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_div, grid_for(n, 256), 256, 0, s, n, y, x, denom);
  return hipGetLastError();
}

static unsigned red_grid(int64_t n) {
  unsigned g = grid_for(n, kRedThreads);
  if (g > unsigned(kMaxRedBlocks)) g = kMaxRedBlocks;
  return g ? g : 1;
}

hipError_t launch_dot(int64_t n, const double* a, const double* b, const RedDev& red, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, red_grid(n), kRedThreads, 0, s, n, a, b, red);
  return hipGetLastError();
}

hipError_t launch_nrm2(int64_t n, const double* a, const RedDev& red, hipStream_t s) {
  RedDev r = red;
  r.sqrt_out = 1;
  hipLaunchKernelGGL(k_dot, red_grid(n), kRedThreads, 0, s, n, a, static_cast<const double*>(nullptr), r);
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

hipError_t launch_givens(int j, int m, double* H, double* cs, double* sn, double* g, double* st, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, 1, 64, 0, s, j, m, H, cs, sn, g, st);
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
