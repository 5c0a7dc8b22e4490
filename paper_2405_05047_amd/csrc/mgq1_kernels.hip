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
//   Batched form: the same slice bodies over the entries of many problems per launch
//   (each block finds its entry by binary search over the entries' first blocks), and
//   segmented Krylov kernels (each block belongs to one problem's vector segment).
//
// Paper correspondence: smoother x + omega S (b - A x), transfers P and R = P^T and the
// coarse solve (Sec. 4.1 "Geometric Multigrid CUDA", Algorithm "Geometric multigrid
// solver"); GMRES building blocks with modified Gram-Schmidt (Sec. 4.2).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "mgq1_internal.h"

namespace mgq1 {
namespace {

constexpr int kThreads = kWave * kSliceWaves;   // 256
constexpr int kTailThreads = 1024;
constexpr int kMaxWaves = 16;

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  // hardware dispatch sends workgroup w to XCD w % 8; give XCD x a contiguous range
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Loads of the operator streams (values, column indices, transfer weights): non-temporal
// (NT) on levels too large to stay in the memory-side cache between kernels, where they
// would only evict the gathered vectors; ordinary loads on the smaller levels, whose
// operators the next kernels read again from that cache.
template <bool NT, class P>
__device__ __forceinline__ P stream_load(const P* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// stored matrix values: load() fetches the raw stored word, dec() widens it to FP32/FP64.  FP16/BF16 values are a_ij / s_i with the
// power-of-two row scale s_i applied once to the finished row sum (exact: scaling by 2^e
// commutes with rounding away from overflow and underflow).
template <int K> struct Val;
template <> struct Val<VK_F64> {
  using raw = double;
  template <bool NT>
  __device__ __forceinline__ static raw load(const void* p, int64_t i) {
    return stream_load<NT>(static_cast<const double*>(p) + i);
  }
  __device__ __forceinline__ static double dec(raw u) { return u; }
};
template <> struct Val<VK_F32> {
  using raw = float;
  template <bool NT>
  __device__ __forceinline__ static raw load(const void* p, int64_t i) {
    return stream_load<NT>(static_cast<const float*>(p) + i);
  }
  __device__ __forceinline__ static float dec(raw u) { return u; }
};
template <> struct Val<VK_F16> {
  using raw = unsigned short;
  template <bool NT>
  __device__ __forceinline__ static raw load(const void* p, int64_t i) {
    return stream_load<NT>(static_cast<const unsigned short*>(p) + i);
  }
  __device__ __forceinline__ static float dec(raw u) { return __half2float(__ushort_as_half(u)); }
};
template <> struct Val<VK_BF16> {
  using raw = unsigned short;
  template <bool NT>
  __device__ __forceinline__ static raw load(const void* p, int64_t i) {
    return stream_load<NT>(static_cast<const unsigned short*>(p) + i);
  }
  __device__ __forceinline__ static float dec(raw u) { return __uint_as_float(static_cast<uint32_t>(u) << 16); }
};

// NB block slots k .. k+NB-1 of a slice: the column indices first, then every value and
// x load of the batch, then the FMAs, so the batch costs two memory round trips.  NB is a
// compile-time constant, so no load sits in a conditional block (a conditional load whose
// result is widened inside the block would force a wait per slot).
// C16: column indices are stored as 16-bit offsets from a per-slot base (the smallest
// column of that slot in the slice, wave-uniform, so a scalar load).
template <bool C16, bool NT>
__device__ __forceinline__ unsigned slot_col(const SellDev& A, int k, int64_t idx) {
  if constexpr (C16) return unsigned(A.colbase[k]) + unsigned(stream_load<NT>(A.col16 + idx));
  else return unsigned(stream_load<NT>(A.col + idx));
}

// slot range [k, k1) of slice su (wave-uniform): computed for uniform-width slices, else
// read from the slice pointers (one dependent round trip before the first slot load)
template <class M>
__device__ __forceinline__ void slot_range(const M& A, int su, int& k, int& k1) {
  if (A.ell > 0) {
    k = su * A.ell;
    k1 = k + A.ell;
  } else {
    k = A.sptr[su];
    k1 = A.sptr[su + 1];
  }
}

// slice su (wave-uniform) of a 16-bit-column operator reads the 32-bit columns instead
__device__ __forceinline__ bool is_wide(const SellDev& A, int su) {
  return A.wide != nullptr && ((A.wide[su >> 5] >> (su & 31)) & 1u);
}

template <int NB, int B, int NR, int K, class XI, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_batch(const SellDev& A, int k, int r, int node, int rl, int q,
                                           const XI* __restrict__ x, T& acc) {
  constexpr int R = kWave / (B * NR);
  constexpr int W = kWave / NR;
  using VR = typename Val<K>::raw;
  // phase 1: column indices and values (independent of each other); phase 2: the x
  // gathers; phase 3: the FMAs.  Scheduling barriers keep the phases apart, otherwise the
  // scheduler interleaves the FMA chain with the loads and adds round trips.
  unsigned js[NB];                         // unsigned: widening needs no sign extension
  VR av[NB][B];
  XI xv[NB][B];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) js[qq] = slot_col<C16, NT>(A, k + qq, int64_t(k + qq) * R + r);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    const int64_t vb = int64_t(k + qq) * B * W + rl;
#pragma unroll
    for (int cc = 0; cc < B; ++cc) av[qq][cc] = Val<K>::template load<NT>(A.val, vb + cc * W);
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (B > 1 && NR == 1) {
    // each lane gathers only its own component of the neighbour node (the B lanes of a
    // node read one contiguous B-vector together) and takes the others from its node's
    // lanes by wave shuffles
    const int c = rl % B, base = rl - c;
    XI xo[NB];
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) xo[qq] = x[uint64_t(js[qq]) * B + c];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int qq = 0; qq < NB; ++qq)
#pragma unroll
      for (int cc = 0; cc < B; ++cc) xv[qq][cc] = __shfl(xo[qq], base + cc, kWave);
  } else {
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) {
      const XI* xj = x + uint64_t(js[qq]) * (B * NR) + q;
#pragma unroll
      for (int cc = 0; cc < B; ++cc) xv[qq][cc] = xj[cc * NR];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq)
#pragma unroll
    for (int cc = 0; cc < B; ++cc) acc += T(Val<K>::dec(av[qq][cc])) * T(xv[qq][cc]);
}

// The same batch for the second of two sweeps from x = 0 with b = 1: the iterate after the
// first sweep, x1_j = omega * (S_j * b_j), is formed on the fly from S and b instead of being
// read (S of node j sits at S[j] for one component and one right-hand side), with the
// rounding of the stored value, so the result is bitwise that of the two separate sweeps.
template <int NB, int K, class X, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_batch_z(const SellDev& A, int k, int rl, int node, const X* __restrict__ S,
                                             const X* __restrict__ b, T omega, T& acc) {
  using VR = typename Val<K>::raw;
  unsigned js[NB];
  VR av[NB];
  X sv[NB], bv[NB];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) js[qq] = slot_col<C16, NT>(A, k + qq, int64_t(k + qq) * kWave + rl);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) av[qq] = Val<K>::template load<NT>(A.val, int64_t(k + qq) * kWave + rl);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    sv[qq] = S[js[qq]];
    bv[qq] = b[js[qq]];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    const X x1 = X(omega * (T(0) + T(sv[qq]) * T(bv[qq])));
    acc += T(Val<K>::dec(av[qq])) * T(x1);
  }
}

template <int N, int K, class X, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_rest_z(int rem, const SellDev& A, int k, int rl, int node,
                                            const X* __restrict__ S, const X* __restrict__ b, T omega, T& acc) {
  if constexpr (N >= 1) {
    if (rem == N) sell_batch_z<N, K, X, T, C16, NT>(A, k, rl, node, S, b, omega, acc);
    else sell_rest_z<N - 1, K, X, T, C16, NT>(rem, A, k, rl, node, S, b, omega, acc);
  }
}

// the slots [k, k1) of one slice for the second of two sweeps from 0
template <int KB, int K, class X, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_loop_z(int k, int k1, const SellDev& A, int rl, int node,
                                            const X* __restrict__ S, const X* __restrict__ b, T omega, T& acc) {
  for (; k + KB <= k1; k += KB) sell_batch_z<KB, K, X, T, C16, NT>(A, k, rl, node, S, b, omega, acc);
  sell_rest_z<KB - 1, K, X, T, C16, NT>(k1 - k, A, k, rl, node, S, b, omega, acc);
}

// the remaining rem < KB slots of a slice as one batch of exactly rem slots
template <int N, int B, int NR, int K, class XI, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_rest(int rem, const SellDev& A, int k, int r, int node, int rl, int q,
                                          const XI* __restrict__ x, T& acc) {
  if constexpr (N >= 1) {
    if (rem == N) sell_batch<N, B, NR, K, XI, T, C16, NT>(A, k, r, node, rl, q, x, acc);
    else sell_rest<N - 1, B, NR, K, XI, T, C16, NT>(rem, A, k, r, node, rl, q, x, acc);
  }
}

// the slots [k, k1) of one slice: batches of KB, then the remainder as one batch
template <int KB, int B, int NR, int K, class XI, class T, bool C16, bool NT>
__device__ __forceinline__ void sell_loop(int k, int k1, const SellDev& A, int r, int node, int rl, int q,
                                          const XI* __restrict__ x, T& acc) {
  for (; k + KB <= k1; k += KB) sell_batch<KB, B, NR, K, XI, T, C16, NT>(A, k, r, node, rl, q, x, acc);
  sell_rest<KB - 1, B, NR, K, XI, T, C16, NT>(k1 - k, A, k, r, node, rl, q, x, acc);
}

template <int B> constexpr int kb_default() { return B <= 2 ? 8 : 4; }
template <int B> constexpr int kb_alt() { return B <= 2 ? 16 : 8; }

// per-lane row dot product of a slice: sum_k sum_cc a(k, cc) x[(col_k * B + cc) * NR + q].
// NR right-hand sides share every matrix entry: lane = (r * B + c) * NR + q, the slice
// holds R = 64 / (B * NR) nodes, and the values of row lane rl = lane / NR sit at
// val[(k * B + cc) * W + rl] with the padded row-lane stride W = 64 / NR (R * B rounded up,
// 64 for one right-hand side).  NR = 1 is the single right-hand-side layout.  Slots are
// consumed in batches of KB, the remainder in one shorter batch (slice-uniform branch);
// the FMAs run in slot order whatever KB is, so every KB gives the same bits.
template <int B, int NR, int K, class XI, class T, int KB = kb_default<B>(), bool C16 = false>
__device__ __forceinline__ T sell_dot(const SellDev& A, int slice, int lane, bool valid,
                                      const XI* __restrict__ x) {
  constexpr int W = kWave / NR;
  constexpr int R = kWave / (B * NR);
  T acc = T(0);
  if (!valid) return acc;
  const int rl = lane / NR, q = lane % NR;
  const int r = rl / B;
  // the slice is the same for the whole wave: keep it (and the slot range, the load bases)
  // in scalar registers
  slice = __builtin_amdgcn_readfirstlane(slice);
  const int node = slice * R + r;
  int k, k1;
  slot_range(A, slice, k, k1);
  const bool wide = C16 && is_wide(A, slice);
  if (A.nt) {
    if (wide) sell_loop<KB, B, NR, K, XI, T, false, true>(k, k1, A, r, node, rl, q, x, acc);
    else sell_loop<KB, B, NR, K, XI, T, C16, true>(k, k1, A, r, node, rl, q, x, acc);
  } else {
    if (wide) sell_loop<KB, B, NR, K, XI, T, false, false>(k, k1, A, r, node, rl, q, x, acc);
    else sell_loop<KB, B, NR, K, XI, T, C16, false>(k, k1, A, r, node, rl, q, x, acc);
  }
  if (K == VK_F16 || K == VK_BF16) acc *= T(ldexpf(1.0f, A.rexp[int64_t(slice) * W + rl]));
  return acc;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}

// sum over the block in a fixed order, returned to every thread
__device__ __forceinline__ double block_allsum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (ln == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += lds[q];
    lds[kMaxWaves] = t;
  }
  __syncthreads();
  const double r = lds[kMaxWaves];
  __syncthreads();
  return r;
}

// sum of partials[0..g) in a fixed order (every block computes the same value)
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int g, double* lds) {
  constexpr int U = 8;                     // loads issued together, summed in index order
  double t = 0.0;
  for (int q0 = threadIdx.x; q0 < g; q0 += blockDim.x * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * int(blockDim.x);
      v[u] = q < g ? p[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
  }
  return block_allsum(t, lds);
}

// ------------------------------------------------------------------ per-slice bodies
// geometry of one wave-slice
struct SliceLane {
  int slice, lane, node;
  int64_t dof;            // (node * B + c) * NR + q
  bool valid;
};

template <int B, int NR>
__device__ __forceinline__ SliceLane slice_lane(const SellDev& A, int slice, int lane) {
  constexpr int R = kWave / (B * NR);
  SliceLane s;
  s.slice = slice;
  s.lane = lane;
  const int pos = slice * R + lane / (B * NR);   // row position of the lane's node
  s.valid = slice < A.nslices && lane < R * B * NR && pos < A.n;
  s.node = (A.perm != nullptr && s.valid) ? A.perm[pos] : pos;
  s.dof = int64_t(s.node) * B * NR + lane % (B * NR);
  return s;
}

// y = A x (MODE 0), b - A x (MODE 1), M (b - A x) (MODE 2); returns the written value
template <int B, int NR, int K, class XI, class XO, class T, int MODE, int KB = kb_default<B>(), bool C16 = false>
__device__ __forceinline__ T spmv_slice(const SellDev& A, const XO* __restrict__ b, const XI* __restrict__ x,
                                        XO* __restrict__ y, const uint8_t* __restrict__ mask, const SliceLane& s) {
  XO bv = XO(0);
  uint8_t mk = 0;
  if (MODE != 0 && s.valid) {              // loaded before the row sum (latency overlap)
    bv = b[s.dof];
    if (MODE == 2) mk = mask[s.dof / NR];
  }
  const T acc = sell_dot<B, NR, K, XI, T, KB, C16>(A, s.slice, s.lane, s.valid, x);
  T out = T(0);
  if (s.valid) {
    if (MODE == 0) {
      out = acc;
    } else {
      out = T(bv) - acc;
      if (MODE == 2 && mk) out = T(0);
    }
    y[s.dof] = XO(out);
  }
  return out;
}

template <int B, int NR, int K, class X, class T, int KB = kb_default<B>(), bool C16 = false>
__device__ __forceinline__ void sweep_slice(const SellDev& A, const X* __restrict__ S, const X* __restrict__ b,
                                            const X* __restrict__ x, X* __restrict__ xo, T omega,
                                            const SliceLane& s) {
  constexpr int W = kWave / NR;
  const int rl = s.lane / NR, q = s.lane % NR;
  // the lane's own b, x and smoother row are loaded before the row sum, so their latency
  // overlaps the slot batches
  X bv = X(0), xv = X(0), sv[B];
#pragma unroll
  for (int cc = 0; cc < B; ++cc) sv[cc] = X(0);
  if (s.valid) {
    bv = b[s.dof];
    xv = x[s.dof];
#pragma unroll
    for (int cc = 0; cc < B; ++cc) sv[cc] = S[(int64_t(s.slice) * B + cc) * W + rl];
  }
  const T acc = sell_dot<B, NR, K, X, T, KB, C16>(A, s.slice, s.lane, s.valid, x);
  const T res = s.valid ? T(bv) - acc : T(0);
  const int base = (rl / B) * B;
  T upd = T(0);
#pragma unroll
  for (int cc = 0; cc < B; ++cc) {
    const T rc = __shfl(res, ((base + cc) * NR + q) & (kWave - 1), kWave);
    if (s.valid) upd += T(sv[cc]) * rc;
  }
  if (s.valid) xo[s.dof] = X(T(xv) + omega * upd);
}

template <int B, int NR, class X, class T>
__device__ __forceinline__ void sweep0_slice(const X* __restrict__ S, const X* __restrict__ b, X* __restrict__ xo,
                                             T omega, const SliceLane& s) {
  constexpr int W = kWave / NR;
  if (!s.valid) return;
  const int rl = s.lane / NR, q = s.lane % NR;
  T upd = T(0);
#pragma unroll
  for (int cc = 0; cc < B; ++cc)
    upd += T(S[(int64_t(s.slice) * B + cc) * W + rl]) * T(b[(int64_t(s.node) * B + cc) * NR + q]);
  xo[s.dof] = X(omega * upd);
}

__device__ __forceinline__ double weight(const CsrDev& M, int k) {
  return M.f32 ? double(static_cast<const float*>(M.val)[k]) : static_cast<const double*>(M.val)[k];
}

// d[t] = M_c sum_k R_jk (M_f r)[k], t = (j*B + c) * NR + q
template <int B, int NR, class X, class T>
__device__ __forceinline__ void restrict_dof(const CsrDev& R, const X* __restrict__ r, X* __restrict__ d,
                                             const uint8_t* __restrict__ mask_c, const uint8_t* __restrict__ mask_f,
                                             int64_t t) {
  const int64_t dof = t / NR;
  const int q = int(t % NR);
  const int j = int(dof / B), c = int(dof % B);
  T acc = T(0);
  if (!mask_c[dof]) {
    for (int k = R.rowptr[j]; k < R.rowptr[j + 1]; ++k) {
      const int64_t fd = int64_t(R.col[k]) * B + c;
      if (mask_f == nullptr || !mask_f[fd]) acc += T(weight(R, k)) * T(r[fd * NR + q]);
    }
  }
  d[t] = X(acc);
}

// x[t] += M_f sum_k P_ik (M_c y)[k]
template <int B, int NR, class X, class T>
__device__ __forceinline__ void prolong_dof(const CsrDev& P, const X* __restrict__ y, X* __restrict__ x,
                                            const uint8_t* __restrict__ mask_f, const uint8_t* __restrict__ mask_c,
                                            int64_t t) {
  const int64_t dof = t / NR;
  const int q = int(t % NR);
  if (mask_f[dof]) return;
  const int i = int(dof / B), c = int(dof % B);
  T acc = T(0);
  for (int k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k) {
    const int64_t cd = int64_t(P.col[k]) * B + c;
    if (!mask_c[cd]) acc += T(weight(P, k)) * T(y[cd * NR + q]);
  }
  x[t] = X(T(x[t]) + acc);
}

// ---- sliced transfers: NB slots of one node row, loads first (straight-line), then the
// weighted sum in slot order.  MC: apply the column mask (entries whose column DoF is
// masked contribute 0).
template <int NB, int B, int NR, class X, class T, class WT, bool MC, bool NT>
__device__ __forceinline__ void tsell_batch(const TSellDev& M, int k, int r, int c, int q,
                                            const X* __restrict__ in, const uint8_t* __restrict__ mcol,
                                            T& acc) {
  const int R = M.R;
  unsigned js[NB];
  WT ws[NB];
  X vs[NB];
  uint8_t ms[NB];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    js[qq] = unsigned(stream_load<NT>(M.col + int64_t(k + qq) * R + r));
    ws[qq] = stream_load<NT>(static_cast<const WT*>(M.w) + int64_t(k + qq) * R + r);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    const uint64_t d = uint64_t(js[qq]) * B + c;
    vs[qq] = in[d * NR + q];
    ms[qq] = MC ? mcol[d] : uint8_t(0);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) acc += T(ws[qq]) * (ms[qq] ? T(0) : T(vs[qq]));
}

template <int N, int B, int NR, class X, class T, class WT, bool MC, bool NT>
__device__ __forceinline__ void tsell_rest(int rem, const TSellDev& M, int k, int r, int c, int q,
                                           const X* __restrict__ in, const uint8_t* __restrict__ mcol, T& acc) {
  if constexpr (N >= 1) {
    if (rem == N) tsell_batch<N, B, NR, X, T, WT, MC, NT>(M, k, r, c, q, in, mcol, acc);
    else tsell_rest<N - 1, B, NR, X, T, WT, MC, NT>(rem, M, k, r, c, q, in, mcol, acc);
  }
}

// one lane of a sliced transfer.  MODE 0: out = restriction sum (zero on masked rows);
// MODE 1: out += prolongation sum (rows whose DoF is masked are left unchanged)
template <int B, int NR, class X, class T, class WT, bool MC, int MODE>
__device__ __forceinline__ void tsell_lane(const TSellDev& M, int slice, int lane, const X* __restrict__ in,
                                           X* __restrict__ out, const uint8_t* __restrict__ mrow,
                                           const uint8_t* __restrict__ mcol) {
  constexpr int KB = 8;
  const int R = M.R;
  const int r = lane / (B * NR), c = (lane / NR) % B, q = lane % NR;
  const int node = slice * R + r;
  if (slice >= M.nslices || lane >= R * B * NR || node >= M.nrows) return;
  const int64_t dof = int64_t(node) * B + c;
  const int64_t t = dof * NR + q;
  // the row mask and (prolongation) the old value are loaded with the first slots; masked
  // rows run the sum too (their columns are valid indices) and drop it at the end, so no
  // branch waits for the mask before the slot loads are issued
  const uint8_t masked = mrow[dof];
  X old = X(0);
  if (MODE == 1) old = out[t];
  const int su = __builtin_amdgcn_readfirstlane(slice);
  int k, k1;
  slot_range(M, su, k, k1);
  T acc = T(0);
  if (M.nt) {
    for (; k + KB <= k1; k += KB) tsell_batch<KB, B, NR, X, T, WT, MC, true>(M, k, r, c, q, in, mcol, acc);
    tsell_rest<KB - 1, B, NR, X, T, WT, MC, true>(k1 - k, M, k, r, c, q, in, mcol, acc);
  } else {
    for (; k + KB <= k1; k += KB) tsell_batch<KB, B, NR, X, T, WT, MC, false>(M, k, r, c, q, in, mcol, acc);
    tsell_rest<KB - 1, B, NR, X, T, WT, MC, false>(k1 - k, M, k, r, c, q, in, mcol, acc);
  }
  if (MODE == 0) out[t] = masked ? X(0) : X(acc);
  else if (!masked) out[t] = X(T(old) + acc);
}

template <int B, int NR, class X, class T, class WT, bool MC, int MODE>
__global__ __launch_bounds__(kThreads) void k_tsell(TSellDev M, const X* __restrict__ in, X* __restrict__ out,
                                                    const uint8_t* __restrict__ mrow,
                                                    const uint8_t* __restrict__ mcol) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  tsell_lane<B, NR, X, T, WT, MC, MODE>(M, bid * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave, in, out,
                                        mrow, mcol);
}

// ------------------------------------------------------------------ grid kernels
// NORM: per-block partial sums of out * out, or of out * dotv[row] when dotv is given
template <int B, int K, class XI, class XO, class T, int MODE, bool NORM, int KB, bool C16>
__global__ __launch_bounds__(kThreads) void k_spmv(SellDev A, const XO* __restrict__ b, const XI* __restrict__ x,
                                                   XO* __restrict__ y, const uint8_t* __restrict__ mask,
                                                   double* __restrict__ partials, const double* __restrict__ dotv) {
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
                                                    const X* __restrict__ x, X* __restrict__ xo, T omega) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const SliceLane s = slice_lane<B, 1>(A, bid * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave);
  sweep_slice<B, 1, K, X, T, KB, C16>(A, S, b, x, xo, omega, s);
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
    sweep_slice<B, 1, K, X, T>(L.A, static_cast<const X*>(L.S), b, x, xo, omega, slice_lane<B, 1>(L.A, sl, ln));
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
      spmv_slice<B, 1, K, X, X, T, 2>(L.A, b, cur, static_cast<X*>(L.r), L.mask, slice_lane<B, 1>(L.A, sl, ln));
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
inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }
inline unsigned slice_grid(int nslices) { return unsigned((nslices + kSliceWaves - 1) / kSliceWaves); }

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
  hipLaunchKernelGGL((k_spmv<B, K, XI, XO, T, MODE, NORM, KB, C16>), g, kThreads, 0, s, A, bb, xx, yy, mask, partials, \
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
                   hipStream_t s) {
  const unsigned g = slice_grid(A.nslices);
  if (g == 0) return hipSuccess;
  const X* SS = static_cast<const X*>(S);
  const X* bb = static_cast<const X*>(b);
  const X* xx = static_cast<const X*>(x);
  X* oo = static_cast<X*>(xo);
#define MGQ1_SWEEP4(KIND, KB, C16) \
  hipLaunchKernelGGL((k_sweep<B, KIND, X, T, KB, C16>), g, kThreads, 0, s, A, SS, bb, xx, oo, T(omega))
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
    if (A.kind != VK_F64) return hipErrorInvalidValue;
    MGQ1_SWEEP(VK_F64);
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

hipError_t tsell_launch(int mode, const TSellDev& M, int B, const void* in, void* out, const uint8_t* mrow,
                        const uint8_t* mcol, int xk, hipStream_t s) {
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
    sweep_slice<B, NR, K, X, T, KB, C16>(e.A, static_cast<const X*>(e.S), static_cast<const X*>(e.in0),
                                    static_cast<const X*>(e.in1), static_cast<X*>(e.out), omega, s);
  else
    spmv_slice<B, NR, K, X, X, T, 2, KB, C16>(e.A, static_cast<const X*>(e.in0), static_cast<const X*>(e.in1),
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
      out = spmv_slice<B, NR, VK_F64, XI, double, double, 0, KB, C16>(e.A, nullptr, static_cast<const XI*>(e.in1),
                                                                 static_cast<double*>(e.out), nullptr, s);
    } else {
      out = spmv_slice<B, NR, VK_F64, double, double, double, 1, KB, C16>(e.A, static_cast<const double*>(e.in0),
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
