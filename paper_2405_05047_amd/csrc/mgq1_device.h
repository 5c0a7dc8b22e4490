// Device-side building blocks shared by the HIP translation units of the multigrid
// library (internal linkage: each unit keeps its own copies): value decoding, the slot
// batches of the sliced-ELL operators, the per-slice row bodies, the sliced transfers,
// deterministic block reductions and launch-size helpers.
#pragma once

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
// FP64 blocks from the level's dictionary (loaded in sell_batch, not through load())
template <> struct Val<VK_DICT> {
  using raw = double;
  __device__ __forceinline__ static double dec(raw u) { return u; }
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
  if constexpr (K == VK_DICT) {
    // the dictionary form: column and block index first, then the block's row from the
    // (cached) dictionary together with the x gathers
    static_assert(NR == 1, "the dictionary form has one right-hand side");
    unsigned short di[NB];
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) js[qq] = slot_col<C16, NT>(A, k + qq, int64_t(k + qq) * R + r);
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) di[qq] = stream_load<NT>(A.didx + int64_t(k + qq) * R + r);
    __builtin_amdgcn_sched_barrier(0);
    const int c = rl % B;
    if (A.dlds) {
      extern __shared__ double dict_lds[];
#pragma unroll
      for (int qq = 0; qq < NB; ++qq)
#pragma unroll
        for (int cc = 0; cc < B; ++cc) av[qq][cc] = dict_lds[(int(di[qq]) * B + c) * B + cc];
    } else {
#pragma unroll
      for (int qq = 0; qq < NB; ++qq)
#pragma unroll
        for (int cc = 0; cc < B; ++cc) av[qq][cc] = A.dtab[(int64_t(di[qq]) * B + c) * B + cc];
    }
  } else {
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) js[qq] = slot_col<C16, NT>(A, k + qq, int64_t(k + qq) * R + r);
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) {
      const int64_t vb = int64_t(k + qq) * B * W + rl;
#pragma unroll
      for (int cc = 0; cc < B; ++cc) av[qq][cc] = Val<K>::template load<NT>(A.val, vb + cc * W);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
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

// dictionary form with dlds set: the workgroup copies the dictionary into LDS before any
// slice work (all threads reach the barrier); launched with ndict * B * B doubles of
// dynamic shared memory
template <int K>
__device__ __forceinline__ void dict_stage(const SellDev& A) {
  if constexpr (K == VK_DICT) {
    if (A.dlds) {
      extern __shared__ double dict_lds[];
      const int n = A.ndict * A.B * A.B;
      for (int i = int(threadIdx.x); i < n; i += int(blockDim.x)) dict_lds[i] = A.dtab[i];
      __syncthreads();
    }
  }
}

template <int K>
inline size_t dict_lds_bytes(const SellDev& A) {
  return (K == VK_DICT && A.dlds) ? size_t(A.ndict) * A.B * A.B * sizeof(double) : 0;
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
// LK: load kind of the operator stream — 0 as the operator says (A.nt), 1 always
// non-temporal (batched form), 2 always ordinary (single-workgroup tail)
template <int B, int NR, int K, class XI, class T, int KB = kb_default<B>(), bool C16 = false, int LK = 0>
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
  if (LK == 1 || (LK == 0 && A.nt)) {
    if constexpr (LK != 2) {
      if (wide) sell_loop<KB, B, NR, K, XI, T, false, true>(k, k1, A, r, node, rl, q, x, acc);
      else sell_loop<KB, B, NR, K, XI, T, C16, true>(k, k1, A, r, node, rl, q, x, acc);
    }
  } else {
    if constexpr (LK != 1) {
      if (wide) sell_loop<KB, B, NR, K, XI, T, false, false>(k, k1, A, r, node, rl, q, x, acc);
      else sell_loop<KB, B, NR, K, XI, T, C16, false>(k, k1, A, r, node, rl, q, x, acc);
    }
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
template <int B, int NR, int K, class XI, class XO, class T, int MODE, int KB = kb_default<B>(), bool C16 = false,
          int LK = 0>
__device__ __forceinline__ T spmv_slice(const SellDev& A, const XO* __restrict__ b, const XI* __restrict__ x,
                                        XO* __restrict__ y, const uint8_t* __restrict__ mask, const SliceLane& s) {
  XO bv = XO(0);
  uint8_t mk = 0;
  if (MODE != 0 && s.valid) {              // loaded before the row sum (latency overlap)
    bv = b[s.dof];
    if (MODE == 2) mk = mask[s.dof / NR];
  }
  const T acc = sell_dot<B, NR, K, XI, T, KB, C16, LK>(A, s.slice, s.lane, s.valid, x);
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

// x_out = x + omega S (b - A x), and with pmode != 0 the three-term (Chebyshev) form
// x_out = x + omega S (b - A x) + beta (x - x_prev): pmode 1 reads x_prev from x_out
// itself (each lane reads its own entry before it overwrites it), pmode 2 takes x_prev = 0
template <int B, int NR, int K, class X, class T, int KB = kb_default<B>(), bool C16 = false, int LK = 0>
__device__ __forceinline__ void sweep_slice(const SellDev& A, const X* __restrict__ S, const X* __restrict__ b,
                                            const X* __restrict__ x, X* __restrict__ xo, T omega,
                                            const SliceLane& s, T beta = T(0), int pmode = 0) {
  constexpr int W = kWave / NR;
  const int rl = s.lane / NR, q = s.lane % NR;
  // the lane's own b, x and smoother row are loaded before the row sum, so their latency
  // overlaps the slot batches
  X bv = X(0), xv = X(0), pv = X(0), sv[B];
#pragma unroll
  for (int cc = 0; cc < B; ++cc) sv[cc] = X(0);
  if (s.valid) {
    bv = b[s.dof];
    xv = x[s.dof];
    // unconditional load (a load inside a branch would make the slot loop wait for it);
    // with pmode != 1 it rereads x and the value is not used
    pv = (pmode == 1 ? static_cast<const X*>(xo) : x)[s.dof];
#pragma unroll
    for (int cc = 0; cc < B; ++cc) sv[cc] = S[(int64_t(s.slice) * B + cc) * W + rl];
  }
  const T acc = sell_dot<B, NR, K, X, T, KB, C16, LK>(A, s.slice, s.lane, s.valid, x);
  const T res = s.valid ? T(bv) - acc : T(0);
  const int base = (rl / B) * B;
  T upd = T(0);
#pragma unroll
  for (int cc = 0; cc < B; ++cc) {
    const T rc = __shfl(res, ((base + cc) * NR + q) & (kWave - 1), kWave);
    if (s.valid) upd += T(sv[cc]) * rc;
  }
  if (s.valid) {
    T nx = T(xv) + omega * upd;
    if (pmode != 0) nx = nx + beta * (T(xv) - (pmode == 1 ? T(pv) : T(0)));
    xo[s.dof] = X(nx);
  }
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

// ---- node form of the sliced transfers: one lane per node computes its B components.  Per
// slot one packed 32-bit entry (16-bit column offset, 8-bit weight code w * 128, the column
// DoFs' mask bits) and B gathers of the column node's vector; the FMAs run in slot order
// with the same operands as the per-DoF form, so the sums are the same bit for bit.  A
// wave issues one entry load per slot for 64 nodes where the per-DoF form issues an index,
// a weight and a mask load per slot for 64 / B nodes.
template <int NB, int B, class X, class T, bool MC>
__device__ __forceinline__ void tnode_batch(const TSellDev& M, int k, int lane, const X* __restrict__ in,
                                            T (&acc)[B]) {
  uint32_t e[NB];
  int32_t base[NB];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    e[qq] = M.ent[int64_t(k + qq) * kWave + lane];
    base[qq] = M.colbase[k + qq];
  }
  __builtin_amdgcn_sched_barrier(0);
  X v[NB][B];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    const uint64_t j = uint64_t(uint32_t(base[qq]) + (e[qq] & 0xffffu));
#pragma unroll
    for (int c = 0; c < B; ++c) v[qq][c] = in[j * B + c];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    const T w = T(float((e[qq] >> 16) & 0xffu) * 0.0078125f);
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const bool ms = MC && ((e[qq] >> (24 + c)) & 1u);
      acc[c] += w * (ms ? T(0) : T(v[qq][c]));
    }
  }
}

template <int N, int B, class X, class T, bool MC>
__device__ __forceinline__ void tnode_rest(int rem, const TSellDev& M, int k, int lane, const X* __restrict__ in,
                                           T (&acc)[B]) {
  if constexpr (N >= 1) {
    if (rem == N) tnode_batch<N, B, X, T, MC>(M, k, lane, in, acc);
    else tnode_rest<N - 1, B, X, T, MC>(rem, M, k, lane, in, acc);
  }
}

// MODE 0: out = restriction sum (zero on masked row DoFs); MODE 1: out += prolongation sum
// (masked row DoFs left unchanged)
template <int B, class X, class T, bool MC, int MODE>
__device__ __forceinline__ void tnode_lane(const TSellDev& M, int slice, int lane, const X* __restrict__ in,
                                           X* __restrict__ out) {
  // slot batch: restriction rows hold up to 3^d entries (27 on 3D box meshes), prolongation
  // rows at most 2^d; a batch is one dependent round trip (entries, then gathers)
  constexpr int KB = MODE == 0 ? 8 : 4;
  const int node = slice * kWave + lane;
  if (slice >= M.nslices || node >= M.nrows) return;
  const int64_t d0 = int64_t(node) * B;
  const uint8_t rm = M.rmask[node];
  X old[B];
  if (MODE == 1) {
#pragma unroll
    for (int c = 0; c < B; ++c) old[c] = out[d0 + c];
  }
  const int su = __builtin_amdgcn_readfirstlane(slice);
  int k, k1;
  slot_range(M, su, k, k1);
  T acc[B];
#pragma unroll
  for (int c = 0; c < B; ++c) acc[c] = T(0);
  for (; k + KB <= k1; k += KB) tnode_batch<KB, B, X, T, MC>(M, k, lane, in, acc);
  tnode_rest<KB - 1, B, X, T, MC>(k1 - k, M, k, lane, in, acc);
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const bool masked = (rm >> c) & 1u;
    if (MODE == 0) out[d0 + c] = masked ? X(0) : X(acc[c]);
    else if (!masked) out[d0 + c] = X(T(old[c]) + acc[c]);
  }
}

template <int B, class X, class T, bool MC, int MODE>
__global__ __launch_bounds__(kThreads) void k_tnode(TSellDev M, const X* __restrict__ in, X* __restrict__ out) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  tnode_lane<B, X, T, MC, MODE>(M, bid * kSliceWaves + threadIdx.x / kWave, threadIdx.x % kWave, in, out);
}

inline unsigned grid_for(int64_t n, int threads) { return unsigned((n + threads - 1) / threads); }
inline unsigned slice_grid(int nslices) { return unsigned((nslices + kSliceWaves - 1) / kSliceWaves); }

}  // namespace
}  // namespace mgq1
