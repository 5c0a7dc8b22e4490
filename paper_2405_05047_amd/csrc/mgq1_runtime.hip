// Host runtime and C ABI of libmgq1: hierarchy setup on the device, the V-cycle driver
// (Algorithm "Geometric multigrid solver", Sec. 2.2), defect-correction and flexible
// GMRES outer loops (Sec. 4.2), and the step-wise entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mgq1.h"
#include "mgq1_internal.h"

#include <cstdio>

using namespace mgq1;

// Partial sums of the allocation-free outer defect (mg_outer_defect_noalloc): one FP64
// per workgroup of the finest-level FP64 SpMV.  Each GPU the library runs on holds its
// own copy of this array until the process ends; host code reaches it only through the
// per-device address taken with hipGetSymbolAddress at setup.
constexpr int kScratchDoubles = 1 << 16;   // 512 KiB: finest levels up to ~16.7M scalar rows
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define MG_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(MG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- host-side helpers
struct HostLevel {
  int32_t n = 0, B = 1;
  int64_t nnzb = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  int32_t pc = 0;
  std::vector<int32_t> prow, pcol;
  std::vector<double> pval;
  std::vector<uint8_t> mask;
  std::vector<double> sblk;         // caller's smoother blocks (empty: derived on the device)
};

// f(begin, end) over [0, n) in contiguous chunks of at least min_chunk iterations on up to
// 16 host threads (MGQ1_HOST_THREADS lowers the cap).  Used by the setup loops whose
// iterations write disjoint outputs, so the results do not depend on the thread count.
// f must not throw or allocate.
template <class F>
void parallel_for(int64_t n, int64_t min_chunk, const F& f) {
  int64_t T = std::min<int64_t>(16, std::max<int64_t>(1, int64_t(std::thread::hardware_concurrency())));
  if (const char* e = std::getenv("MGQ1_HOST_THREADS")) T = std::max<int64_t>(1, std::min<int64_t>(T, std::atoi(e)));
  T = std::min<int64_t>(T, (n + min_chunk - 1) / std::max<int64_t>(1, min_chunk));
  if (T <= 1) {
    if (n > 0) f(int64_t(0), n);
    return;
  }
  const int64_t step = (n + T - 1) / T;
  std::vector<std::thread> th;
  th.reserve(size_t(T));
  for (int64_t t = 1; t < T; ++t) {
    const int64_t a = t * step, b = std::min(n, a + step);
    if (a >= b) continue;
    try {
      th.emplace_back([&f, a, b] { f(a, b); });
    } catch (...) {
      f(a, b);                                      // no thread available: run it here
    }
  }
  f(int64_t(0), std::min(n, step));
  for (std::thread& x : th) x.join();
}

template <class T>
int fetch(std::vector<T>& dst, const T* src, size_t n, bool on_device) {
  if (n == 0) {
    dst.clear();
    return MG_OK;
  }
  if (!src) return fail(MG_EINVAL, "null input array");
  if (on_device) {
    dst.resize(n);
    MG_HIP(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
  } else {
    dst.assign(src, src + n);
  }
  return MG_OK;
}

int validate_host(const HostLevel& L, const HostLevel* C, int level) {
  const std::string at = "level " + std::to_string(level) + ": ";
  const int B = L.B;
  if (L.n <= 0) return fail(MG_EINVAL, at + "n_nodes must be positive");
  if (B < 1 || B > 8) return fail(MG_EINVAL, at + "block must be 1..8");
  if (int64_t(L.n) * B >= (int64_t(1) << 31)) return fail(MG_EINVAL, at + "too many DoFs for int32 indices");
  if (L.rowptr[0] != 0) return fail(MG_EINVAL, at + "rowptr[0] != 0");
  for (int32_t i = 0; i < L.n; ++i)
    if (L.rowptr[i + 1] < L.rowptr[i]) return fail(MG_EINVAL, at + "rowptr not monotone");
  if (L.rowptr[L.n] != L.nnzb) return fail(MG_EINVAL, at + "rowptr[n] != nnzb");
  // per-row checks in parallel chunks; the error reported is that of the first failing
  // row, as in a sequential pass
  static const char* const kRowError[] = {"", "column index out of range", "columns not sorted/unique",
                                          "non-finite matrix value",
                                          "constrained DoF row/column is not an identity row/column",
                                          "missing diagonal block"};
  auto row_error = [&](int32_t i) -> int {
    bool diag = false;
    for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1]; ++k) {
      const int32_t j = L.col[k];
      if (j < 0 || j >= L.n) return 1;
      if (k > L.rowptr[i] && L.col[k - 1] >= j) return 2;
      diag |= (j == i);
      for (int z = 0; z < B * B; ++z) {
        const double v = L.val[size_t(k) * B * B + z];
        if (!std::isfinite(v)) return 3;
        const int c = z / B, cc = z % B;
        const bool mr = L.mask[size_t(i) * B + c], mc = L.mask[size_t(j) * B + cc];
        if (mr || mc) {
          const double want = (i == j && c == cc && mr) ? 1.0 : 0.0;
          if (v != want) return 4;
        }
      }
    }
    return diag ? 0 : 5;
  };
  const int64_t nchunk = 64;
  std::vector<int64_t> first_row(size_t(nchunk), -1);
  std::vector<int> first_code(size_t(nchunk), 0);
  const int64_t rows_per = (int64_t(L.n) + nchunk - 1) / nchunk;
  parallel_for(nchunk, 1, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t i = c * rows_per; i < std::min<int64_t>(L.n, (c + 1) * rows_per); ++i) {
        const int e = row_error(int32_t(i));
        if (e) {
          first_row[size_t(c)] = i;
          first_code[size_t(c)] = e;
          break;
        }
      }
  });
  for (int64_t c = 0; c < nchunk; ++c)
    if (first_row[size_t(c)] >= 0) return fail(MG_EINVAL, at + kRowError[first_code[size_t(c)]]);
  for (double v : L.sblk)
    if (!std::isfinite(v)) return fail(MG_EINVAL, at + "non-finite smoother block value");
  if (C) {
    if (C->B != B) return fail(MG_EINVAL, at + "block size differs between levels");
    if (L.pc != C->n) return fail(MG_EINVAL, at + "p_cols != n_nodes of the coarser level");
    if (L.prow.size() != size_t(L.n) + 1 || L.prow[0] != 0) return fail(MG_EINVAL, at + "bad P rowptr");
    for (int32_t i = 0; i < L.n; ++i) {
      if (L.prow[i + 1] < L.prow[i]) return fail(MG_EINVAL, at + "P rowptr not monotone");
      for (int32_t k = L.prow[i]; k < L.prow[i + 1]; ++k) {
        const int32_t j = L.pcol[k];
        if (j < 0 || j >= C->n) return fail(MG_EINVAL, at + "P column out of range");
        if (k > L.prow[i] && L.pcol[k - 1] >= j) return fail(MG_EINVAL, at + "P columns not sorted/unique");
        if (!std::isfinite(L.pval[k])) return fail(MG_EINVAL, at + "non-finite P weight");
      }
    }
  }
  return MG_OK;
}

int load_level(const mg_level_in& in, bool on_dev, bool want_p, HostLevel& L) {
  L.n = in.n_nodes;
  L.B = in.block;
  L.nnzb = in.nnzb;
  if (L.n <= 0 || L.B < 1 || L.B > 8 || L.nnzb < L.n) return fail(MG_EINVAL, "bad level sizes");
  int rc;
  if ((rc = fetch(L.rowptr, in.A_rowptr, size_t(L.n) + 1, on_dev))) return rc;
  if ((rc = fetch(L.col, in.A_col, size_t(L.nnzb), on_dev))) return rc;
  if ((rc = fetch(L.val, in.A_val, size_t(L.nnzb) * L.B * L.B, on_dev))) return rc;
  if ((rc = fetch(L.mask, in.dof_mask, size_t(L.n) * L.B, on_dev))) return rc;
  if (in.smoother_blocks && (rc = fetch(L.sblk, in.smoother_blocks, size_t(L.n) * L.B * L.B, on_dev))) return rc;
  if (want_p) {
    L.pc = in.p_cols;
    if (!in.P_rowptr) return fail(MG_EINVAL, "missing P on a level above 0");
    if ((rc = fetch(L.prow, in.P_rowptr, size_t(L.n) + 1, on_dev))) return rc;
    if (L.prow[L.n] != in.p_nnz || in.p_nnz < 0) return fail(MG_EINVAL, "P rowptr[n] != p_nnz");
    if ((rc = fetch(L.pcol, in.P_col, size_t(in.p_nnz), on_dev))) return rc;
    if ((rc = fetch(L.pval, in.P_val, size_t(in.p_nnz), on_dev))) return rc;
  }
  return MG_OK;
}

// smallest e with max |a| <= 2^e (0 for a zero row)
int row_exponent(double mx) {
  if (mx == 0.0) return 0;
  int e;
  const double m = std::frexp(mx, &e);
  return m == 0.5 ? e - 1 : e;
}

// round an FP64 value to FP16 (RNE, straight from FP64) and return the bits
uint16_t to_f16_bits(double v) {
  if (v == 0.0) return std::signbit(v) ? 0x8000 : 0;
  const double a = std::fabs(v);
  double r;
  if (a >= 0x1p-14) {
    int e;
    const double m = std::frexp(a, &e);            // a = m 2^e, m in [0.5, 1)
    r = std::ldexp(std::nearbyint(std::ldexp(m, 11)), e - 11);
  } else {
    r = std::ldexp(std::nearbyint(std::ldexp(a, 24)), -24);
  }
  // r is exactly representable in FP16; build its bits
  uint16_t bits;
  if (r == 0.0) {
    bits = 0;
  } else if (r < 0x1p-14) {
    bits = uint16_t(std::ldexp(r, 24));
  } else {
    int e;
    const double m = std::frexp(r, &e);
    const int E = e - 1 + 15;                       // r = 1.f 2^(e-1)
    if (E >= 31) bits = 0x7c00;                      // overflow -> inf (not reached for |q| <= 1)
    else bits = uint16_t((E << 10) | (uint32_t(std::ldexp(m, 11)) & 0x3ff));
  }
  return std::signbit(v) ? uint16_t(bits | 0x8000) : bits;
}

uint16_t to_bf16_bits(double v) {
  if (v == 0.0) return std::signbit(v) ? 0x8000 : 0;
  int e;
  const double m = std::frexp(v, &e);
  const double r = std::ldexp(std::nearbyint(std::ldexp(m, 8)), e - 8);
  const float f = float(r);                         // exact
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return uint16_t(u >> 16);
}

struct HostSell {
  int32_t n = 0, B = 1, R = 64, W = 64, nslices = 0, ell = 0;
  int64_t slots = 0;
  std::vector<int32_t> perm;                        // node at each row position (empty: itself)
  std::vector<int32_t> sptr, col;
  std::vector<double> val;                          // slots * B * W
  std::vector<int8_t> rexp;                         // nslices * W
};

// Uniform slice width (plain ELL) on levels of up to 2^18 scalar rows, whose kernels wait
// on memory latency rather than bandwidth, when padding every slice to the widest one
// adds at most 12.5% slots (on larger levels only when it adds none: there the extra
// bytes cost more than the saved slice-pointer load, measured +2% on the 3D sweeps); the
// kernels then compute a slice's slot range instead of loading it.  Padding slots
// contribute exact zeros, so the results are those of the variable widths (MGQ1_NO_ELL=1
// keeps those, for tests).
bool want_ell(int64_t slots, int64_t nslices, int32_t maxw, int64_t rows) {
  const char* off = std::getenv("MGQ1_NO_ELL");
  if (off && std::atoi(off) != 0) return false;
  const int64_t ell = nslices * int64_t(maxw);
  if (maxw <= 0 || ell >= (int64_t(1) << 31)) return false;
  return ell == slots || (rows <= (int64_t(1) << 18) && ell * 8 <= slots * 9);
}

// Operator streams of at most half the 256 MB memory-side cache (MALL) are read with
// ordinary loads, so that the next kernel touching the level finds them there; larger ones
// with non-temporal loads, which leave the cache to the gathered vectors.  Measured on the
// 1M-unknown 2D problem: FP64 solve 8% faster with ordinary loads (its 91 MB finest operator
// stays cached); on the 1 GB 3D operator 6% slower.  MGQ1_LOADS=nt or =t forces one kind
// everywhere (tests; the results are identical).
constexpr int64_t kCachedStreamBytes = int64_t(128) << 20;

int stream_nt(int64_t bytes) {
  if (const char* e = std::getenv("MGQ1_LOADS")) {
    if (std::strcmp(e, "nt") == 0) return 1;
    if (std::strcmp(e, "t") == 0) return 0;
  }
  return bytes > kCachedStreamBytes ? 1 : 0;
}

// slice pointers of uniform width w
void make_uniform(std::vector<int32_t>& sptr, int32_t nslices, int32_t w) {
  for (int32_t s = 0; s <= nslices; ++s) sptr[s] = s * w;
}

int32_t max_width(const std::vector<int32_t>& sptr, int32_t nslices) {
  int32_t w = 0;
  for (int32_t s = 0; s < nslices; ++s) w = std::max(w, sptr[s + 1] - sptr[s]);
  return w;
}

// Rows of block systems (B >= 2) are sorted by length, longest first and otherwise in node
// order, inside windows of kSortSlices slices when that saves at least 3% of the slots: on
// adaptive meshes a constrained node (one diagonal block) or a master next to hanging nodes
// (up to 43 blocks in 3D) would otherwise set the width of a whole slice.  Every row keeps
// its slot order, so its sum is unchanged; only the lane that computes it moves.  One
// component per node is left in node order (the fused two-sweep kernel relies on it).
// MGQ1_NO_SORT=1 keeps the node order everywhere (tests).
constexpr int kSortSlices = 64;

std::vector<int32_t> sorted_positions(const HostLevel& L, int R) {
  std::vector<int32_t> perm;
  const char* off = std::getenv("MGQ1_NO_SORT");
  if (L.B < 2 || L.n == 0 || (off && std::atoi(off) != 0)) return perm;
  auto len = [&](int32_t i) { return L.rowptr[i + 1] - L.rowptr[i]; };
  auto slots_of = [&](const std::vector<int32_t>* p) {
    int64_t t = 0;
    for (int64_t s0 = 0; s0 < L.n; s0 += R) {
      int32_t w = 0;
      for (int64_t q = s0; q < std::min<int64_t>(s0 + R, L.n); ++q) w = std::max(w, len(p ? (*p)[q] : int32_t(q)));
      t += w;
    }
    return t;
  };
  perm.resize(size_t(L.n));
  std::iota(perm.begin(), perm.end(), 0);
  const int64_t win = int64_t(R) * kSortSlices;
  for (int64_t w0 = 0; w0 < L.n; w0 += win)
    std::stable_sort(perm.begin() + w0, perm.begin() + std::min<int64_t>(w0 + win, L.n),
                     [&](int32_t a, int32_t c) { return len(a) > len(c); });
  if (slots_of(&perm) * 100 > slots_of(nullptr) * 97) perm.clear();
  return perm;
}

// sliced ELL with slices of R = 64 / (B * NR) nodes and padded row-lane stride W = 64 / NR
HostSell build_sell(const HostLevel& L, int NR = 1) {
  HostSell S;
  S.n = L.n;
  S.B = L.B;
  S.R = kWave / (L.B * NR);
  S.W = kWave / NR;
  S.nslices = (L.n + S.R - 1) / S.R;
  S.perm = sorted_positions(L, S.R);
  auto node_at = [&](int64_t pos) -> int64_t { return S.perm.empty() ? pos : S.perm[size_t(pos)]; };
  S.sptr.assign(size_t(S.nslices) + 1, 0);
  for (int32_t s = 0; s < S.nslices; ++s) {
    int32_t w = 0;
    for (int r = 0; r < S.R; ++r) {
      const int64_t pos = int64_t(s) * S.R + r;
      if (pos >= L.n) continue;
      const int64_t i = node_at(pos);
      w = std::max(w, L.rowptr[i + 1] - L.rowptr[i]);
    }
    S.sptr[s + 1] = S.sptr[s] + w;
  }
  const int32_t maxw = max_width(S.sptr, S.nslices);
  if (want_ell(S.sptr[S.nslices], S.nslices, maxw, int64_t(L.n) * L.B)) {
    S.ell = maxw;
    make_uniform(S.sptr, S.nslices, maxw);
  }
  S.slots = S.sptr[S.nslices];
  const int B = L.B, W = S.W;
  S.col.assign(size_t(S.slots) * S.R, 0);
  S.val.assign(size_t(S.slots) * B * W, 0.0);
  S.rexp.assign(size_t(S.nslices) * W, 0);
  // every slice fills its own slots and exponents (parallel over slices)
  parallel_for(S.nslices, 1024, [&](int64_t s0, int64_t s1) {
  for (int64_t s = s0; s < s1; ++s) {
    const int32_t w = S.sptr[s + 1] - S.sptr[s];
    for (int r = 0; r < S.R; ++r) {
      const int64_t pos = int64_t(s) * S.R + r;
      if (pos >= L.n) continue;
      const int64_t i = node_at(pos);
      const int32_t len = L.rowptr[i + 1] - L.rowptr[i];
      double mx[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int32_t k = 0; k < w; ++k) {
        const int64_t slot = int64_t(S.sptr[s]) + k;
        if (k < len) {
          const int64_t src = int64_t(L.rowptr[i]) + k;
          S.col[slot * S.R + r] = L.col[src];
          for (int c = 0; c < B; ++c)
            for (int cc = 0; cc < B; ++cc) {
              const double v = L.val[size_t(src) * B * B + c * B + cc];
              S.val[(slot * B + cc) * W + r * B + c] = v;
              mx[c] = std::max(mx[c], std::fabs(v));
            }
        } else {
          S.col[slot * S.R + r] = int32_t(i);
        }
      }
      for (int c = 0; c < B; ++c) S.rexp[size_t(s) * W + r * B + c] = int8_t(row_exponent(mx[c]));
    }
  }
  });
  return S;
}

struct CsrHost {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
};

// sliced ELL of a scalar transfer matrix for block size B and NR right-hand sides: slices
// of R = 64 / (B * NR) node rows, slice width = longest row, padded slots weight 0 and a
// column of their own row
struct TSellHost {
  int32_t nrows = 0, ncols = 0, R = 64, nslices = 0, ell = 0;
  std::vector<int32_t> sptr, col;
  std::vector<double> w;
  std::vector<uint8_t> empty;   // per slot entry: lane of an empty row or past the last row
};

TSellHost build_tsell(const CsrHost& C, int B, int NR) {
  TSellHost S;
  S.nrows = C.nrows;
  S.ncols = C.ncols;
  S.R = kWave / (B * NR);
  S.nslices = (C.nrows + S.R - 1) / S.R;
  S.sptr.assign(size_t(S.nslices) + 1, 0);
  for (int32_t sl = 0; sl < S.nslices; ++sl) {
    int32_t wd = 0;
    for (int r = 0; r < S.R; ++r) {
      const int64_t i = int64_t(sl) * S.R + r;
      if (i < C.nrows) wd = std::max(wd, C.rowptr[i + 1] - C.rowptr[i]);
    }
    S.sptr[sl + 1] = S.sptr[sl] + wd;
  }
  const int32_t maxw = max_width(S.sptr, S.nslices);
  if (want_ell(S.sptr[S.nslices], S.nslices, maxw, int64_t(C.nrows) * B)) {
    S.ell = maxw;
    make_uniform(S.sptr, S.nslices, maxw);
  }
  const int64_t slots = S.sptr[S.nslices];
  S.col.assign(size_t(slots) * S.R, 0);
  S.w.assign(size_t(slots) * S.R, 0.0);
  S.empty.assign(size_t(slots) * S.R, 1);
  for (int32_t sl = 0; sl < S.nslices; ++sl)
    for (int r = 0; r < S.R; ++r) {
      const int64_t i = int64_t(sl) * S.R + r;
      if (i >= C.nrows) continue;
      const int32_t b0 = C.rowptr[i], len = C.rowptr[i + 1] - b0;
      if (len > 0)
        for (int32_t k = 0; k < S.sptr[sl + 1] - S.sptr[sl]; ++k) S.empty[size_t((S.sptr[sl] + k) * S.R + r)] = 0;
      for (int32_t k = 0; k < S.sptr[sl + 1] - S.sptr[sl]; ++k) {
        const int64_t slot = int64_t(S.sptr[sl]) + k;
        if (k < len) {
          S.col[slot * S.R + r] = C.col[b0 + k];
          S.w[slot * S.R + r] = C.val[b0 + k];
        } else {
          S.col[slot * S.R + r] = len > 0 ? C.col[b0 + len - 1] : 0;
        }
      }
    }
  return S;
}

CsrHost transpose(int32_t nrows, int32_t ncols, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                  const std::vector<double>& v) {
  CsrHost T;
  T.nrows = ncols;
  T.ncols = nrows;
  T.rowptr.assign(size_t(ncols) + 1, 0);
  for (int32_t c : ci) ++T.rowptr[c + 1];
  for (int32_t j = 0; j < ncols; ++j) T.rowptr[j + 1] += T.rowptr[j];
  T.col.resize(ci.size());
  T.val.resize(ci.size());
  std::vector<int32_t> fill(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int32_t i = 0; i < nrows; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t q = fill[ci[k]]++;
      T.col[q] = i;
      T.val[q] = v[k];
    }
  return T;
}

}  // namespace

// ---------------------------------------------------------------- handle
// owner of device allocations (freed on destruction)
struct DevOwner {
  std::vector<void*> allocs;
  DevOwner() = default;
  DevOwner(const DevOwner&) = delete;
  DevOwner& operator=(const DevOwner&) = delete;
  ~DevOwner() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

struct LevelDev {
  int32_t n = 0, B = 1;
  int64_t N = 0, nnzb = 0;
  SellDev A64;            // FP64 operator (all levels in FP64 mode; finest level in mixed mode)
  SellDev Ac;             // operator used inside the cycle (== A64 in FP64 mode)
  void* S = nullptr;      // smoother blocks, lane layout, cycle precision
  uint8_t* mask = nullptr;
  CsrDev P, R;            // from level l-1 (l >= 1)
  TSellDev Ps, Rs;        // the same transfers, sliced (grid kernels)
  void *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;   // cycle vectors
  double us_def = 0.0, us_alt = 0.0;  // measured sweep time of the two slot batches (tuning)
  // host copies of the operator's geometry (single-problem handles): BSR row pointers,
  // slice pointers and row positions of the sliced layout, to map stored values back
  std::vector<int32_t> hrow, hsptr, hperm;
};

struct mg_handle : DevOwner {
  mg_config cfg{};
  int L = 0;
  int xk = X_F64;         // vector kind inside the cycle
  std::vector<LevelDev> lv;
  double* Ainv = nullptr; // coarse inverse, row-major
  int n0 = 0;
  int tail_top = -1;      // levels 0..tail_top run in the single-workgroup tail kernel
  TailLevel* dtail = nullptr;
  // outer loop
  double* V = nullptr;    // (m+1) x N_L FP64
  void* Z = nullptr;      // m x N_L, cycle precision
  void* e = nullptr;      // correction (cycle precision), N_L
  double* rout = nullptr; // FP64 outer residual, N_L
  void* bcyc = nullptr;   // cycle-precision copy of the cycle input (mixed mode)
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double* dsc = nullptr;  // device scalars: [0] norm, [1] one, [2..3] givens status
  double* pbig = nullptr; // per-block partials of the outer defect norm
  double* scratch_dev = nullptr;  // this device's copy of `scratch` (device address)
  int scratch_cap = kScratchDoubles;
  double* pv[2] = {nullptr, nullptr};   // per-block partials of the vector reductions
  int* dflag = nullptr;
  bool fuse2z = true;     // fused first two pre-sweeps for block size 1 (MGQ1_NO_FUSE=1: off)
  // Chebyshev smoother (levels >= 1): estimated largest eigenvalue of S A per level and
  // the step coefficients x_{k+1} = x_k + alpha_k S r_k + beta_k (x_k - x_{k-1})
  std::vector<double> lam;
  std::vector<std::vector<double>> cheb_alpha, cheb_beta;
  double* hs = nullptr;   // pinned host scalars
  double* hst = nullptr;  // pinned, device-mapped: Givens output of step j at [2j], [2j+1]
  double* hst_dev = nullptr;             // the same memory as the kernels address it
  std::vector<hipEvent_t> step_done;     // recorded after FGMRES step j
  hipStream_t cap = nullptr;             // private stream used only to capture graphs
  std::vector<hipGraphExec_t> step_graph; // FGMRES step j (V-cycle, SpMV, MGS, Givens)
  ~mg_handle() {
    for (hipGraphExec_t g : step_graph)
      if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : step_done)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    if (hs) (void)hipHostFree(hs);
    if (hst) (void)hipHostFree(hst);
  }
};

namespace {

template <class T>
int dalloc(DevOwner* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(MG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return MG_OK;
}

template <class T>
int upload(DevOwner* h, T** p, const std::vector<T>& src, hipStream_t s) {
  int rc = dalloc(h, p, src.size());
  if (rc) return rc;
  if (!src.empty()) MG_HIP(hipMemcpyAsync(*p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return MG_OK;
}

size_t xsize(int xk) { return xk == X_F64 ? 8 : 4; }

int upload_sell(DevOwner* h, const HostSell& S, int kind, SellDev& D, hipStream_t s) {
  D.n = S.n;
  D.B = S.B;
  D.R = S.R;
  D.nslices = S.nslices;
  D.ell = S.ell;
  D.slots = S.slots;
  D.kind = kind;
  int rc;
  int32_t* sp;
  int32_t* cl;
  if ((rc = upload(h, &sp, S.sptr, s))) return rc;
  if ((rc = upload(h, &cl, S.col, s))) return rc;
  D.sptr = sp;
  D.col = cl;
  if (!S.perm.empty()) {
    int32_t* pm;
    if ((rc = upload(h, &pm, S.perm, s))) return rc;
    D.perm = pm;
  }
  // 16-bit column offsets from a per-slot base (the smallest column of the slot over the
  // slice's rows) in every slice whose slots all span less than 2^16; the other ("wide")
  // slices read the 32-bit columns, marked in a bit mask.  Used when the wide slices hold at
  // most 1/8 of the slots.  Rows past the end of the last slice store offset 0.
  // MGQ1_WIDE_EVERY=n also marks every n-th slice wide (tests of the mixed format).
  int every = 0;
  if (const char* e = std::getenv("MGQ1_WIDE_EVERY")) every = std::max(0, std::atoi(e));
  std::vector<uint16_t> c16(S.col.size(), 0);
  std::vector<int32_t> base(size_t(S.slots), 0);
  std::vector<uint8_t> is_wide(size_t(S.nslices), 0);
  // per slice (parallel): offsets and bases, or the wide mark
  parallel_for(S.nslices, 1024, [&](int64_t s0, int64_t s1) {
  for (int64_t sl = s0; sl < s1; ++sl) {
    bool fits = !(every > 0 && sl % every == 0);
    for (int64_t k = S.sptr[sl]; k < S.sptr[sl + 1] && fits; ++k) {
      int32_t lo = INT32_MAX, hi = INT32_MIN;
      for (int r = 0; r < S.R; ++r)
        if (int64_t(sl) * S.R + r < S.n) {
          lo = std::min(lo, S.col[size_t(k) * S.R + r]);
          hi = std::max(hi, S.col[size_t(k) * S.R + r]);
        }
      if (int64_t(hi) - lo > 65535) { fits = false; break; }
      base[size_t(k)] = lo;
      for (int r = 0; r < S.R; ++r)
        if (int64_t(sl) * S.R + r < S.n) c16[size_t(k) * S.R + r] = uint16_t(S.col[size_t(k) * S.R + r] - lo);
    }
    if (!fits) {
      is_wide[size_t(sl)] = 1;
      for (int64_t k = S.sptr[sl]; k < S.sptr[sl + 1]; ++k) {
        base[size_t(k)] = 0;
        for (int r = 0; r < S.R; ++r) c16[size_t(k) * S.R + r] = 0;
      }
    }
  }
  });
  std::vector<uint32_t> wide((size_t(S.nslices) + 31) / 32, 0u);
  int64_t wide_slots = 0;
  for (int64_t sl = 0; sl < S.nslices; ++sl)
    if (is_wide[size_t(sl)]) {
      wide[size_t(sl) / 32] |= 1u << (sl % 32);
      wide_slots += S.sptr[sl + 1] - S.sptr[sl];
    }
  const char* off = std::getenv("MGQ1_NO_COL16");
  if (wide_slots * 8 <= S.slots && !(off && std::atoi(off) != 0)) {
    uint16_t* c;
    int32_t* bs;
    if ((rc = upload(h, &c, c16, s))) return rc;
    if ((rc = upload(h, &bs, base, s))) return rc;
    if (wide_slots > 0) {
      uint32_t* wm;
      if ((rc = upload(h, &wm, wide, s))) return rc;
      D.wide = wm;
    }
    MG_HIP(hipStreamSynchronize(s));
    D.col16 = c;
    D.colbase = bs;
  }
  const size_t nv = S.val.size();
  const int vbytes = kind == VK_F64 ? 8 : kind == VK_F32 ? 4 : 2;
  D.nt = stream_nt(int64_t(nv) * vbytes + int64_t(S.col.size()) * (D.col16 ? 2 : 4));
  if (kind == VK_F64) {
    double* v;
    if ((rc = upload(h, &v, S.val, s))) return rc;
    D.val = v;
  } else if (kind == VK_F32) {
    std::vector<float> f(nv);
    parallel_for(int64_t(nv), int64_t(1) << 20, [&](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) f[size_t(i)] = float(S.val[size_t(i)]);
    });
    float* v;
    if ((rc = upload(h, &v, f, s))) return rc;
    MG_HIP(hipStreamSynchronize(s));
    D.val = v;
  } else {
    std::vector<uint16_t> q(nv);
    parallel_for(S.nslices, 1024, [&](int64_t s0, int64_t s1) {
      for (int64_t sl = s0; sl < s1; ++sl)
        for (int32_t k = S.sptr[sl]; k < S.sptr[sl + 1]; ++k)
          for (int cc = 0; cc < S.B; ++cc)
            for (int ln = 0; ln < S.W; ++ln) {
              const size_t idx = (size_t(k) * S.B + cc) * S.W + ln;
              const double sc = std::ldexp(S.val[idx], -int(S.rexp[size_t(sl) * S.W + ln]));
              q[idx] = kind == VK_F16 ? to_f16_bits(sc) : to_bf16_bits(sc);
            }
    });
    uint16_t* v;
    if ((rc = upload(h, &v, q, s))) return rc;
    int8_t* re;
    if ((rc = upload(h, &re, S.rexp, s))) return rc;
    MG_HIP(hipStreamSynchronize(s));
    D.val = v;
    D.rexp = re;
  }
  return MG_OK;
}

// Dictionary form of a level's FP64 blocks (MG_PREC_FP64_DICT): the distinct B x B blocks
// of the sliced layout once (padding blocks are zero blocks), a 16-bit index per slot and
// node row.  Applied when the level has at most 65,535 distinct blocks (blocks compare
// bitwise); the kernels then read the same doubles, so every result has the same bits.
struct BlockKey {
  uint64_t w[16];
  int n;
  bool operator==(const BlockKey& o) const {
    for (int i = 0; i < n; ++i)
      if (w[i] != o.w[i]) return false;
    return true;
  }
};
struct BlockHash {
  size_t operator()(const BlockKey& k) const {
    uint64_t x = 1469598103934665603ull;
    for (int i = 0; i < k.n; ++i) {
      x ^= k.w[i] + 0x9e3779b97f4a7c15ull + (x << 6) + (x >> 2);
      x *= 1099511628211ull;
    }
    return size_t(x ^ (x >> 29));
  }
};

int upload_dict(DevOwner* h, const HostSell& S, SellDev& D, hipStream_t s, bool* applied) {
  *applied = false;
  const int B = S.B, BB = B * B, W = S.W, R = S.R;
  if (BB > 16 || W != kWave) return MG_OK;
  const int64_t nblk = S.slots * R;
  auto key_at = [&](int64_t e, BlockKey& key) {
    const int64_t k = e / R, r = e % R;
    key.n = BB;
    for (int c = 0; c < B; ++c)
      for (int cc = 0; cc < B; ++cc) {
        const double v = S.val[size_t((k * B + cc) * W + r * B + c)];
        std::memcpy(&key.w[c * B + cc], &v, 8);
      }
  };
  constexpr size_t kMaxDict = 65535;
  // pass 1: distinct blocks per chunk, in first-seen order
  const int64_t nchunk = 64;
  const int64_t per = (nblk + nchunk - 1) / nchunk;
  std::vector<std::vector<BlockKey>> seen(static_cast<size_t>(nchunk));
  std::vector<int> bad(size_t(nchunk), 0);
  parallel_for(nchunk, 1, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      try {
        std::unordered_map<BlockKey, uint32_t, BlockHash> m;
        BlockKey key;
        for (int64_t e = c * per; e < std::min(nblk, (c + 1) * per); ++e) {
          key_at(e, key);
          if (m.emplace(key, uint32_t(m.size())).second) {
            seen[size_t(c)].push_back(key);
            if (m.size() > kMaxDict) { bad[size_t(c)] = 1; break; }
          }
        }
      } catch (...) {
        bad[size_t(c)] = 2;
      }
    }
  });
  for (int b : bad)
    if (b == 2) return fail(MG_ENOMEM, "host allocation failed (block dictionary)");
  for (int b : bad)
    if (b) return MG_OK;                           // too many distinct blocks: plain values
  std::unordered_map<BlockKey, uint32_t, BlockHash> dict;
  std::vector<double> tab;
  for (const auto& v : seen)
    for (const BlockKey& key : v)
      if (dict.emplace(key, uint32_t(dict.size())).second) {
        if (dict.size() > kMaxDict) return MG_OK;
        for (int i = 0; i < BB; ++i) {
          double d;
          std::memcpy(&d, &key.w[i], 8);
          tab.push_back(d);
        }
      }
  // pass 2: the index of every block (read-only lookups)
  std::vector<uint16_t> idx(static_cast<size_t>(nblk));
  parallel_for(nblk, 1 << 16, [&](int64_t a, int64_t b) {
    BlockKey key;
    for (int64_t e = a; e < b; ++e) {
      key_at(e, key);
      idx[size_t(e)] = uint16_t(dict.find(key)->second);
    }
  });
  int rc;
  uint16_t* di;
  double* dt;
  if ((rc = upload(h, &di, idx, s)) || (rc = upload(h, &dt, tab, s))) return rc;
  MG_HIP(hipStreamSynchronize(s));
  D.kind = VK_DICT;
  D.didx = di;
  D.dtab = dt;
  D.ndict = int32_t(dict.size());
  D.dlds = tab.size() * sizeof(double) <= 16384 ? 1 : 0;     // small tables: one LDS copy per workgroup
  D.nt = stream_nt(int64_t(S.col.size()) * (D.col16 ? 2 : 4) + nblk * 2);
  *applied = true;
  return MG_OK;
}

int upload_csr(DevOwner* h, const CsrHost& C, CsrDev& D, hipStream_t s) {
  D.nrows = C.nrows;
  D.ncols = C.ncols;
  D.nnz = int64_t(C.col.size());
  bool exact = true;
  for (double w : C.val) exact = exact && (double(float(w)) == w);
  D.f32 = exact;
  int rc;
  int32_t *rp, *cl;
  if ((rc = upload(h, &rp, C.rowptr, s))) return rc;
  if ((rc = upload(h, &cl, C.col, s))) return rc;
  D.rowptr = rp;
  D.col = cl;
  if (exact) {
    std::vector<float> f(C.val.begin(), C.val.end());
    float* v;
    if ((rc = upload(h, &v, f, s))) return rc;
    MG_HIP(hipStreamSynchronize(s));
    D.val = v;
  } else {
    double* v;
    if ((rc = upload(h, &v, C.val, s))) return rc;
    D.val = v;
  }
  return MG_OK;
}

int upload_tsell(DevOwner* h, const TSellHost& T, TSellDev& D, hipStream_t s) {
  D.nrows = T.nrows;
  D.ncols = T.ncols;
  D.R = T.R;
  D.nslices = T.nslices;
  D.ell = T.ell;
  bool exact = true;
  for (double w : T.w) exact = exact && (double(float(w)) == w);
  D.f32 = exact;
  D.nt = stream_nt(int64_t(T.col.size()) * (4 + (exact ? 4 : 8)));
  int rc;
  int32_t *sp, *cl;
  if ((rc = upload(h, &sp, T.sptr, s))) return rc;
  if ((rc = upload(h, &cl, T.col, s))) return rc;
  D.sptr = sp;
  D.col = cl;
  if (exact) {
    std::vector<float> f(T.w.begin(), T.w.end());
    float* v;
    if ((rc = upload(h, &v, f, s))) return rc;
    MG_HIP(hipStreamSynchronize(s));
    D.w = v;
  } else {
    double* v;
    if ((rc = upload(h, &v, T.w, s))) return rc;
    MG_HIP(hipStreamSynchronize(s));
    D.w = v;
  }
  return MG_OK;
}

// Node form of a single-right-hand-side transfer C (rows x cols nodes, block size B): slices
// of 64 nodes, one packed 32-bit entry per slot and lane.  Applies when every weight is a
// multiple of 1/128 up to 255/128 (the weights of nested box meshes, with their hanging-node
// products) and every slot's columns span less than 2^16; *applied tells whether it did (else
// the caller stores the per-DoF form).  The span counts the lanes of non-empty rows only: an
// empty row (a Dirichlet node's row of P~) and a lane past the last row add 0 * in[j] to +0
// whatever j, so they read the slot's base column.  Padding slots of a row keep its last
// column and weight 0, as in the per-DoF form, so every sum is the same bit for bit.
// MGQ1_PLAIN_TRANSFERS=1 keeps the per-DoF form everywhere (tests).
int upload_tnode(DevOwner* h, const CsrHost& C, int B, const std::vector<uint8_t>& row_mask,
                 const std::vector<uint8_t>& col_mask, TSellDev& D, hipStream_t s, bool* applied) {
  *applied = false;
  const char* plain = std::getenv("MGQ1_PLAIN_TRANSFERS");
  if ((plain && std::atoi(plain) != 0) || B < 1 || B > 8) return MG_OK;
  if (row_mask.size() != size_t(C.nrows) * B || col_mask.size() != size_t(C.ncols) * B) return MG_OK;
  for (double w : C.val) {
    const double cd = w * 128.0;
    if (!(cd >= 0.0 && cd <= 255.0 && cd == std::floor(cd))) return MG_OK;
  }
  const TSellHost T = build_tsell(C, 1, 1);            // 64 node rows per slice
  const int64_t slots = int64_t(T.col.size()) / T.R;
  std::vector<int32_t> base(size_t(std::max<int64_t>(slots, 1)), 0);
  for (int64_t k = 0; k < slots; ++k) {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int r = 0; r < T.R; ++r) {
      const size_t e = size_t(k * T.R + r);
      if (T.empty[e]) continue;
      lo = std::min(lo, T.col[e]);
      hi = std::max(hi, T.col[e]);
    }
    if (lo > hi) lo = hi = 0;
    if (int64_t(hi) - lo >= 65536) return MG_OK;
    base[size_t(k)] = lo;
  }
  std::vector<uint32_t> ent(T.col.size(), 0u);
  for (int64_t k = 0; k < slots; ++k)
    for (int r = 0; r < T.R; ++r) {
      const size_t e = size_t(k * T.R + r);
      const int32_t j = T.empty[e] ? base[size_t(k)] : T.col[e];
      uint32_t v = uint32_t(j - base[size_t(k)]) | (uint32_t(T.w[e] * 128.0) << 16);
      for (int c = 0; c < B; ++c)
        if (col_mask[size_t(j) * B + c]) v |= 1u << (24 + c);
      ent[e] = v;
    }
  std::vector<uint8_t> rm(size_t(C.nrows), 0);
  for (int64_t i = 0; i < C.nrows; ++i)
    for (int c = 0; c < B; ++c)
      if (row_mask[size_t(i) * B + c]) rm[size_t(i)] |= uint8_t(1u << c);
  int rc;
  int32_t *sp, *cb;
  uint32_t* en;
  uint8_t* rmd;
  if ((rc = upload(h, &sp, T.sptr, s)) || (rc = upload(h, &cb, base, s)) || (rc = upload(h, &en, ent, s)) ||
      (rc = upload(h, &rmd, rm, s)))
    return rc;
  MG_HIP(hipStreamSynchronize(s));
  D = TSellDev();
  D.nrows = T.nrows;
  D.ncols = T.ncols;
  D.R = T.R;
  D.nslices = T.nslices;
  D.ell = T.ell;
  D.sptr = sp;
  D.node = 1;
  D.ent = en;
  D.colbase = cb;
  D.rmask = rmd;
  *applied = true;
  return MG_OK;
}

// ---------------------------------------------------------------- V-cycle
bool chebyshev_on(const mg_handle* h, int l) { return h->cfg.smoother == MG_SMOOTH_CHEBYSHEV && l >= 1; }

// damping of the first step of a smoothing phase (the first sweep from x = 0 included)
double first_omega(const mg_handle* h, int l) { return chebyshev_on(h, l) ? h->cheb_alpha[l][0] : h->cfg.omega; }

// `sweeps` smoothing steps k0, k0 + 1, ... of a phase on level l, ping-pong between cur
// and other (cur holds x_k on entry, the result on exit).  Damped (block-)Jacobi: every
// step is x + omega S (b - A x).  Chebyshev (levels >= 1): step k >= 1 also adds
// beta_k (x_k - x_{k-1}), with x_{k-1} in `other` (or 0 when prev_zero is set for the first
// step taken here), overwritten in place by x_{k+1}.
int smooth_level(mg_handle* h, int l, const void* b, void*& cur, void*& other, int sweeps, hipStream_t s,
                 int k0 = 0, bool prev_zero = false) {
  LevelDev& L = h->lv[l];
  const bool cheb = chebyshev_on(h, l);
  for (int q = 0; q < sweeps; ++q) {
    const int k = k0 + q;
    if (!cheb || k == 0) {
      MG_HIP(launch_sweep(L.Ac, L.S, b, cur, other, cheb ? h->cheb_alpha[l][0] : h->cfg.omega, h->xk, s));
    } else {
      const int pmode = (q == 0 && prev_zero) ? 2 : 1;
      MG_HIP(launch_sweep(L.Ac, L.S, b, cur, other, h->cheb_alpha[l][size_t(k)], h->xk, s,
                          h->cheb_beta[l][size_t(k)], pmode));
    }
    std::swap(cur, other);
  }
  return MG_OK;
}

// x = GMG(L, 0, b) (xinit = false) or GMG(L, x, b) with the initial iterate in xL (xinit =
// true), b and x in cycle precision; x must not alias b.
// Levels above tail_top use grid-wide kernels; levels 0..tail_top run in one
// single-workgroup launch (same steps, same order of ping-pong buffers).
int vcycle_cycle(mg_handle* h, const void* bL, void* xL, hipStream_t s, bool xinit = false) {
  const int L = h->L;
  const mg_config& c = h->cfg;
  const int top = h->tail_top;
  std::vector<const void*> bb(L + 1);
  std::vector<void*> cur(L + 1), oth(L + 1);
  for (int l = 0; l <= L; ++l) bb[l] = h->lv[l].b;
  bb[L] = bL;
  const int pre_pp = c.nu1 >= 1 ? c.nu1 - 1 : 0;
  // choose the first buffer so that the ping-pong ends in the level's own x (or xL)
  auto first_buffers = [&](int l, int pingpongs) {
    void* own = (l == L) ? xL : h->lv[l].x;
    void* tmp = h->lv[l].t;
    if (pingpongs % 2 == 0) { cur[l] = own; oth[l] = tmp; }
    else { cur[l] = tmp; oth[l] = own; }
  };
  for (int l = L; l > top; --l) {
    LevelDev& Lv = h->lv[l];
    if (l == L && xinit) {
      // nu1 + nu2 full sweeps from the given iterate: start in xL when their number is
      // even, else in a copy of it, so that the last post-sweep writes xL
      if ((c.nu1 + c.nu2) % 2 == 0) { cur[l] = xL; oth[l] = Lv.t; }
      else {
        MG_HIP(launch_convert(Lv.N, xL, h->xk, Lv.t, h->xk, s));
        cur[l] = Lv.t;
        oth[l] = xL;
      }
      int rc = smooth_level(h, l, bb[l], cur[l], oth[l], c.nu1, s);
      if (rc) return rc;
      MG_HIP(launch_spmv(Lv.Ac, bb[l], cur[l], Lv.r, Lv.mask, h->xk, h->xk, 2, nullptr, s));
      MG_HIP(launch_restrict_s(Lv.Rs, Lv.B, Lv.r, h->lv[l - 1].b, h->lv[l - 1].mask, nullptr, h->xk, s));
      continue;
    }
    first_buffers(l, pre_pp + c.nu2);
    if (c.nu1 >= 2 && Lv.B == 1 && h->fuse2z) {
      // the first two sweeps from 0 in one pass; leaves the iterate where the second
      // separate sweep would have left it
      MG_HIP(launch_sweep2z(Lv.Ac, Lv.S, bb[l], oth[l], c.omega, h->xk, s));
      std::swap(cur[l], oth[l]);
      int rc = smooth_level(h, l, bb[l], cur[l], oth[l], c.nu1 - 2, s);
      if (rc) return rc;
    } else if (c.nu1 >= 1) {
      MG_HIP(launch_sweep0(Lv.Ac, Lv.S, bb[l], cur[l], first_omega(h, l), h->xk, s));
      int rc = smooth_level(h, l, bb[l], cur[l], oth[l], c.nu1 - 1, s, 1, true);
      if (rc) return rc;
    } else {
      MG_HIP(launch_fill(Lv.N, cur[l], h->xk, 0.0, s));
    }
    MG_HIP(launch_spmv(Lv.Ac, bb[l], cur[l], Lv.r, Lv.mask, h->xk, h->xk, 2, nullptr, s));
    MG_HIP(launch_restrict_s(Lv.Rs, Lv.B, Lv.r, h->lv[l - 1].b, h->lv[l - 1].mask, nullptr, h->xk, s));
  }
  if (top == 0) {
    // coarse solve with grid-wide kernels: one wavefront per row of the dense inverse
    LevelDev& C0 = h->lv[0];
    void* x0 = (L == 0) ? xL : C0.x;
    if (c.coarse_mode == MG_COARSE_EXACT) {
      MG_HIP(launch_coarse_gemv(h->n0, h->Ainv, bb[0], x0, h->xk, s));
    } else {
      const int k = std::max(1, c.coarse_sweeps);
      void* cu = ((k - 1) % 2 == 0) ? x0 : C0.t;
      void* ot = ((k - 1) % 2 == 0) ? C0.t : x0;
      MG_HIP(launch_sweep0(C0.Ac, C0.S, bb[0], cu, c.omega, h->xk, s));
      int rc = smooth_level(h, 0, bb[0], cu, ot, k - 1, s);
      if (rc) return rc;
    }
    if (L == 0) return MG_OK;
  } else {
    // the tail reads level top's right-hand side from its own b and leaves x in its own x
    if (top == L) MG_HIP(launch_convert(h->lv[L].N, bL, h->xk, h->lv[L].b, h->xk, s));
    TailParams tp;
    tp.top = top;
    tp.nu1 = c.nu1;
    tp.nu2 = c.nu2;
    tp.omega = c.omega;
    tp.Ainv = h->Ainv;
    tp.n0 = h->n0;
    tp.coarse_mode = c.coarse_mode;
    tp.coarse_sweeps = c.coarse_sweeps;
    MG_HIP(launch_tail(h->dtail, h->lv[0].B, h->lv[0].Ac.kind, h->xk, tp, s));
    if (top == L) {
      MG_HIP(launch_convert(h->lv[L].N, h->lv[L].x, h->xk, xL, h->xk, s));
      return MG_OK;
    }
  }
  for (int l = top + 1; l <= L; ++l) {
    LevelDev& Lv = h->lv[l];
    const void* y = (l - 1 == top) ? h->lv[top].x : cur[l - 1];
    MG_HIP(launch_prolong_s(Lv.Ps, Lv.B, y, cur[l], Lv.mask, h->lv[l - 1].mask, h->xk, s));
    int rc = smooth_level(h, l, bb[l], cur[l], oth[l], c.nu2, s);
    if (rc) return rc;
  }
  return MG_OK;
}

// z = V(v) with v FP64 (finest), z in cycle precision; converted = the cycle-precision
// copy of v is already in bcyc
int precond(mg_handle* h, const double* v, void* z, hipStream_t s, bool converted = false) {
  if (h->xk == X_F64) return vcycle_cycle(h, v, z, s);
  if (!converted) MG_HIP(launch_convert(h->lv[h->L].N, v, X_F64, h->bcyc, h->xk, s));
  return vcycle_cycle(h, h->bcyc, z, s);
}

int read_scalars(mg_handle* h, const double* d, int k, hipStream_t s) {
  MG_HIP(hipMemcpyAsync(h->hs, d, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

// r = b - A x, h->hs[0] = ||r||
int outer_defect(mg_handle* h, const double* b, const double* x, hipStream_t s) {
  LevelDev& T = h->lv[h->L];
  MG_HIP(launch_spmv(T.A64, b, x, h->rout, nullptr, X_F64, X_F64, 1, h->pbig, s));
  MG_HIP(launch_finish(h->pbig, spmv_grid(T.A64), h->dsc + 0, 1, s));
  return read_scalars(h, h->dsc, 1, s);
}

// One FGMRES step j on internal buffers: z_j = V(v_j), w = A z_j, modified Gram-Schmidt
// against v_0..v_j (Sec. 4.2), v_{j+1} = w / ||w||, Givens rotation j.
int enqueue_fgmres_step(mg_handle* h, int j, hipStream_t s) {
  const int m = h->cfg.gmres_m;
  LevelDev& T = h->lv[h->L];
  const int64_t N = T.N;
  double* vj = h->V + int64_t(j) * N;
  double* w = h->V + int64_t(j + 1) * N;
  void* zj = static_cast<char*>(h->Z) + size_t(j) * N * xsize(h->xk);
  int rc;
  // the cycle-precision copy of v_j was written by the kernel that produced v_j
  if ((rc = precond(h, vj, zj, s, true))) return rc;
  // w = A z_j together with the partial sums of (w, v_0) for the first Gram-Schmidt step
  MG_HIP(launch_spmv(T.A64, nullptr, zj, w, nullptr, h->xk, X_F64, 0, h->pbig, s, h->V));
  double* Hj = h->H + int64_t(j) * (m + 1);
  // each step subtracts the projection on v_i and forms the partial dot products with
  // v_{i+1} (or with w itself after the last step)
  for (int i = 0; i <= j; ++i) {
    const double* vi = h->V + int64_t(i) * N;
    const double* vn = (i < j) ? h->V + int64_t(i + 1) * N : nullptr;
    const double* pin = (i == 0) ? h->pbig : h->pv[i & 1];
    MG_HIP(launch_mgs_step(N, w, vi, vn, pin, h->pv[(i + 1) & 1], Hj + i, s, i == 0 ? spmv_grid(T.A64) : 0));
  }
  // v_{j+1} = w / ||w|| (and its cycle-precision copy for step j+1), then Givens rotation
  // j, whose |g_{j+1}| and breakdown flag go straight to pinned host memory (slot j) so the
  // host can read them while step j+1 is already queued
  float* wc = h->xk == X_F64 ? nullptr : static_cast<float*>(h->bcyc);
  MG_HIP(launch_mgs_normalize(N, w, h->pv[(j + 1) & 1], Hj + j + 1, s, j, m, h->H, h->cs, h->sn, h->g,
                              h->hst_dev + 2 * j, wc));
  return MG_OK;
}

// enqueue step j on the caller's stream: replay its captured graph (captured on first
// use on a private stream) or launch the kernels directly
int fgmres_step(mg_handle* h, int j, hipStream_t s) {
  if (!h->cfg.use_graph) return enqueue_fgmres_step(h, j, s);
  if (!h->step_graph[j]) {
    hipGraph_t g = nullptr;
    MG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_fgmres_step(h, j, h->cap);
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(MG_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(MG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    h->step_graph[j] = ex;
  }
  MG_HIP(hipGraphLaunch(h->step_graph[j], s));
  return MG_OK;
}

int enqueue_step(mg_handle* h, int j, hipStream_t s) {
  int rc = fgmres_step(h, j, s);
  if (rc) return rc;
  MG_HIP(hipEventRecord(h->step_done[j], s));
  return MG_OK;
}

int solve_impl(mg_handle* h, const double* b, double* x, mg_solve_stats* st, void* stream, int fixed) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mg_config& c = h->cfg;
  LevelDev& T = h->lv[h->L];
  const int64_t N = T.N;
  mg_solve_stats S{};
  int rc;
  // ||b|| (to dsc[4]) and the initial defect r = b - A x with ||r|| (to dsc[0]), read
  // back with one synchronisation
  MG_HIP(launch_dot_partials(N, b, nullptr, h->pv[0], s));
  MG_HIP(launch_finish(h->pv[0], reduction_grid(N), h->dsc + 4, 1, s));
  MG_HIP(launch_spmv(T.A64, b, x, h->rout, nullptr, X_F64, X_F64, 1, h->pbig, s));
  MG_HIP(launch_finish(h->pbig, spmv_grid(T.A64), h->dsc + 0, 1, s));
  if ((rc = read_scalars(h, h->dsc, 5, s))) return rc;
  const double bn = h->hs[4];
  const double tol = c.rtol * bn;
  const int limit = fixed > 0 ? fixed : c.maxit;
  double beta = h->hs[0];
  S.res0 = beta;
  int status = MG_OK;
  if (c.outer == MG_OUTER_IR) {
    while (true) {
      if (!std::isfinite(beta) || beta > 1e6 * std::max(S.res0, 1e-300)) { status = MG_ENUMERIC; break; }
      if (fixed <= 0 && beta <= tol) { S.converged = 1; break; }
      if (S.iters >= limit) { status = fixed > 0 ? MG_OK : MG_ENOCONV; break; }
      if ((rc = precond(h, h->rout, h->e, s))) return rc;
      MG_HIP(launch_axpy(N, x, X_F64, h->e, h->xk, 1.0, h->dsc + 1, s));
      ++S.iters;
      if ((rc = outer_defect(h, b, x, s))) return rc;
      beta = h->hs[0];
    }
  } else {
    const int m = c.gmres_m;
    while (true) {
      if (!std::isfinite(beta) || beta > 1e6 * std::max(S.res0, 1e-300)) { status = MG_ENUMERIC; break; }
      if (fixed <= 0 && beta <= tol) { S.converged = 1; break; }
      if (S.iters >= limit || beta == 0.0) { status = (fixed > 0 || beta == 0.0) ? MG_OK : MG_ENOCONV; break; }
      MG_HIP(launch_scale_div(N, h->V, h->rout, h->dsc + 0, s,
                              h->xk == X_F64 ? nullptr : static_cast<float*>(h->bcyc)));
      MG_HIP(launch_init_g(m, h->g, h->dsc + 0, s));
      // Step j+1 is queued before the host waits for step j whenever the residual
      // estimates predict that it will be needed (a mispredicted step only costs time: it
      // writes basis vectors and Hessenberg entries beyond the ones the update uses).
      int k = 0;
      double last = beta, rate = 0.5;
      if ((rc = enqueue_step(h, 0, s))) return rc;
      for (int j = 0; j < m; ++j) {
        ++S.iters;
        const bool more = j + 1 < m && S.iters < limit;
        const bool spec = more && (fixed > 0 || last * rate > 2.0 * tol);
        if (spec && (rc = enqueue_step(h, j + 1, s))) return rc;
        MG_HIP(hipEventSynchronize(h->step_done[j]));
        k = j + 1;
        const double est = h->hst[2 * j];
        const bool breakdown = h->hst[2 * j + 1] != 0.0;
        if (!std::isfinite(est)) { status = MG_ENUMERIC; break; }
        if (breakdown || S.iters >= limit) break;
        if (fixed <= 0 && est <= tol) break;
        if (est > 0.0 && last > 0.0) rate = std::min(1.0, est / last);
        last = est;
        if (!spec && more && (rc = enqueue_step(h, j + 1, s))) return rc;
      }
      if (status == MG_ENUMERIC) break;
      MG_HIP(launch_backsolve(k, m, h->H, h->g, h->y, s));
      MG_HIP(launch_update_x(N, x, h->Z, h->xk, N, h->y, k, s));
      ++S.restarts;
      if ((rc = outer_defect(h, b, x, s))) return rc;
      beta = h->hs[0];
    }
    if (status == MG_OK && fixed <= 0 && beta > tol) status = MG_ENOCONV;
  }
  S.res_final = beta;
  S.converged = (beta <= tol) ? 1 : 0;
  if (status == MG_OK && fixed <= 0 && !S.converged) status = MG_ENOCONV;
  S.status = status;
  MG_HIP(hipStreamSynchronize(s));
  S.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = S;
  if (status == MG_ENUMERIC) return fail(MG_ENUMERIC, "non-finite or diverging residual");
  if (status == MG_ENOCONV) return fail(MG_ENOCONV, "maxit reached before rtol");
  return MG_OK;
}

int check_level(const mg_handle* h, int level) {
  if (!h) return fail(MG_EINVAL, "null handle");
  if (level < 0 || level > h->L) return fail(MG_EINVAL, "level out of range");
  return MG_OK;
}

}  // namespace

namespace {

int value_kind(int precision) {
  return precision == MG_PREC_FP64 ? VK_F64
         : precision == MG_PREC_FP32 ? VK_F32
         : precision == MG_PREC_FP32_F16VAL ? VK_F16
         : precision == MG_PREC_FP64_DICT ? VK_F64 : VK_BF16;
}

int check_config(const mg_config& c) {
  if (!(c.omega > 0.0) || c.nu1 < 0 || c.nu2 < 0 || c.nu1 + c.nu2 < 1 || c.gmres_m < 1 || c.gmres_m > 64 ||
      c.maxit < 0 || !(c.rtol >= 0.0) || c.precision < MG_PREC_FP64 || c.precision > MG_PREC_FP64_DICT ||
      (c.outer != MG_OUTER_IR && c.outer != MG_OUTER_FGMRES) ||
      (c.coarse_mode != MG_COARSE_EXACT && c.coarse_mode != MG_COARSE_SMOOTH))
    return fail(MG_EINVAL, "invalid configuration");
  if (c.smoother != MG_SMOOTH_JACOBI && c.smoother != MG_SMOOTH_CHEBYSHEV) return fail(MG_EINVAL, "unknown smoother");
  if (c.smoother == MG_SMOOTH_CHEBYSHEV &&
      (!(c.cheb_lo > 0.0) || !(c.cheb_hi > c.cheb_lo) || !std::isfinite(c.cheb_hi) || c.power_its < 1 || c.power_its > 1000))
    return fail(MG_EINVAL, "Chebyshev smoother needs 0 < cheb_lo < cheb_hi and 1 <= power_its <= 1000");
  return MG_OK;
}

// Largest eigenvalue of S A on every level >= 1 by power iteration from the Weyl vector
// (v <- S A v / ||S A v||, power_its steps, the last norm is the estimate), then the
// Chebyshev step coefficients on [cheb_lo, cheb_hi] * lambda (three-term recurrence of
// the Chebyshev iteration, Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.3).
int setup_chebyshev(mg_handle* h, hipStream_t s) {
  const mg_config& c = h->cfg;
  const int kmax = std::max(std::max(c.nu1, c.nu2), 1);
  h->lam.assign(size_t(h->L) + 1, 0.0);
  h->cheb_alpha.assign(size_t(h->L) + 1, {});
  h->cheb_beta.assign(size_t(h->L) + 1, {});
  for (int l = 1; l <= h->L; ++l) {
    LevelDev& Lv = h->lv[l];
    const int64_t n = Lv.N;
    MG_HIP(launch_weyl(n, Lv.t, h->xk, s));
    MG_HIP(launch_sumsq_partials(n, Lv.t, h->xk, h->pv[0], s));
    MG_HIP(launch_finish(h->pv[0], reduction_grid(n), h->dsc + 6, 1, s));
    MG_HIP(launch_scale_inv(n, Lv.x, Lv.t, h->xk, h->dsc + 6, s));
    for (int it = 0; it < c.power_its; ++it) {
      MG_HIP(launch_spmv(Lv.Ac, nullptr, Lv.x, Lv.r, nullptr, h->xk, h->xk, 0, nullptr, s));
      MG_HIP(launch_sweep0(Lv.Ac, Lv.S, Lv.r, Lv.t, 1.0, h->xk, s));
      MG_HIP(launch_sumsq_partials(n, Lv.t, h->xk, h->pv[0], s));
      MG_HIP(launch_finish(h->pv[0], reduction_grid(n), h->dsc + 6, 1, s));
      MG_HIP(launch_scale_inv(n, Lv.x, Lv.t, h->xk, h->dsc + 6, s));
    }
    double lam = 0.0;
    MG_HIP(hipMemcpyAsync(&lam, h->dsc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (!(lam > 0.0) || !std::isfinite(lam)) return fail(MG_ENUMERIC, "eigenvalue estimate of S A is not positive and finite");
    h->lam[size_t(l)] = lam;
    const double a = c.cheb_lo * lam, bnd = c.cheb_hi * lam;
    const double theta = 0.5 * (bnd + a), delta = 0.5 * (bnd - a), sigma = theta / delta;
    std::vector<double>& al = h->cheb_alpha[size_t(l)];
    std::vector<double>& be = h->cheb_beta[size_t(l)];
    al.assign(size_t(kmax), 0.0);
    be.assign(size_t(kmax), 0.0);
    al[0] = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int k = 1; k < kmax; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      al[size_t(k)] = 2.0 * rn / delta;
      be[size_t(k)] = rn * rho;
      rho = rn;
    }
  }
  return MG_OK;
}

int load_hierarchy(const mg_level_in* lv, int n_levels, bool on_dev, std::vector<HostLevel>& H) {
  H.resize(n_levels);
  try {
    for (int l = 0; l < n_levels; ++l) {
      int rc = load_level(lv[l], on_dev, l > 0, H[l]);
      if (rc) return rc;
      rc = validate_host(H[l], l > 0 ? &H[l - 1] : nullptr, l);
      if (rc) return rc;
    }
  } catch (const std::bad_alloc&) {
    return fail(MG_ENOMEM, "host allocation failed");
  }
  if (H[0].B > 4) return fail(MG_EUNSUPPORTED, "block sizes above 4 are not implemented");
  if (int64_t(H[0].n) * H[0].B > 4096) return fail(MG_EUNSUPPORTED, "coarse problem above 4096 DoFs");
  return MG_OK;
}

// MGQ1_SETUP_TIMES=1: print the wall time of each setup phase to stderr (diagnostics)
struct PhaseTimer {
  bool on = false;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  PhaseTimer() {
    const char* e = std::getenv("MGQ1_SETUP_TIMES");
    on = e && std::atoi(e) != 0;
  }
  void mark(const char* what, int level = -1) {
    if (!on) return;
    const auto n = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(n - t).count();
    if (level >= 0) std::fprintf(stderr, "[mgq1 setup] %s %d: %.1f ms\n", what, level, ms);
    else std::fprintf(stderr, "[mgq1 setup] %s: %.1f ms\n", what, ms);
    t = n;
  }
};

// one level on the device: FP64 and cycle operators (sliced ELL for NR right-hand sides),
// smoother blocks, mask, P~ and R = P~^T; with vectors = true also x, b, r, t
// single: a single-problem handle (keeps the host pattern for the step-wise entry points
// and stores its transfers in the node form where they qualify); the batch reads the
// per-DoF form
int setup_level(DevOwner* h, const HostLevel& L, bool has_p, int NR, int vkind, int xk, bool vectors, int* flag,
                hipStream_t s, LevelDev& D, bool single = false, const HostLevel* coarser = nullptr,
                bool dict = false) {
  const bool keep_host = single;
  int rc;
  D.n = L.n;
  D.B = L.B;
  D.N = int64_t(L.n) * L.B;
  D.nnzb = L.nnzb;
  PhaseTimer pt;
  HostSell S = build_sell(L, NR);
  pt.mark("  sliced layout");
  if ((rc = upload_sell(h, S, VK_F64, D.A64, s))) return rc;
  pt.mark("  FP64 operator upload");
  if (vkind == VK_F64) D.Ac = D.A64;
  else if ((rc = upload_sell(h, S, vkind, D.Ac, s))) return rc;
  pt.mark("  cycle operator");
  const size_t sblk = size_t(S.nslices) * L.B * S.W;
  if ((rc = dalloc(h, reinterpret_cast<char**>(&D.S), sblk * xsize(xk)))) return rc;
  if (L.sblk.empty()) {
    MG_HIP(launch_fill(int64_t(sblk), D.S, xk, 0.0, s));
    MG_HIP(launch_block_invert(D.A64, D.S, xk, flag, NR, s));
  } else {
    // the caller's fixed smoother matrix S (Sec. 4.1) in the lane layout of the sweeps:
    // lane r * B + c of a slice holds row c of its node's block, column cc at
    // S[(slice * B + cc) * W + r * B + c]
    std::vector<double> lane(sblk, 0.0);
    const int B = L.B;
    for (int64_t pos = 0; pos < L.n; ++pos) {
      const int64_t node = S.perm.empty() ? pos : S.perm[size_t(pos)];
      const int64_t slice = pos / S.R, r = pos % S.R;
      for (int c = 0; c < B; ++c)
        for (int cc = 0; cc < B; ++cc)
          lane[size_t((slice * B + cc) * S.W + r * B + c)] = L.sblk[size_t(node * B * B + c * B + cc)];
    }
    if (xk == X_F64) {
      MG_HIP(hipMemcpyAsync(D.S, lane.data(), sblk * sizeof(double), hipMemcpyHostToDevice, s));
      MG_HIP(hipStreamSynchronize(s));
    } else {
      std::vector<float> lf(lane.begin(), lane.end());
      MG_HIP(hipMemcpyAsync(D.S, lf.data(), sblk * sizeof(float), hipMemcpyHostToDevice, s));
      MG_HIP(hipStreamSynchronize(s));
    }
  }
  if (keep_host) {
    D.hrow = L.rowptr;
    D.hsptr = S.sptr;
    D.hperm = S.perm;
  }
  if ((rc = upload(h, &D.mask, L.mask, s))) return rc;
  pt.mark("  smoother blocks and mask");
  if (dict && NR == 1) {
    // the smoother blocks above were computed from the plain FP64 values; from here on the
    // level's kernels read the dictionary form of the same values
    MG_HIP(hipStreamSynchronize(s));
    bool ok = false;
    if ((rc = upload_dict(h, S, D.A64, s, &ok))) return rc;
    if (ok) D.Ac = D.A64;
    pt.mark("  block dictionary");
  }
  if (has_p) {
    CsrHost P;
    P.nrows = L.n;
    P.ncols = L.pc;
    P.rowptr = L.prow;
    P.col = L.pcol;
    P.val = L.pval;
    if ((rc = upload_csr(h, P, D.P, s))) return rc;
    CsrHost R = transpose(L.n, L.pc, L.prow, L.pcol, L.pval);
    if ((rc = upload_csr(h, R, D.R, s))) return rc;
    bool pn = false, rn = false;
    if (single && NR == 1 && coarser) {
      if ((rc = upload_tnode(h, P, L.B, L.mask, coarser->mask, D.Ps, s, &pn))) return rc;
      if ((rc = upload_tnode(h, R, L.B, coarser->mask, L.mask, D.Rs, s, &rn))) return rc;
    }
    if (!pn && (rc = upload_tsell(h, build_tsell(P, L.B, NR), D.Ps, s))) return rc;
    if (!rn && (rc = upload_tsell(h, build_tsell(R, L.B, NR), D.Rs, s))) return rc;
    pt.mark("  transfers");
  }
  if (vectors) {
    const size_t vb = size_t(D.N) * NR * xsize(xk);
    char* p;
    for (void** v : {&D.x, &D.b, &D.r, &D.t}) {
      if ((rc = dalloc(h, &p, vb))) return rc;
      *v = p;
    }
  }
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

// dense inverse of the coarse operator (GPU Gauss-Jordan), row-major FP64
int setup_coarse_inverse(DevOwner* h, const HostLevel& C0, int* flag, hipStream_t s, double** Ainv, int* n0out) {
  const int B = C0.B;
  const int n0 = C0.n * B;
  *n0out = n0;
  std::vector<double> M(size_t(n0) * 2 * n0, 0.0);
  for (int32_t i = 0; i < C0.n; ++i)
    for (int32_t k = C0.rowptr[i]; k < C0.rowptr[i + 1]; ++k)
      for (int c1 = 0; c1 < B; ++c1)
        for (int c2 = 0; c2 < B; ++c2)
          M[size_t(i * B + c1) * 2 * n0 + size_t(C0.col[k]) * B + c2] = C0.val[size_t(k) * B * B + c1 * B + c2];
  for (int i = 0; i < n0; ++i) M[size_t(i) * 2 * n0 + n0 + i] = 1.0;
  double *dM, *piv;
  int rc;
  if ((rc = upload(h, &dM, M, s))) return rc;
  MG_HIP(hipStreamSynchronize(s));
  if ((rc = dalloc(h, &piv, size_t(2) * n0))) return rc;
  if ((rc = dalloc(h, Ainv, size_t(n0) * n0))) return rc;
  MG_HIP(launch_coarse_invert(n0, dM, *Ainv, piv, flag, s));
  return MG_OK;
}

int check_flag(int* flag, hipStream_t s) {
  int hflag = 0;
  MG_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hflag) return fail(MG_ESINGULAR, "singular nodal diagonal block or coarse matrix");
  return MG_OK;
}

// Slot-batch choice per level.  slot_batch == 0: time the level's smoothing sweep with
// both slot-batch variants (interleaved repetitions, minimum kept) and keep the faster for
// the sweeps and defects of that level; the finest FP64 operator of a mixed-precision
// handle is timed with the outer defect.  Otherwise the given value is used everywhere.
// Both variants run the FMAs in the same order, so the choice never changes a result.
int tune_levels(mg_handle* h, hipStream_t s) {
  const int req = h->cfg.slot_batch;
  for (LevelDev& D : h->lv) {
    int kd, ko;
    slot_batch_choices(D.B, &kd, &ko);
    if (req != 0 && req != kd && req != ko)
      return fail(MG_EINVAL, "slot_batch must be 0 or one of the two batch sizes built for this block size");
    if (req != 0) {
      D.Ac.kb = D.A64.kb = req;
      continue;
    }
  }
  if (req != 0) return MG_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  int rc = MG_OK;
  auto timed = [&](auto&& launch, int reps, float* ms) -> int {
    MG_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) MG_HIP(launch(i));
    MG_HIP(hipEventRecord(e1, s));
    MG_HIP(hipEventSynchronize(e1));
    MG_HIP(hipEventElapsedTime(ms, e0, e1));
    return MG_OK;
  };
  const double omega = h->cfg.omega;
  for (size_t l = 0; l < h->lv.size() && rc == MG_OK; ++l) {
    LevelDev& D = h->lv[l];
    int kb[2];
    slot_batch_choices(D.B, &kb[0], &kb[1]);
    if ((rc = launch_fill(D.N, D.x, h->xk, 1.0, s) == hipSuccess ? MG_OK : MG_EDEVICE)) break;
    if ((rc = launch_fill(D.N, D.b, h->xk, 1.0, s) == hipSuccess ? MG_OK : MG_EDEVICE)) break;
    float best[2] = {1e30f, 1e30f};
    for (int rep = 0; rep < 3 && rc == MG_OK; ++rep)
      for (int v = 0; v < 2 && rc == MG_OK; ++v) {
        D.Ac.kb = kb[v];
        float ms = 0.f;
        rc = timed([&](int i) {
          return (i & 1) ? launch_sweep(D.Ac, D.S, D.b, D.t, D.x, omega, h->xk, s)
                         : launch_sweep(D.Ac, D.S, D.b, D.x, D.t, omega, h->xk, s);
        }, 10, &ms);
        best[v] = std::min(best[v], ms);
      }
    const int pick = best[1] < best[0] ? 1 : 0;
    D.Ac.kb = kb[pick];
    if (h->xk == X_F64) D.A64.kb = kb[pick];
    D.us_def = 100.0 * best[0];          // ms per 10 launches -> us per launch
    D.us_alt = 100.0 * best[1];
  }
  if (rc == MG_OK && h->xk != X_F64) {
    // FP64 outer defect of a mixed-precision handle: r = b - A x with norm partials
    LevelDev& T = h->lv[h->L];
    int kb[2];
    slot_batch_choices(T.B, &kb[0], &kb[1]);
    double* xb = h->V ? h->V : nullptr;
    if (xb == nullptr) {
      T.A64.kb = T.Ac.kb;
    } else {
      const int64_t N = T.N;
      if ((rc = launch_fill(2 * N, xb, X_F64, 1.0, s) == hipSuccess ? MG_OK : MG_EDEVICE) == MG_OK) {
        float best[2] = {1e30f, 1e30f};
        for (int rep = 0; rep < 3 && rc == MG_OK; ++rep)
          for (int v = 0; v < 2 && rc == MG_OK; ++v) {
            T.A64.kb = kb[v];
            float ms = 0.f;
            rc = timed([&](int) {
              return launch_spmv(T.A64, xb, xb + N, h->rout, nullptr, X_F64, X_F64, 1, h->pbig, s);
            }, 10, &ms);
            best[v] = std::min(best[v], ms);
          }
        T.A64.kb = kb[best[1] < best[0] ? 1 : 0];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int setup_handle(mg_handle* h, const std::vector<HostLevel>& H, hipStream_t s) {
  PhaseTimer pt;
  const mg_config& c = h->cfg;
  const int n_levels = int(H.size());
  int rc;
  int* flag;
  if ((rc = dalloc(h, &flag, 1))) return rc;
  h->dflag = flag;
  MG_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  const int vkind = value_kind(c.precision);
  for (int l = 0; l < n_levels; ++l) {
    if ((rc = setup_level(h, H[l], l > 0, 1, vkind, h->xk, true, flag, s, h->lv[l], true,
                          l > 0 ? &H[l - 1] : nullptr, c.precision == MG_PREC_FP64_DICT)))
      return rc;
    if (pt.on) MG_HIP(hipStreamSynchronize(s));
    pt.mark("level", l);
  }
  if ((rc = setup_coarse_inverse(h, H[0], flag, s, &h->Ainv, &h->n0))) return rc;
  if ((rc = check_flag(flag, s))) return rc;
  pt.mark("coarse inverse");
  // outer-loop storage
  const int64_t N = h->lv[h->L].N;
  const int m = c.gmres_m;
  if ((rc = dalloc(h, &h->rout, size_t(N)))) return rc;
  char* p;
  if ((rc = dalloc(h, &p, size_t(N) * xsize(h->xk)))) return rc;
  h->e = p;
  if ((rc = dalloc(h, &p, size_t(N) * xsize(h->xk)))) return rc;
  h->bcyc = p;
  if (c.outer == MG_OUTER_FGMRES) {
    if ((rc = dalloc(h, &h->V, size_t(m + 1) * N))) return rc;
    if ((rc = dalloc(h, &p, size_t(m) * N * xsize(h->xk)))) return rc;
    h->Z = p;
  }
  if ((rc = dalloc(h, &h->H, size_t(m + 1) * m))) return rc;
  if ((rc = dalloc(h, &h->cs, size_t(m)))) return rc;
  if ((rc = dalloc(h, &h->sn, size_t(m)))) return rc;
  if ((rc = dalloc(h, &h->g, size_t(m) + 1))) return rc;
  if ((rc = dalloc(h, &h->y, size_t(m)))) return rc;
  if ((rc = dalloc(h, &h->dsc, 8))) return rc;
  MG_HIP(launch_fill(8, h->dsc, X_F64, 0.0, s));
  MG_HIP(launch_fill(1, h->dsc + 1, X_F64, 1.0, s));
  int64_t maxgrid = 1;
  for (const LevelDev& D : h->lv) maxgrid = std::max<int64_t>(maxgrid, spmv_grid(D.A64));
  if ((rc = dalloc(h, &h->pbig, size_t(maxgrid)))) return rc;
  for (int q = 0; q < 2; ++q)
    if ((rc = dalloc(h, &h->pv[q], size_t(kMaxRedBlocks)))) return rc;
  pt.mark("outer-loop storage");
  if (c.smoother == MG_SMOOTH_CHEBYSHEV && (rc = setup_chebyshev(h, s))) return rc;
  if ((rc = tune_levels(h, s))) return rc;
  pt.mark("Chebyshev bounds and slot-batch timing");
  if (const char* e = std::getenv("MGQ1_NO_FUSE")) h->fuse2z = std::atoi(e) == 0;
  if (c.smoother == MG_SMOOTH_CHEBYSHEV) h->fuse2z = false;   // the fused pair is two Jacobi sweeps
  if (c.precision == MG_PREC_FP64_DICT) h->fuse2z = false;     // the fused pair reads plain values
  // tail: every level up to the largest one with at most tail_dofs unknowns.  Default off:
  // on MI355X one workgroup walking several levels was measured slower (dependent-load
  // latency serialises) than separate grid launches per step.
  int64_t tail_dofs = 0;
  if (const char* e = std::getenv("MGQ1_TAIL_DOFS")) tail_dofs = std::atoll(e);
  int top = 0;
  for (int l = 1; l <= h->L; ++l)
    if (h->lv[l].N <= tail_dofs) top = l;
  if (top >= 1 && c.precision == MG_PREC_FP64_DICT)
    return fail(MG_EUNSUPPORTED, "the single-workgroup tail reads plain values");
  if (top >= 1 && c.smoother == MG_SMOOTH_CHEBYSHEV)
    return fail(MG_EUNSUPPORTED, "the single-workgroup tail runs damped Jacobi sweeps only");
  h->tail_top = top;
  std::vector<TailLevel> tl(top + 1);
  for (int l = 0; l <= top; ++l) {
    const LevelDev& D = h->lv[l];
    tl[l].A = D.Ac;
    tl[l].S = D.S;
    tl[l].mask = D.mask;
    tl[l].P = D.P;
    tl[l].R = D.R;
    tl[l].x = D.x;
    tl[l].b = D.b;
    tl[l].r = D.r;
    tl[l].t = D.t;
  }
  if ((rc = dalloc(h, &h->dtail, tl.size()))) return rc;
  MG_HIP(hipMemcpyAsync(h->dtail, tl.data(), tl.size() * sizeof(TailLevel), hipMemcpyHostToDevice, s));
  MG_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hs), 16 * sizeof(double), hipHostMallocDefault));
  MG_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hst), 2 * size_t(m) * sizeof(double),
                       hipHostMallocMapped | hipHostMallocCoherent));
  MG_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->hst_dev), h->hst, 0));
  h->step_done.assign(size_t(m), nullptr);
  for (hipEvent_t& e : h->step_done) MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  h->step_graph.assign(size_t(m), nullptr);
  if (c.use_graph) MG_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

}  // namespace


// ---------------------------------------------------------------- batched handle
struct BLaunch {
  int kind = 0;
  size_t e0 = 0;     // first entry in the batch's entry table
  int ne = 0, nb = 0;
  int depth = -1;    // levels below each problem's finest level (-1: outer-loop launch)
  int kb = 0;        // slot batch of the slice kernels (0: default)
};

struct mg_batch : DevOwner {
  mg_config cfg{};
  int NR = 1, P = 0, B = 1, xk = X_F64, vkind = VK_F64, n_inst = 0, Dmax = 0;
  struct Prob {
    int L = 0;
    std::vector<LevelDev> lv;
    double* Ainv = nullptr;
    int n0 = 0;
  };
  std::vector<Prob> pr;
  std::vector<int64_t> off;           // P + 1 element offsets in the concatenated vectors
  int64_t Ntot = 0;
  void *btop = nullptr, *ttop = nullptr, *rtop = nullptr;   // top-level cycle vectors
  double *V = nullptr, *rout = nullptr;
  void* Z = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *yv = nullptr, *st = nullptr;
  double *beta = nullptr, *bnorm = nullptr, *tolv = nullptr;
  int *kk = nullptr, *iact = nullptr;
  int* pact = nullptr;                // problem has an unconverged instance
  int* pstep = nullptr;               // problem has an instance whose Krylov cycle is still open
  double* pvec[2] = {nullptr, nullptr};
  double* pbig = nullptr;
  BSegs segs, segs_act, segs_step;   // vector segments: all problems / pact / pstep
  int *bigfirst = nullptr, *bigcount = nullptr;
  std::vector<BEntry> hE;             // entry tables of every planned launch
  BEntry* dE = nullptr;
  BEntry* dEdef = nullptr;            // outer-defect entries (rebuilt per solve for b, x)
  std::vector<std::vector<BLaunch>> plan;   // per Krylov index: V-cycle launches
  std::vector<BLaunch> spmv64;        // per Krylov index: w = A z_j
  int nbig = 0;                       // blocks of the outer FP64 products
  int kb64 = 0;                       // slot batch of the outer FP64 products
  bool c16 = false;                   // all operators carry 16-bit column differences
  hipStream_t cap = nullptr;
  std::vector<hipGraphExec_t> graphs;
  int* hkk = nullptr;                 // pinned host copy of kk (read after every step)
  ~mg_batch() {
    for (hipGraphExec_t gx : graphs)
      if (gx) (void)hipGraphExecDestroy(gx);
    if (cap) (void)hipStreamDestroy(cap);
    if (hkk) (void)hipHostFree(hkk);
  }
};

namespace {

// append one launch (entries already filled except `first`) to the batch plan
BLaunch add_launch(mg_batch* h, int kind, std::vector<BEntry>& es, int depth = -1) {
  BLaunch L;
  L.kind = kind;
  L.depth = depth;
  L.e0 = h->hE.size();
  int first = 0;
  for (BEntry& e : es) {
    e.first = first;
    first += batched_blocks(kind, e.A, e.Ts, e.n0, h->NR);
    h->hE.push_back(e);
  }
  L.ne = int(es.size());
  L.nb = first;
  return L;
}

// static launch plan of one V-cycle of every problem for Krylov index j: the top level of
// problem p reads its right-hand side from the cycle copy of v_j and writes z_j
void build_plan(mg_batch* h, int j, std::vector<BLaunch>& out) {
  const mg_config& c = h->cfg;
  const int pre_pp = c.nu1 >= 1 ? c.nu1 - 1 : 0;
  const int pp = pre_pp + c.nu2;
  const size_t xs = xsize(h->xk);
  auto top_x = [&](int p) { return static_cast<char*>(h->Z) + (size_t(j) * h->Ntot + h->off[p]) * xs; };
  auto top_b = [&](int p) -> void* {
    if (h->xk == X_F64) return reinterpret_cast<char*>(h->V + int64_t(j) * h->Ntot + h->off[p]);
    return static_cast<char*>(h->btop) + size_t(h->off[p]) * xs;
  };
  const int P = h->P;
  std::vector<std::vector<void*>> own(P), tmp(P), bb(P), rr(P), cur(P), oth(P);
  for (int p = 0; p < P; ++p) {
    const int L = h->pr[p].L;
    own[p].resize(L + 1);
    tmp[p].resize(L + 1);
    bb[p].resize(L + 1);
    rr[p].resize(L + 1);
    cur[p].resize(L + 1);
    oth[p].resize(L + 1);
    for (int l = 0; l <= L; ++l) {
      const LevelDev& D = h->pr[p].lv[l];
      own[p][l] = (l == L) ? static_cast<void*>(top_x(p)) : D.x;
      tmp[p][l] = (l == L) ? static_cast<char*>(h->ttop) + size_t(h->off[p]) * xs : static_cast<char*>(D.t);
      bb[p][l] = (l == L) ? top_b(p) : D.b;
      rr[p][l] = (l == L) ? static_cast<char*>(h->rtop) + size_t(h->off[p]) * xs : static_cast<char*>(D.r);
      cur[p][l] = (pp % 2 == 0) ? own[p][l] : tmp[p][l];
      oth[p][l] = (pp % 2 == 0) ? tmp[p][l] : own[p][l];
    }
  }
  auto level_entry = [&](int p, int l) {
    const LevelDev& D = h->pr[p].lv[l];
    BEntry e;
    e.A = D.Ac;
    e.S = D.S;
    e.mask = D.mask;
    e.prob = p;
    return e;
  };
  // descent, aligned by depth below each problem's finest level
  for (int d = 0; d < h->Dmax; ++d) {
    std::vector<int> ps;
    for (int p = 0; p < P; ++p)
      if (h->pr[p].L - d >= 1) ps.push_back(p);
    if (ps.empty()) continue;
    std::vector<BEntry> es;
    if (c.nu1 >= 1) {
      es.clear();
      for (int p : ps) {
        const int l = h->pr[p].L - d;
        BEntry e = level_entry(p, l);
        e.in0 = bb[p][l];
        e.out = cur[p][l];
        es.push_back(e);
      }
      out.push_back(add_launch(h, BK_SWEEP0, es, d));
      for (int q = 1; q < c.nu1; ++q) {
        es.clear();
        for (int p : ps) {
          const int l = h->pr[p].L - d;
          BEntry e = level_entry(p, l);
          e.in0 = bb[p][l];
          e.in1 = cur[p][l];
          e.out = oth[p][l];
          es.push_back(e);
          std::swap(cur[p][l], oth[p][l]);
        }
        out.push_back(add_launch(h, BK_SWEEP, es, d));
      }
    } else {
      es.clear();
      for (int p : ps) {
        const int l = h->pr[p].L - d;
        BEntry e = level_entry(p, l);
        e.out = cur[p][l];
        es.push_back(e);
      }
      out.push_back(add_launch(h, BK_FILL0, es, d));
    }
    es.clear();
    for (int p : ps) {
      const int l = h->pr[p].L - d;
      BEntry e = level_entry(p, l);
      e.in0 = bb[p][l];
      e.in1 = cur[p][l];
      e.out = rr[p][l];
      es.push_back(e);
    }
    out.push_back(add_launch(h, BK_DEFECT, es, d));
    es.clear();
    for (int p : ps) {
      const int l = h->pr[p].L - d;
      BEntry e = level_entry(p, l);
      e.Ts = h->pr[p].lv[l].Rs;
      e.mask_c = h->pr[p].lv[l - 1].mask;
      e.in0 = rr[p][l];
      e.out = bb[p][l - 1];
      es.push_back(e);
    }
    out.push_back(add_launch(h, BK_RESTRICT, es, d));
  }
  // coarse solves of all problems
  {
    std::vector<BEntry> es;
    for (int p = 0; p < P; ++p) {
      BEntry e = level_entry(p, 0);
      e.Ainv = h->pr[p].Ainv;
      e.n0 = h->pr[p].n0;
      e.in0 = bb[p][0];
      e.out = own[p][0];
      es.push_back(e);
    }
    out.push_back(add_launch(h, BK_COARSE, es));
  }
  // ascent
  for (int d = h->Dmax - 1; d >= 0; --d) {
    std::vector<int> ps;
    for (int p = 0; p < P; ++p)
      if (h->pr[p].L - d >= 1) ps.push_back(p);
    if (ps.empty()) continue;
    // the descent left cur at the pre-smoothed iterate; the coarser level's correction
    // sits in its own x (its post-smoothing ends there)
    std::vector<BEntry> es;
    for (int p : ps) {
      const int l = h->pr[p].L - d;
      BEntry e = level_entry(p, l);
      e.Ts = h->pr[p].lv[l].Ps;
      e.mask_c = h->pr[p].lv[l - 1].mask;
      e.in0 = own[p][l - 1];
      e.out = cur[p][l];
      es.push_back(e);
    }
    out.push_back(add_launch(h, BK_PROLONG, es, d));
    for (int q = 0; q < c.nu2; ++q) {
      es.clear();
      for (int p : ps) {
        const int l = h->pr[p].L - d;
        BEntry e = level_entry(p, l);
        e.in0 = bb[p][l];
        e.in1 = cur[p][l];
        e.out = oth[p][l];
        es.push_back(e);
        std::swap(cur[p][l], oth[p][l]);
      }
      out.push_back(add_launch(h, BK_SWEEP, es, d));
    }
  }
}

int run_launch(mg_batch* h, const BLaunch& L, const BEntry* table, const int* active, double* partials, hipStream_t s) {
  int kb = L.kb;
  if (h->c16) {                       // every operator of the batch has 16-bit columns
    int kd, ko;
    slot_batch_choices(h->B, &kd, &ko);
    kb = -(kb ? kb : kd);
  }
  MG_HIP(launch_batched(L.kind, table + L.e0, L.ne, L.nb, h->B, h->NR, h->vkind, h->xk, h->cfg.omega, active,
                        partials, kb, s));
  return MG_OK;
}

// Slot-batch choice for the batch: per depth, both built sizes of that depth's sweep launch
// are timed (3 interleaved repetitions of 5 launches, minimum kept) and the faster is used
// by every sweep and defect launch of that depth; the outer FP64 products likewise with
// the first SpMV launch.  Bitwise-neutral like the single-problem tuner.
int tune_batch(mg_batch* h, hipStream_t s) {
  int kb[2];
  slot_batch_choices(h->B, &kb[0], &kb[1]);
  const int req = h->cfg.slot_batch;
  if (req != 0 && req != kb[0] && req != kb[1])
    return fail(MG_EINVAL, "slot_batch must be 0 or one of the two batch sizes built for this block size");
  auto apply = [&](auto&& pred, int v) {
    for (auto& pl : h->plan)
      for (BLaunch& L : pl)
        if (pred(L)) L.kb = v;
    for (BLaunch& L : h->spmv64)
      if (pred(L)) L.kb = v;
  };
  auto level_kind = [](const BLaunch& L, int d) {
    return L.depth == d && (L.kind == BK_SWEEP || L.kind == BK_DEFECT);
  };
  if (req != 0) {
    for (int d = 0; d < h->Dmax; ++d) apply([&](const BLaunch& L) { return level_kind(L, d); }, req);
    apply([](const BLaunch& L) { return L.kind == BK_SPMV64; }, req);
    h->kb64 = req;
    return MG_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  int rc = MG_OK;
  auto best_of = [&](BLaunch L, int* pick) -> int {
    float best[2] = {1e30f, 1e30f};
    for (int rep = 0; rep < 3; ++rep)
      for (int v = 0; v < 2; ++v) {
        L.kb = kb[v];
        MG_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < 5; ++i) {
          const int r = run_launch(h, L, h->dE, nullptr, nullptr, s);
          if (r) return r;
        }
        MG_HIP(hipEventRecord(e1, s));
        MG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        MG_HIP(hipEventElapsedTime(&ms, e0, e1));
        best[v] = std::min(best[v], ms);
      }
    *pick = best[1] < best[0] ? kb[1] : kb[0];
    return MG_OK;
  };
  for (int d = 0; d < h->Dmax && rc == MG_OK; ++d) {
    const BLaunch* probe = nullptr;
    for (const BLaunch& L : h->plan[0])
      if (L.depth == d && L.kind == BK_SWEEP) { probe = &L; break; }
    if (!probe) continue;
    int pick = kb[0];
    if ((rc = best_of(*probe, &pick))) break;
    apply([&](const BLaunch& L) { return level_kind(L, d); }, pick);
  }
  if (rc == MG_OK && !h->spmv64.empty()) {
    int pick = kb[0];
    if ((rc = best_of(h->spmv64[0], &pick)) == MG_OK) {
      apply([](const BLaunch& L) { return L.kind == BK_SPMV64; }, pick);
      h->kb64 = pick;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// one lockstep FGMRES step j for every instance
int enqueue_batch_step(mg_batch* h, int j, hipStream_t s) {
  const int m = h->cfg.gmres_m;
  const int64_t N = h->Ntot;
  int rc;
  // the cycle-precision copy of v_j (btop) was written by the kernel that produced v_j
  for (const BLaunch& L : h->plan[j])
    if ((rc = run_launch(h, L, h->dE, h->pstep, nullptr, s))) return rc;
  // w = A z_j.  (The first Gram-Schmidt dot is a separate pass here: the SpMV's blocks are
  // far more numerous than the vector blocks, and re-summing their partials per block of
  // the first step would cost more than the pass.)
  if ((rc = run_launch(h, h->spmv64[j], h->dE, h->pstep, nullptr, s))) return rc;
  double* w = h->V + int64_t(j + 1) * N;
  const int64_t hs = int64_t(m + 1) * m;
  double* Hj = h->H + int64_t(j) * (m + 1);
  const BSegs& sg = h->segs_step;
  MG_HIP(launch_bdot(sg, w, h->V, h->pvec[0], s));
  for (int i = 0; i <= j; ++i) {
    const double* vi = h->V + int64_t(i) * N;
    const double* vn = (i < j) ? h->V + int64_t(i + 1) * N : nullptr;
    MG_HIP(launch_bmgs_step(sg, w, vi, vn, h->pvec[i & 1], h->pvec[(i + 1) & 1], Hj + i, hs, s));
  }
  float* wc = h->xk == X_F64 ? nullptr : static_cast<float*>(h->btop);
  MG_HIP(launch_bmgs_normalize(sg, w, h->pvec[(j + 1) & 1], Hj + j + 1, hs, s, wc));
  MG_HIP(launch_bgivens(j, m, h->n_inst, h->H, h->cs, h->sn, h->g, h->st, h->tolv, h->kk, h->iact, s));
  return MG_OK;
}

int batch_step(mg_batch* h, int j, hipStream_t s) {
  if (!h->cfg.use_graph) return enqueue_batch_step(h, j, s);
  if (!h->graphs[j]) {
    hipGraph_t gr = nullptr;
    MG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch_step(h, j, h->cap);
    const hipError_t e = hipStreamEndCapture(h->cap, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return fail(MG_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e2 != hipSuccess) return fail(MG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    h->graphs[j] = ex;
  }
  MG_HIP(hipGraphLaunch(h->graphs[j], s));
  return MG_OK;
}

// beta = ||b - A x|| per instance of the active problems (r stored in rout)
int batch_defect(mg_batch* h, hipStream_t s) {
  BLaunch L;
  L.kind = BK_DEFECT64;
  L.e0 = 0;
  L.ne = h->P;
  L.nb = h->nbig;
  L.kb = h->kb64;
  int rc;
  if ((rc = run_launch(h, L, h->dEdef, h->pact, h->pbig, s))) return rc;
  MG_HIP(launch_bfinish(h->pbig, h->bigfirst, h->bigcount, h->n_inst, h->NR, h->beta, 1, s));
  return MG_OK;
}

int setup_batch(mg_batch* h, const std::vector<std::vector<HostLevel>>& HH, hipStream_t s) {
  const mg_config& c = h->cfg;
  const int P = h->P, NR = h->NR;
  int rc;
  int* flag;
  if ((rc = dalloc(h, &flag, 1))) return rc;
  MG_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  h->pr.resize(P);
  h->off.assign(size_t(P) + 1, 0);
  for (int p = 0; p < P; ++p) {
    const auto& H = HH[p];
    auto& pr = h->pr[p];
    pr.L = int(H.size()) - 1;
    h->Dmax = std::max(h->Dmax, pr.L);
    pr.lv.resize(H.size());
    for (int l = 0; l <= pr.L; ++l)
      if ((rc = setup_level(h, H[l], l > 0, NR, h->vkind, h->xk, l < pr.L, flag, s, pr.lv[l]))) return rc;
    if ((rc = setup_coarse_inverse(h, H[0], flag, s, &pr.Ainv, &pr.n0))) return rc;
    h->off[p + 1] = h->off[p] + pr.lv[pr.L].N * NR;
  }
  if ((rc = check_flag(flag, s))) return rc;
  h->c16 = true;
  for (const auto& pr : h->pr)
    for (const LevelDev& D : pr.lv) h->c16 = h->c16 && D.Ac.col16 && D.A64.col16;
  // one launch streams the operators of every problem: they stay in the memory-side cache
  // only if the whole batch's do, so the load kind of the transfers follows the batch
  // total (the batched slice kernels always read their operators non-temporally)
  {
    // value lanes per slot: B * W with the row-lane stride W = kWave / NR of the batch
    const int64_t W = kWave / NR;
    auto sbytes = [W](const SellDev& A) {
      const int vb = A.kind == VK_F64 ? 8 : A.kind == VK_F32 ? 4 : 2;
      return A.slots * (int64_t(A.B) * W * vb + int64_t(A.R) * (A.col16 ? 2 : 4));
    };
    int64_t tot = 0;
    for (const auto& pr : h->pr)
      for (const LevelDev& D : pr.lv) tot += sbytes(D.Ac) + (D.A64.val != D.Ac.val ? sbytes(D.A64) : 0);
    const int nt = stream_nt(tot);
    for (auto& pr : h->pr)
      for (LevelDev& D : pr.lv) D.Ps.nt = D.Rs.nt = nt;
  }
  const int64_t N = h->Ntot = h->off[P];
  const int m = c.gmres_m;
  const size_t xs = xsize(h->xk);
  char* p8;
  for (void** v : {&h->btop, &h->ttop, &h->rtop}) {
    if ((rc = dalloc(h, &p8, size_t(N) * xs))) return rc;
    *v = p8;
  }
  if ((rc = dalloc(h, &h->V, size_t(m + 1) * N))) return rc;
  if ((rc = dalloc(h, &h->rout, size_t(N)))) return rc;
  if ((rc = dalloc(h, &p8, size_t(m) * N * xs))) return rc;
  h->Z = p8;
  const int ni = h->n_inst = P * NR;
  if ((rc = dalloc(h, &h->H, size_t(ni) * (m + 1) * m))) return rc;
  if ((rc = dalloc(h, &h->cs, size_t(ni) * m))) return rc;
  if ((rc = dalloc(h, &h->sn, size_t(ni) * m))) return rc;
  if ((rc = dalloc(h, &h->g, size_t(ni) * (m + 1)))) return rc;
  if ((rc = dalloc(h, &h->yv, size_t(ni) * m))) return rc;
  if ((rc = dalloc(h, &h->st, size_t(ni) * 2))) return rc;
  if ((rc = dalloc(h, &h->beta, size_t(ni)))) return rc;
  if ((rc = dalloc(h, &h->bnorm, size_t(ni)))) return rc;
  if ((rc = dalloc(h, &h->tolv, size_t(ni)))) return rc;
  if ((rc = dalloc(h, &h->kk, size_t(ni)))) return rc;
  if ((rc = dalloc(h, &h->iact, size_t(ni)))) return rc;
  if ((rc = dalloc(h, &h->pact, size_t(P)))) return rc;
  if ((rc = dalloc(h, &h->pstep, size_t(P)))) return rc;
  // vector segments: up to kSegBlocksMax blocks per problem
  std::vector<int64_t> len(P);
  std::vector<int> vfirst(P), vcount(P), blk;
  for (int p = 0; p < P; ++p) {
    len[p] = h->off[p + 1] - h->off[p];
    vfirst[p] = int(blk.size());
    vcount[p] = int(std::min<int64_t>(kSegBlocksMax, std::max<int64_t>(1, (len[p] + 1023) / 1024)));
    for (int b = 0; b < vcount[p]; ++b) blk.push_back(p);
  }
  int64_t *doff, *dlen;
  int *dvf, *dvc, *dblk;
  std::vector<int64_t> offv(h->off.begin(), h->off.end() - 1);
  if ((rc = upload(h, &doff, offv, s))) return rc;
  if ((rc = upload(h, &dlen, len, s))) return rc;
  if ((rc = upload(h, &dvf, vfirst, s))) return rc;
  if ((rc = upload(h, &dvc, vcount, s))) return rc;
  if ((rc = upload(h, &dblk, blk, s))) return rc;
  h->segs.off = doff;
  h->segs.len = dlen;
  h->segs.vfirst = dvf;
  h->segs.vcount = dvc;
  h->segs.blk_prob = dblk;
  h->segs.n_blocks = int(blk.size());
  h->segs.NR = NR;
  h->segs_act = h->segs;
  h->segs_act.on = h->pact;
  h->segs_step = h->segs;
  h->segs_step.on = h->pstep;
  for (int q = 0; q < 2; ++q)
    if ((rc = dalloc(h, &h->pvec[q], blk.size() * NR))) return rc;
  // outer FP64 products: blocks per problem
  std::vector<int> bf(P), bc(P);
  int nbig = 0;
  for (int p = 0; p < P; ++p) {
    bf[p] = nbig;
    bc[p] = spmv_grid(h->pr[p].lv[h->pr[p].L].A64);
    nbig += bc[p];
  }
  h->nbig = nbig;
  if ((rc = upload(h, &h->bigfirst, bf, s))) return rc;
  if ((rc = upload(h, &h->bigcount, bc, s))) return rc;
  if ((rc = dalloc(h, &h->pbig, size_t(nbig) * NR))) return rc;
  if ((rc = dalloc(h, &h->dEdef, size_t(P)))) return rc;
  // launch plans
  h->plan.assign(size_t(m), {});
  h->spmv64.assign(size_t(m), BLaunch());
  for (int j = 0; j < m; ++j) {
    build_plan(h, j, h->plan[j]);
    std::vector<BEntry> es;
    for (int p = 0; p < P; ++p) {
      const LevelDev& D = h->pr[p].lv[h->pr[p].L];
      BEntry e;
      e.A = D.A64;
      e.prob = p;
      e.in1 = static_cast<char*>(h->Z) + (size_t(j) * N + h->off[p]) * xs;
      e.out = h->V + int64_t(j + 1) * N + h->off[p];
      es.push_back(e);
    }
    h->spmv64[j] = add_launch(h, BK_SPMV64, es);
  }
  if ((rc = upload(h, &h->dE, h->hE, s))) return rc;
  MG_HIP(hipStreamSynchronize(s));
  if ((rc = tune_batch(h, s))) return rc;
  MG_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hkk), sizeof(int) * ni, hipHostMallocDefault));
  h->graphs.assign(size_t(m), nullptr);
  if (c.use_graph) MG_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

template <class T>
int to_host(T* dst, const T* src, size_t n, hipStream_t s) {
  MG_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

template <class T>
int to_dev(T* dst, const T* src, size_t n, hipStream_t s) {
  MG_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
}

int solve_batch_impl(mg_batch* h, const double* b, double* x, mg_solve_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const mg_config& c = h->cfg;
  const int P = h->P, NR = h->NR, ni = h->n_inst, m = c.gmres_m;
  const int64_t N = h->Ntot;
  int rc;
  // outer-defect entries for this call's b and x
  std::vector<BEntry> es(P);
  int first = 0;
  for (int p = 0; p < P; ++p) {
    const LevelDev& D = h->pr[p].lv[h->pr[p].L];
    es[p].A = D.A64;
    es[p].prob = p;
    es[p].in0 = b + h->off[p];
    es[p].in1 = x + h->off[p];
    es[p].out = h->rout + h->off[p];
    es[p].first = first;
    first += spmv_grid(D.A64);
  }
  if ((rc = to_dev(h->dEdef, es.data(), es.size(), s))) return rc;
  // per-instance ||b|| and tolerances
  MG_HIP(launch_bdot(h->segs, b, nullptr, h->pvec[0], s));
  MG_HIP(launch_bfinish(h->pvec[0], h->segs.vfirst, h->segs.vcount, ni, NR, h->bnorm, 1, s));
  std::vector<double> bn(ni), tol(ni), beta(ni), res0(ni), resf(ni);
  if ((rc = to_host(bn.data(), h->bnorm, ni, s))) return rc;
  for (int i = 0; i < ni; ++i) tol[i] = c.rtol * bn[i];
  if ((rc = to_dev(h->tolv, tol.data(), ni, s))) return rc;
  std::vector<int> iact(ni, 1), pact(P, 1), iters(ni, 0), restarts(ni, 0), conv(ni, 0), status(ni, MG_OK), kk(ni);
  if ((rc = to_dev(h->pact, pact.data(), P, s))) return rc;
  if ((rc = batch_defect(h, s))) return rc;
  if ((rc = to_host(beta.data(), h->beta, ni, s))) return rc;
  for (int i = 0; i < ni; ++i) {
    res0[i] = resf[i] = beta[i];
    if (!std::isfinite(beta[i])) { status[i] = MG_ENUMERIC; iact[i] = 0; }
    else if (beta[i] <= tol[i]) { conv[i] = 1; iact[i] = 0; }
  }
  for (int i = 0; i < ni; ++i)
    if (iact[i] && c.maxit <= 0) iact[i] = 0;
  while (true) {
    bool any = false;
    for (int p = 0; p < P; ++p) {
      pact[p] = 0;
      for (int q = 0; q < NR; ++q) pact[p] |= iact[p * NR + q];
      any = any || pact[p];
    }
    if (!any) break;
    if ((rc = to_dev(h->iact, iact.data(), ni, s))) return rc;
    if ((rc = to_dev(h->pact, pact.data(), P, s))) return rc;
    std::vector<int> pstep(pact);
    if ((rc = to_dev(h->pstep, pstep.data(), P, s))) return rc;
    MG_HIP(launch_bscale(h->segs_act, h->V, h->rout, h->beta, h->iact, s,
                         h->xk == X_F64 ? nullptr : static_cast<float*>(h->btop)));
    MG_HIP(launch_binit(m, ni, h->g, h->beta, h->kk, s));
    int jl = 0;
    for (int j = 0; j < m; ++j) {
      if ((rc = batch_step(h, j, s))) return rc;
      jl = j;
      if ((rc = to_host(h->hkk, h->kk, ni, s))) return rc;
      // an instance whose V-cycle budget ends here closes its cycle like the single solve
      bool dirty = false;
      for (int i = 0; i < ni; ++i)
        if (iact[i] && h->hkk[i] == 0 && iters[i] + j + 1 >= c.maxit) {
          h->hkk[i] = j + 1;
          dirty = true;
        }
      if (dirty && (rc = to_dev(h->kk, h->hkk, ni, s))) return rc;
      // problems whose instances have all closed their cycles wait for the restart
      bool open = false, changed = false;
      for (int p = 0; p < P; ++p) {
        int o = 0;
        for (int q = 0; q < NR; ++q) o |= iact[p * NR + q] && h->hkk[p * NR + q] == 0;
        changed = changed || (o != pstep[p]);
        pstep[p] = o;
        open = open || o;
      }
      if (!open) break;
      if (changed && (rc = to_dev(h->pstep, pstep.data(), P, s))) return rc;
    }
    MG_HIP(launch_bclose(jl, ni, h->kk, h->iact, s));
    MG_HIP(launch_bbacksolve(m, ni, h->H, h->g, h->yv, h->kk, s));
    MG_HIP(launch_bupdate(h->segs_act, x, h->Z, h->xk, N, h->yv, m, h->kk, s));
    if ((rc = to_host(kk.data(), h->kk, ni, s))) return rc;
    if ((rc = batch_defect(h, s))) return rc;
    if ((rc = to_host(beta.data(), h->beta, ni, s))) return rc;
    for (int i = 0; i < ni; ++i) {
      if (!iact[i]) continue;
      iters[i] += kk[i];
      restarts[i] += 1;
      resf[i] = beta[i];
      if (!std::isfinite(beta[i]) || beta[i] > 1e6 * std::max(res0[i], 1e-300)) {
        status[i] = MG_ENUMERIC;
        iact[i] = 0;
      } else if (beta[i] <= tol[i]) {
        conv[i] = 1;
        iact[i] = 0;
      } else if (iters[i] >= c.maxit) {
        iact[i] = 0;
      }
    }
  }
  MG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int worst = MG_OK;
  for (int i = 0; i < ni; ++i) {
    if (status[i] == MG_OK && !conv[i]) status[i] = MG_ENOCONV;
    if (status[i] == MG_ENUMERIC) worst = MG_ENUMERIC;
    else if (status[i] == MG_ENOCONV && worst == MG_OK) worst = MG_ENOCONV;
    if (st) {
      st[i].iters = iters[i];
      st[i].restarts = restarts[i];
      st[i].status = status[i];
      st[i].converged = conv[i];
      st[i].res0 = res0[i];
      st[i].res_final = resf[i];
      st[i].t_solve_ms = ms;
    }
  }
  if (worst == MG_ENUMERIC) return fail(MG_ENUMERIC, "non-finite or diverging residual in a batch instance");
  if (worst == MG_ENOCONV) return fail(MG_ENOCONV, "maxit reached before rtol in a batch instance");
  return MG_OK;
}

// Device address of `scratch` on the current device, taken once per device.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch_addr[kMaxDevices] = {};

int scratch_address(double** out) {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MG_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(MG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return MG_OK;
}

// ---------------------------------------------------------------- time stepping
// Right-hand-side operator R, interpolation H and Dirichlet positions of a
// backward-Euler run (Algorithm "Nonstationary Linear Problem"), on the device.
struct TimeDev : DevOwner {
  mg_handle* h = nullptr;
  int32_t n = 0, n_g = 0;
  double dt = 1.0;
  const int32_t *rrow = nullptr, *rcol = nullptr, *hrow = nullptr, *hcol = nullptr, *gpos = nullptr;
  const double *rval = nullptr, *hval = nullptr;
  double* b = nullptr;   // right-hand side of the current step
};

// CSR with `rows` rows over `cols` columns: monotone row pointers from 0, indices in range
int check_csr(const int32_t* rowptr, const int32_t* col, const double* val, int32_t rows, int64_t cols,
              const char* what) {
  if (!rowptr || (rowptr[rows] > 0 && (!col || !val))) return fail(MG_EINVAL, std::string(what) + ": null array");
  if (rowptr[0] != 0) return fail(MG_EINVAL, std::string(what) + ": row pointers must start at 0");
  for (int32_t i = 0; i < rows; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(MG_EINVAL, std::string(what) + ": decreasing row pointers");
  for (int32_t k = 0; k < rowptr[rows]; ++k) {
    if (col[k] < 0 || col[k] >= cols) return fail(MG_EINVAL, std::string(what) + ": column out of range");
    if (!std::isfinite(val[k])) return fail(MG_EINVAL, std::string(what) + ": non-finite value");
  }
  return MG_OK;
}

int time_setup(TimeDev* t, const int32_t* R_rowptr, const int32_t* R_col, const double* R_val,
               const int32_t* H_rowptr, const int32_t* H_col, const double* H_val, const int32_t* g_idx,
               hipStream_t s) {
  const int32_t n = t->n, ng = t->n_g;
  int rc;
  if ((rc = check_csr(R_rowptr, R_col, R_val, n, int64_t(n) + ng, "R"))) return rc;
  if ((rc = check_csr(H_rowptr, H_col, H_val, n, n, "H"))) return rc;
  std::vector<int32_t> gpos(size_t(n), -1);
  for (int32_t k = 0; k < ng; ++k) {
    const int32_t d = g_idx[k];
    if (d < 0 || d >= n) return fail(MG_EINVAL, "Dirichlet DoF out of range");
    if (gpos[size_t(d)] >= 0) return fail(MG_EINVAL, "duplicate Dirichlet DoF");
    gpos[size_t(d)] = k;
  }
  const size_t rnnz = size_t(R_rowptr[n]), hnnz = size_t(H_rowptr[n]);
  std::vector<int32_t> rr(R_rowptr, R_rowptr + n + 1), rc_(R_col, R_col + rnnz);
  std::vector<double> rv(R_val, R_val + rnnz);
  std::vector<int32_t> hr(H_rowptr, H_rowptr + n + 1), hc(H_col, H_col + hnnz);
  std::vector<double> hv(H_val, H_val + hnnz);
  int32_t *p32;
  double* p64;
  if ((rc = upload(t, &p32, rr, s))) return rc;
  t->rrow = p32;
  if ((rc = upload(t, &p32, rc_, s))) return rc;
  t->rcol = p32;
  if ((rc = upload(t, &p64, rv, s))) return rc;
  t->rval = p64;
  if ((rc = upload(t, &p32, hr, s))) return rc;
  t->hrow = p32;
  if ((rc = upload(t, &p32, hc, s))) return rc;
  t->hcol = p32;
  if ((rc = upload(t, &p64, hv, s))) return rc;
  t->hval = p64;
  if ((rc = upload(t, &p32, gpos, s))) return rc;
  t->gpos = p32;
  if ((rc = dalloc(t, &t->b, size_t(n)))) return rc;
  MG_HIP(hipStreamSynchronize(s));   // the host vectors above are freed on return
  return MG_OK;
}

// ---------------------------------------------------------------- pressure correction
// Matrices and work vectors of the explicit pressure-correction step on the device.
struct NsDev : DevOwner {
  mg_handle* hp = nullptr;      // pressure Poisson hierarchy (caller-owned)
  int32_t n_v = 0, n_p = 0;
  double nu = 0.0, dt = 1.0;
  NsEll V, G, D;
  const double *m_v = nullptr, *m_p = nullptr, *dval = nullptr;
  const uint8_t* dmask = nullptr;
  double *ubuf = nullptr, *du = nullptr, *rhs = nullptr;
};

// sliced ELL of `nval` value arrays on one CSR pattern (rows x cols), see NsEll
int upload_ns_ell(DevOwner* h, int32_t rows, const int32_t* rowptr, const int32_t* col, const double* const* vals,
                  int nval, NsEll& E, hipStream_t s) {
  const int64_t nsl = (int64_t(rows) + kWave - 1) / kWave;
  std::vector<int32_t> sptr(size_t(nsl) + 1, 0);
  for (int64_t sl = 0; sl < nsl; ++sl) {
    int32_t w = 0;
    for (int64_t r = sl * kWave; r < std::min<int64_t>(rows, (sl + 1) * kWave); ++r)
      w = std::max(w, rowptr[r + 1] - rowptr[r]);
    if (int64_t(sptr[size_t(sl)]) + w > INT32_MAX) return fail(MG_EUNSUPPORTED, "matrix too large for 32-bit slot offsets");
    sptr[size_t(sl) + 1] = sptr[size_t(sl)] + w;
  }
  const int64_t slots = sptr.back();
  std::vector<int32_t> ce(size_t(slots) * kWave, 0);
  std::vector<double> ve(size_t(slots) * kWave * size_t(nval), 0.0);
  for (int64_t sl = 0; sl < nsl; ++sl)
    for (int lane = 0; lane < kWave; ++lane) {
      const int64_t r = sl * kWave + lane;
      if (r >= rows) continue;
      const int32_t b0 = rowptr[r], len = rowptr[r + 1] - b0;
      for (int32_t t = 0; t < sptr[size_t(sl) + 1] - sptr[size_t(sl)]; ++t) {
        const int64_t slot = int64_t(sptr[size_t(sl)]) + t;
        const size_t e = size_t(slot) * kWave + size_t(lane);
        if (t < len) {
          ce[e] = col[b0 + t];
          for (int v = 0; v < nval; ++v) ve[(size_t(slot) * size_t(nval) + size_t(v)) * kWave + size_t(lane)] = vals[v][b0 + t];
        } else {
          ce[e] = len > 0 ? col[b0 + len - 1] : 0;   // a valid column with weight 0
        }
      }
    }
  int32_t *ps, *pc;
  double* pv;
  int rc;
  if ((rc = upload(h, &ps, sptr, s)) || (rc = upload(h, &pc, ce, s)) || (rc = upload(h, &pv, ve, s))) return rc;
  MG_HIP(hipStreamSynchronize(s));   // the host vectors are freed on return
  E.nrows = rows;
  E.nslices = nsl;
  E.sptr = ps;
  E.col = pc;
  E.val = pv;
  return MG_OK;
}

template <class T>
int upload_array(DevOwner* h, const T** out, const T* src, size_t n, hipStream_t s) {
  std::vector<T> v(src, src + n);
  T* p;
  int rc = upload(h, &p, v, s);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(s));
  *out = p;
  return MG_OK;
}

int ns_setup(NsDev* t, const mg_ns_in& in, hipStream_t s) {
  int rc;
  const int32_t nv = in.n_v, np = in.n_p;
  for (int a = 0; a < 3; ++a) {
    if ((rc = check_csr(in.V_rowptr, in.V_col, in.C_val[a], nv, nv, "C"))) return rc;
    if ((rc = check_csr(in.G_rowptr, in.G_col, in.G_val[a], nv, np, "G"))) return rc;
    if ((rc = check_csr(in.D_rowptr, in.D_col, in.D_val[a], np, nv, "D"))) return rc;
  }
  if ((rc = check_csr(in.V_rowptr, in.V_col, in.K_val, nv, nv, "K"))) return rc;
  for (int32_t i = 0; i < nv; ++i)
    if (!(in.m_v[i] > 0.0) || !std::isfinite(in.m_v[i])) return fail(MG_EINVAL, "velocity lumped mass must be positive");
  for (int32_t i = 0; i < np; ++i)
    if (!(in.m_p[i] > 0.0) || !std::isfinite(in.m_p[i])) return fail(MG_EINVAL, "pressure lumped mass must be positive");
  for (int64_t i = 0; i < int64_t(nv) * 3; ++i)
    if (!std::isfinite(in.dir_val[i])) return fail(MG_EINVAL, "non-finite Dirichlet value");
  const double* vv[4] = {in.K_val, in.C_val[0], in.C_val[1], in.C_val[2]};
  if ((rc = upload_ns_ell(t, nv, in.V_rowptr, in.V_col, vv, 4, t->V, s))) return rc;
  if ((rc = upload_ns_ell(t, nv, in.G_rowptr, in.G_col, in.G_val, 3, t->G, s))) return rc;
  if ((rc = upload_ns_ell(t, np, in.D_rowptr, in.D_col, in.D_val, 3, t->D, s))) return rc;
  if ((rc = upload_array(t, &t->m_v, in.m_v, size_t(nv), s))) return rc;
  if ((rc = upload_array(t, &t->m_p, in.m_p, size_t(np), s))) return rc;
  if ((rc = upload_array(t, &t->dmask, in.dir_mask, size_t(nv) * 3, s))) return rc;
  if ((rc = upload_array(t, &t->dval, in.dir_val, size_t(nv) * 3, s))) return rc;
  if ((rc = dalloc(t, &t->ubuf, size_t(nv) * 3))) return rc;
  if ((rc = dalloc(t, &t->du, size_t(np)))) return rc;
  if ((rc = dalloc(t, &t->rhs, size_t(np)))) return rc;
  return MG_OK;
}

// ---------------------------------------------------------------- GPU assembly
// Contribution lists of the assembly: for every stored block, the (cell size class,
// corner a, corner b, hanging weight) of every element entry that reaches it through H.
struct AsmDev : DevOwner {
  int dim = 2, B = 1, nd = 0;
  int64_t nnzb = 0;
  const int32_t *brow = nullptr, *bcol = nullptr;
  const uint32_t* cptr = nullptr;
  const uint16_t* code = nullptr;
  const double* sizes = nullptr;
  const uint8_t* mask = nullptr;
  double* table = nullptr;
};

// exponent e with w = 2^-e (0 <= e <= 7), or -1
int dyadic_exponent(double w) {
  for (int e = 0; e <= 7; ++e)
    if (w == std::ldexp(1.0, -e)) return e;
  return -1;
}

int asm_setup(AsmDev* A, const mg_asm_in& in, hipStream_t s) {
  const int dim = in.dim, B = in.block, nb = 1 << dim;
  const int32_t n = in.n_nodes;
  // cell size classes
  std::vector<double> sizes(in.cell_size, in.cell_size + in.n_cells);
  for (double v : sizes)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(MG_EINVAL, "cell sizes must be positive");
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  if (sizes.size() > 32) return fail(MG_EUNSUPPORTED, "more than 32 distinct cell sizes");
  // node expansions through H: (node, weight exponent)
  std::vector<int32_t> hslot(size_t(n), -1);
  for (int32_t h = 0; h < in.n_hanging; ++h) {
    const int32_t v = in.hang_node[h];
    if (v < 0 || v >= n || hslot[size_t(v)] >= 0) return fail(MG_EINVAL, "bad or repeated hanging node");
    hslot[size_t(v)] = h;
    for (int q = 0; q < 4; ++q) {
      const int32_t m = in.hang_master[4 * h + q];
      if (m < 0) continue;
      if (m >= n) return fail(MG_EINVAL, "hanging master out of range");
      if (dyadic_exponent(in.hang_weight[4 * h + q]) < 0) return fail(MG_EUNSUPPORTED, "hanging weights must be 2^-e, e <= 7");
    }
  }
  auto expand = [&](int32_t v, int32_t* node, int* ex) {
    const int32_t h = hslot[size_t(v)];
    if (h < 0) {
      node[0] = v;
      ex[0] = 0;
      return 1;
    }
    int c = 0;
    for (int q = 0; q < 4; ++q) {
      const int32_t m = in.hang_master[4 * h + q];
      if (m < 0) continue;
      node[c] = m;
      ex[c] = dyadic_exponent(in.hang_weight[4 * h + q]);
      ++c;
    }
    return c;
  };
  auto row_free = [&](int32_t i) {
    for (int c = 0; c < B; ++c)
      if (!in.dof_mask[size_t(i) * B + c]) return true;
    return false;
  };
  // pattern checks
  if (in.A_rowptr[0] != 0 || int64_t(in.A_rowptr[n]) != in.nnzb) return fail(MG_EINVAL, "bad row pointers");
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = in.A_rowptr[i]; k < in.A_rowptr[i + 1]; ++k)
      if (in.A_col[k] < 0 || in.A_col[k] >= n || (k > in.A_rowptr[i] && in.A_col[k] <= in.A_col[k - 1]))
        return fail(MG_EINVAL, "columns must be in range, sorted and unique");
  // contributions, cell by cell, counted per block then placed (stable)
  std::vector<std::pair<int64_t, uint16_t>> contrib;
  for (int32_t e = 0; e < in.n_cells; ++e) {
    const int d = int(std::lower_bound(sizes.begin(), sizes.end(), in.cell_size[e]) - sizes.begin());
    for (int a = 0; a < nb; ++a) {
      const int32_t va = in.cell_corner[size_t(e) * nb + a];
      if (va < 0 || va >= n) return fail(MG_EINVAL, "cell corner out of range");
      int32_t na[4];
      int xa[4];
      const int ca = expand(va, na, xa);
      for (int b = 0; b < nb; ++b) {
        const int32_t vb = in.cell_corner[size_t(e) * nb + b];
        if (vb < 0 || vb >= n) return fail(MG_EINVAL, "cell corner out of range");
        int32_t nbn[4];
        int xb[4];
        const int cb = expand(vb, nbn, xb);
        for (int qa = 0; qa < ca; ++qa) {
          const int32_t i = na[qa];
          if (!row_free(i)) continue;
          const int32_t* r0 = in.A_col + in.A_rowptr[i];
          const int32_t* r1 = in.A_col + in.A_rowptr[i + 1];
          for (int qb = 0; qb < cb; ++qb) {
            const int32_t* it = std::lower_bound(r0, r1, nbn[qb]);
            if (it == r1 || *it != nbn[qb]) continue;   // a constrained column node
            const int ex = xa[qa] + xb[qb];
            if (ex > 7) return fail(MG_EUNSUPPORTED, "hanging weight product below 2^-7");
            contrib.push_back({int64_t(it - in.A_col), uint16_t(d | a << 5 | b << 8 | ex << 11)});
          }
        }
      }
    }
  }
  if (contrib.size() >= (size_t(1) << 32)) return fail(MG_EUNSUPPORTED, "more than 2^32 contributions");
  std::vector<uint32_t> cptr(size_t(in.nnzb) + 1, 0);
  for (const auto& c : contrib) ++cptr[size_t(c.first) + 1];
  for (int64_t k = 0; k < in.nnzb; ++k) cptr[size_t(k) + 1] += cptr[size_t(k)];
  std::vector<uint16_t> code(contrib.size());
  {
    std::vector<uint32_t> fill(cptr.begin(), cptr.end() - 1);
    for (const auto& c : contrib) code[fill[size_t(c.first)]++] = c.second;
  }
  std::vector<int32_t> brow(size_t(in.nnzb)), bcol(in.A_col, in.A_col + in.nnzb);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = in.A_rowptr[i]; k < in.A_rowptr[i + 1]; ++k) brow[size_t(k)] = i;
  std::vector<uint8_t> mask(in.dof_mask, in.dof_mask + size_t(n) * B);
  int rc;
  int32_t *p32;
  uint32_t* pu;
  uint16_t* p16;
  double* pd;
  uint8_t* p8;
  if ((rc = upload(A, &p32, brow, s))) return rc;
  A->brow = p32;
  if ((rc = upload(A, &p32, bcol, s))) return rc;
  A->bcol = p32;
  if ((rc = upload(A, &pu, cptr, s))) return rc;
  A->cptr = pu;
  if ((rc = upload(A, &p16, code, s))) return rc;
  A->code = p16;
  if ((rc = upload(A, &pd, sizes, s))) return rc;
  A->sizes = pd;
  if ((rc = upload(A, &p8, mask, s))) return rc;
  A->mask = p8;
  A->nd = int(sizes.size());
  if ((rc = dalloc(A, &A->table, size_t(A->nd) * nb * nb * B * B))) return rc;
  MG_HIP(hipStreamSynchronize(s));   // the host vectors are freed on return
  A->dim = dim;
  A->B = B;
  A->nnzb = in.nnzb;
  return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

int mg_validate_level(const mg_level_in* lv, const mg_level_in* coarser) {
  if (!lv) return fail(MG_EINVAL, "null level");
  HostLevel L, C;
  int rc = load_level(*lv, false, coarser != nullptr, L);
  if (rc) return rc;
  if (coarser) {
    rc = load_level(*coarser, false, false, C);
    if (rc) return rc;
  }
  return validate_host(L, coarser ? &C : nullptr, coarser ? 1 : 0);
}

int mg_setup_hierarchy(const mg_level_in* lv, int32_t n_levels, const mg_config* cfg, int32_t inputs_on_device,
                       void* stream, mg_handle** out) {
  if (!lv || !cfg || !out || n_levels < 1) return fail(MG_EINVAL, "null argument or no levels");
  *out = nullptr;
  int rc = check_config(*cfg);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<HostLevel> H;
  PhaseTimer pt;
  if ((rc = load_hierarchy(lv, n_levels, inputs_on_device != 0, H))) return rc;
  pt.mark("load and validate");
  mg_handle* h = new (std::nothrow) mg_handle();
  if (!h) return fail(MG_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->L = n_levels - 1;
  h->xk = (cfg->precision == MG_PREC_FP64 || cfg->precision == MG_PREC_FP64_DICT) ? X_F64 : X_F32;
  h->lv.resize(n_levels);
  if (const char* lim = std::getenv("MGQ1_SCRATCH_LIMIT")) h->scratch_cap = std::min(kScratchDoubles, std::max(0, std::atoi(lim)));
  if ((rc = scratch_address(&h->scratch_dev))) {
    delete h;
    return rc;
  }
  try {
    rc = setup_handle(h, H, s);
  } catch (const std::bad_alloc&) {
    rc = fail(MG_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return MG_OK;
}

int mg_vcycle(mg_handle* h, const double* b, double* x, int32_t x_is_zero, void* stream) {
  if (!h || !b || !x) return fail(MG_EINVAL, "null argument");
  if (static_cast<const void*>(b) == static_cast<const void*>(x)) return fail(MG_EINVAL, "x must not alias b");
  const bool xinit = x_is_zero == 0;
  if (xinit && h->L > 0 && h->tail_top == h->L)
    return fail(MG_EUNSUPPORTED, "an initial iterate needs the finest level outside the single-workgroup tail");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->xk == X_F64) return vcycle_cycle(h, b, x, s, xinit);
  const int64_t N = h->lv[h->L].N;
  MG_HIP(launch_convert(N, b, X_F64, h->bcyc, h->xk, s));
  if (xinit) MG_HIP(launch_convert(N, x, X_F64, h->e, h->xk, s));
  int rc = vcycle_cycle(h, h->bcyc, h->e, s, xinit);
  if (rc) return rc;
  MG_HIP(launch_convert(N, h->e, h->xk, x, X_F64, s));
  return MG_OK;
}

int mg_solve(mg_handle* h, const double* b, double* x, mg_solve_stats* st, void* stream) {
  if (!h || !b || !x) return fail(MG_EINVAL, "null argument");
  return solve_impl(h, b, x, st, stream, 0);
}

int mg_solve_fixed(mg_handle* h, const double* b, double* x, int32_t iters, mg_solve_stats* st, void* stream) {
  if (!h || !b || !x || iters < 1) return fail(MG_EINVAL, "null argument or iters < 1");
  return solve_impl(h, b, x, st, stream, iters);
}

int mg_outer_defect(mg_handle* h, const double* b, const double* x, double* r, double* norm, void* stream) {
  if (!h || !b || !x || !r || !norm) return fail(MG_EINVAL, "null argument");
  if (static_cast<const void*>(r) == static_cast<const void*>(x) || static_cast<const void*>(r) == static_cast<const void*>(b))
    return fail(MG_EINVAL, "r must not alias b or x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  LevelDev& T = h->lv[h->L];
  MG_HIP(launch_spmv(T.A64, b, x, r, nullptr, X_F64, X_F64, 1, h->pbig, s));
  MG_HIP(launch_finish(h->pbig, spmv_grid(T.A64), norm, 1, s));
  return MG_OK;
}

int mg_outer_defect_noalloc(mg_handle* h, const double* b, const double* x, double* r, double* norm, void* stream) {
  if (!h || !b || !x || !r || !norm) return fail(MG_EINVAL, "null argument");
  if (static_cast<const void*>(r) == static_cast<const void*>(x) || static_cast<const void*>(r) == static_cast<const void*>(b))
    return fail(MG_EINVAL, "r must not alias b or x");
  LevelDev& T = h->lv[h->L];
  const int g = spmv_grid(T.A64);
  if (g > h->scratch_cap)
    return fail(MG_EUNSUPPORTED, "the finest level needs " + std::to_string(g) + " partial sums; the static scratch array holds " +
                                     std::to_string(h->scratch_cap));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every workgroup writes its own partial and the finish kernel reads exactly g of them,
  // so nothing left in the array by an earlier call is read
  MG_HIP(launch_spmv(T.A64, b, x, r, nullptr, X_F64, X_F64, 1, h->scratch_dev, s));
  MG_HIP(launch_finish(h->scratch_dev, g, norm, 1, s));
  return MG_OK;
}

int mg_level_defect(mg_handle* h, int32_t level, const void* b, const void* x, void* r, int32_t masked,
                    void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (r == x || r == b) return fail(MG_EINVAL, "defect output must not alias its inputs");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_spmv(L.Ac, b, x, r, L.mask, h->xk, h->xk, masked ? 2 : 1, nullptr, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_level_spmv(mg_handle* h, int32_t level, const void* x, void* y, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (x == y) return fail(MG_EINVAL, "product output must not alias its input");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_spmv(L.Ac, nullptr, x, y, nullptr, h->xk, h->xk, 0, nullptr, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_level_sweep(mg_handle* h, int32_t level, const void* b, const void* x, void* x_out, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (x == x_out || b == x_out) return fail(MG_EINVAL, "sweep output must not alias its inputs");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_sweep(L.Ac, L.S, b, x, x_out, h->cfg.omega, h->xk, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_level_sweep0(mg_handle* h, int32_t level, const void* b, void* x_out, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (b == x_out) return fail(MG_EINVAL, "sweep output must not alias its input");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_sweep0(L.Ac, L.S, b, x_out, h->cfg.omega, h->xk, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_level_smooth(mg_handle* h, int32_t level, const void* b, const void* x, void* x_out, int32_t x_is_zero,
                    int32_t sweeps, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (sweeps < 1) return fail(MG_EINVAL, "sweeps must be at least 1");
  if (x_out == b || (!x_is_zero && (x == nullptr || x_out == x))) return fail(MG_EINVAL, "smoother output must not alias its inputs");
  if (chebyshev_on(h, level) && sweeps > int(h->cheb_alpha[size_t(level)].size()))
    return fail(MG_EUNSUPPORTED, "more Chebyshev steps than the configured nu1 / nu2");
  hipStream_t s = static_cast<hipStream_t>(stream);
  LevelDev& L = h->lv[level];
  // the ping-pong between x_out and the level's work buffer t starts where it ends in x_out
  if (x_is_zero) {
    const int rest = sweeps - 1;
    void* cur = (rest % 2 == 0) ? x_out : L.t;
    void* oth = (cur == x_out) ? L.t : x_out;
    MG_HIP(launch_sweep0(L.Ac, L.S, b, cur, first_omega(h, level), h->xk, s));
    return smooth_level(h, level, b, cur, oth, rest, s, 1, true);
  }
  void* cur = (sweeps % 2 == 0) ? x_out : L.t;
  void* oth = (cur == x_out) ? L.t : x_out;
  MG_HIP(launch_convert(L.N, x, h->xk, cur, h->xk, s));
  return smooth_level(h, level, b, cur, oth, sweeps, s, 0, false);
}

int mg_level_eigen_estimate(const mg_handle* h, int32_t level, double* lambda_max) {
  if (!h || !lambda_max || level < 0 || level > h->L) return fail(MG_EINVAL, "bad handle, level or output");
  if (h->cfg.smoother != MG_SMOOTH_CHEBYSHEV || level < 1) return fail(MG_EUNSUPPORTED, "no estimate: not a Chebyshev level");
  *lambda_max = h->lam[size_t(level)];
  return MG_OK;
}

int mg_level_restrict(mg_handle* h, int32_t level, const void* r_fine, void* d_coarse, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (level < 1) return fail(MG_EINVAL, "restriction needs level >= 1");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_restrict_s(L.Rs, L.B, r_fine, d_coarse, h->lv[level - 1].mask, L.mask, h->xk,
                           static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_level_prolong(mg_handle* h, int32_t level, const void* y_coarse, void* x_fine, void* stream) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (level < 1) return fail(MG_EINVAL, "prolongation needs level >= 1");
  LevelDev& L = h->lv[level];
  MG_HIP(launch_prolong_s(L.Ps, L.B, y_coarse, x_fine, L.mask, h->lv[level - 1].mask, h->xk,
                          static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_coarse_solve(mg_handle* h, const void* b, void* x, void* stream) {
  int rc = check_level(h, 0);
  if (rc) return rc;
  if (b == x) return fail(MG_EINVAL, "coarse solution must not alias its right-hand side");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->cfg.coarse_mode == MG_COARSE_EXACT) {
    MG_HIP(launch_coarse_gemv(h->n0, h->Ainv, b, x, h->xk, s));
    return MG_OK;
  }
  LevelDev& C0 = h->lv[0];
  const int k = std::max(1, h->cfg.coarse_sweeps);
  void* cu = ((k - 1) % 2 == 0) ? x : C0.t;
  void* ot = ((k - 1) % 2 == 0) ? C0.t : x;
  MG_HIP(launch_sweep0(C0.Ac, C0.S, b, cu, h->cfg.omega, h->xk, s));
  return smooth_level(h, 0, b, cu, ot, k - 1, s);
}

int mg_level_export(const mg_handle* h, int32_t level, void* values, int8_t* row_exp) {
  if (!h || !values || level < 0 || level > h->L) return fail(MG_EINVAL, "bad handle, level or output");
  const LevelDev& L = h->lv[level];
  const SellDev& A = L.Ac;
  if (L.hrow.empty()) return fail(MG_EUNSUPPORTED, "no host geometry kept for this level");
  if (A.kind == VK_DICT) return fail(MG_EUNSUPPORTED, "the level's values are stored as a block dictionary");
  if ((A.kind == VK_F16 || A.kind == VK_BF16) && !row_exp) return fail(MG_EINVAL, "row_exp is required for 16-bit values");
  const int B = L.B, W = kWave, R = A.R;
  const int vb = A.kind == VK_F64 ? 8 : A.kind == VK_F32 ? 4 : 2;
  const int64_t slots = L.hsptr.back();
  std::vector<char> dv(size_t(slots) * B * W * vb);
  MG_HIP(hipMemcpy(dv.data(), A.val, dv.size(), hipMemcpyDeviceToHost));
  std::vector<int8_t> de;
  if (A.rexp) {
    de.resize(size_t(A.nslices) * W);
    MG_HIP(hipMemcpy(de.data(), A.rexp, de.size(), hipMemcpyDeviceToHost));
  }
  char* out = static_cast<char*>(values);
  for (int64_t pos = 0; pos < L.n; ++pos) {
    const int64_t node = L.hperm.empty() ? pos : L.hperm[size_t(pos)];
    const int64_t slice = pos / R, r = pos % R;
    const int32_t len = L.hrow[size_t(node) + 1] - L.hrow[size_t(node)];
    for (int32_t k = 0; k < len; ++k) {
      const int64_t slot = int64_t(L.hsptr[size_t(slice)]) + k;
      const int64_t blk = int64_t(L.hrow[size_t(node)]) + k;
      for (int c = 0; c < B; ++c)
        for (int cc = 0; cc < B; ++cc)
          std::memcpy(out + (size_t(blk) * B * B + c * B + cc) * vb,
                      dv.data() + (size_t(slot * B + cc) * W + r * B + c) * vb, vb);
    }
    if (A.rexp)
      for (int c = 0; c < B; ++c) row_exp[size_t(node) * B + c] = de[size_t(slice) * W + r * B + c];
  }
  return MG_OK;
}

int mg_level_info(const mg_handle* h, int32_t level, int32_t* n_nodes, int32_t* block, int64_t* nnzb) {
  if (!h || level < 0 || level > h->L) return fail(MG_EINVAL, "bad handle or level");
  const LevelDev& L = h->lv[level];
  if (n_nodes) *n_nodes = L.n;
  if (block) *block = L.B;
  if (nnzb) *nnzb = L.nnzb;
  return MG_OK;
}

int mg_level_tuning(const mg_handle* h, int32_t level, int32_t* slot_batch, int32_t* col_bytes,
                    double* us_default, double* us_other) {
  if (!h || level < 0 || level > h->L) return fail(MG_EINVAL, "bad handle or level");
  const LevelDev& L = h->lv[level];
  int kd, ko;
  slot_batch_choices(L.B, &kd, &ko);
  if (slot_batch) *slot_batch = L.Ac.kb ? L.Ac.kb : kd;
  if (col_bytes) *col_bytes = L.A64.col16 ? 2 : 4;
  if (us_default) *us_default = L.us_def;
  if (us_other) *us_other = L.us_alt;
  return MG_OK;
}

int mg_level_transfer_format(const mg_handle* h, int32_t level, int32_t* p_col_bytes, int32_t* r_col_bytes,
                             int32_t* weight_bytes) {
  if (!h || level < 1 || level > h->L) return fail(MG_EINVAL, "bad handle or level (transfers exist on levels >= 1)");
  const TSellDev& P = h->lv[level].Ps;
  const TSellDev& R = h->lv[level].Rs;
  if (p_col_bytes) *p_col_bytes = P.node ? 2 : 4;
  if (r_col_bytes) *r_col_bytes = R.node ? 2 : 4;
  if (weight_bytes) *weight_bytes = P.node ? 1 : P.f32 ? 4 : 8;
  return MG_OK;
}

int mg_level_dictionary(const mg_handle* h, int32_t level, int32_t* n_blocks) {
  if (!h || !n_blocks || level < 0 || level > h->L) return fail(MG_EINVAL, "bad handle, level or output");
  const SellDev& A = h->lv[level].A64;
  *n_blocks = A.kind == VK_DICT ? A.ndict : 0;
  return MG_OK;
}

int32_t mg_num_levels(const mg_handle* h) { return h ? h->L + 1 : 0; }

void mg_destroy(mg_handle* h) { delete h; }

const char* mg_status_string(int status) {
  switch (status) {
    case MG_OK: return "ok";
    case MG_EINVAL: return "invalid argument or malformed input";
    case MG_ENOMEM: return "out of memory";
    case MG_EDEVICE: return "HIP runtime error";
    case MG_ESINGULAR: return "singular diagonal block or coarse matrix";
    case MG_ENOCONV: return "not converged within maxit";
    case MG_ENUMERIC: return "non-finite or diverging residual";
    case MG_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char* mg_last_error(void) { return g_err.c_str(); }

int mg_setup_batch(const mg_level_in* const* problems, const int32_t* n_levels, int32_t n_problems, int32_t nrhs,
                   const mg_config* cfg, int32_t inputs_on_device, void* stream, mg_batch** out) {
  if (!problems || !n_levels || !cfg || !out || n_problems < 1) return fail(MG_EINVAL, "null argument or no problems");
  *out = nullptr;
  if (nrhs != 1 && nrhs != 8) return fail(MG_EUNSUPPORTED, "batched solves support 1 or 8 right-hand sides");
  int rc = check_config(*cfg);
  if (rc) return rc;
  if (cfg->outer != MG_OUTER_FGMRES) return fail(MG_EUNSUPPORTED, "batched solves use the FGMRES outer loop");
  if (cfg->coarse_mode != MG_COARSE_EXACT) return fail(MG_EUNSUPPORTED, "batched solves use the exact coarse solve");
  if (cfg->smoother != MG_SMOOTH_JACOBI) return fail(MG_EUNSUPPORTED, "batched solves use the damped (block-)Jacobi smoother");
  if (cfg->precision == MG_PREC_FP64_DICT) return fail(MG_EUNSUPPORTED, "batched solves store plain values");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<std::vector<HostLevel>> HH(n_problems);
  for (int p = 0; p < n_problems; ++p) {
    if (n_levels[p] < 1 || !problems[p]) return fail(MG_EINVAL, "problem without levels");
    if ((rc = load_hierarchy(problems[p], n_levels[p], inputs_on_device != 0, HH[p]))) return rc;
    if (HH[p][0].B != HH[0][0].B) return fail(MG_EINVAL, "all problems of a batch need the same block size");
  }
  const int B = HH[0][0].B;
  if (nrhs == 8 && B != 1) return fail(MG_EUNSUPPORTED, "8 right-hand sides are implemented for block size 1");
  if (B == 2) return fail(MG_EUNSUPPORTED, "batched solves support block sizes 1, 3 and 4");
  mg_batch* h = new (std::nothrow) mg_batch();
  if (!h) return fail(MG_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->NR = nrhs;
  h->P = n_problems;
  h->B = B;
  h->xk = cfg->precision == MG_PREC_FP64 ? X_F64 : X_F32;
  h->vkind = value_kind(cfg->precision);
  try {
    rc = setup_batch(h, HH, s);
  } catch (const std::bad_alloc&) {
    rc = fail(MG_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return MG_OK;
}

int mg_batch_offsets(const mg_batch* h, int64_t* offsets) {
  if (!h || !offsets) return fail(MG_EINVAL, "null argument");
  for (size_t p = 0; p < h->off.size(); ++p) offsets[p] = h->off[p];
  return MG_OK;
}

int mg_solve_batch(mg_batch* h, const double* b, double* x, mg_solve_stats* stats, void* stream) {
  if (!h || !b || !x) return fail(MG_EINVAL, "null argument");
  try {
    return solve_batch_impl(h, b, x, stats, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    return fail(MG_ENOMEM, "host allocation failed");
  }
}

void mg_destroy_batch(mg_batch* h) { delete h; }


struct mg_time : TimeDev {};

int mg_time_setup(mg_handle* h, int32_t n_g, const int32_t* R_rowptr, const int32_t* R_col, const double* R_val,
                  const int32_t* H_rowptr, const int32_t* H_col, const double* H_val, const int32_t* g_idx,
                  double dt, void* stream, mg_time** out) {
  if (!h || !out || (n_g > 0 && !g_idx) || n_g < 0) return fail(MG_EINVAL, "null argument or negative n_g");
  *out = nullptr;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MG_EINVAL, "dt must be positive and finite");
  const int64_t N = h->lv[h->L].N;
  if (N + n_g > INT32_MAX) return fail(MG_EUNSUPPORTED, "more than 2^31 - 1 columns in R");
  mg_time* t = new (std::nothrow) mg_time();
  if (!t) return fail(MG_ENOMEM, "host allocation failed");
  t->h = h;
  t->n = int32_t(N);
  t->n_g = n_g;
  t->dt = dt;
  int rc;
  try {
    rc = time_setup(t, R_rowptr, R_col, R_val, H_rowptr, H_col, H_val, g_idx, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    rc = fail(MG_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete t;
    return rc;
  }
  *out = t;
  return MG_OK;
}

int mg_time_rhs(mg_time* t, const double* theta, const double* f, const double* g, double* b, void* stream) {
  if (!t || !theta || !f || !b || (t->n_g > 0 && !g)) return fail(MG_EINVAL, "null argument");
  if (b == theta || b == f || b == g) return fail(MG_EINVAL, "b must not alias the inputs");
  MG_HIP(launch_time_rhs(t->n, t->rrow, t->rcol, t->rval, theta, f, g, t->dt, b, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_time_theta(mg_time* t, const double* x, const double* g, double* theta, void* stream) {
  if (!t || !x || !theta || (t->n_g > 0 && !g)) return fail(MG_EINVAL, "null argument");
  if (theta == x || theta == g) return fail(MG_EINVAL, "theta must not alias the inputs");
  MG_HIP(launch_time_theta(t->n, t->hrow, t->hcol, t->hval, t->gpos, x, g, theta, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_time_run(mg_time* t, int32_t steps, double* theta, const double* F, const double* G, double* x,
                double* history, mg_solve_stats* stats, void* stream) {
  if (!t || !theta || !x || steps < 0 || (steps > 0 && !F) || (steps > 0 && t->n_g > 0 && !G))
    return fail(MG_EINVAL, "null argument or negative step count");
  if (theta == x) return fail(MG_EINVAL, "theta must not alias x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = t->n, ng = t->n_g;
  for (int32_t k = 0; k < steps; ++k) {
    const double* f = F + k * n;
    const double* g = ng > 0 ? G + k * ng : nullptr;
    MG_HIP(launch_time_rhs(t->n, t->rrow, t->rcol, t->rval, theta, f, g, t->dt, t->b, s));
    int rc = solve_impl(t->h, t->b, x, stats ? stats + k : nullptr, s, 0);
    if (rc) return rc;
    MG_HIP(launch_time_theta(t->n, t->hrow, t->hcol, t->hval, t->gpos, x, g, theta, s));
    if (history)
      MG_HIP(hipMemcpyAsync(history + k * n, theta, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return MG_OK;
}

void mg_time_destroy(mg_time* t) { delete t; }

struct mg_ns : NsDev {};

int mg_ns_setup(const mg_ns_in* in, mg_handle* pressure, void* stream, mg_ns** out) {
  if (!in || !pressure || !out) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if (in->n_v < 1 || in->n_p < 1 || !in->m_v || !in->m_p || !in->dir_mask || !in->dir_val)
    return fail(MG_EINVAL, "empty problem or missing array");
  if (!(in->dt > 0.0) || !std::isfinite(in->dt) || !(in->nu >= 0.0) || !std::isfinite(in->nu))
    return fail(MG_EINVAL, "dt must be positive and nu non-negative");
  const LevelDev& T = pressure->lv[pressure->L];
  if (T.B != 1 || T.n != in->n_p) return fail(MG_EINVAL, "pressure hierarchy must be scalar with n_p finest nodes");
  if (pressure->xk != X_F64) return fail(MG_EUNSUPPORTED, "the pressure solve runs on an FP64 handle");
  if (int64_t(in->n_v) * 3 > INT32_MAX) return fail(MG_EUNSUPPORTED, "too many velocity nodes");
  mg_ns* t = new (std::nothrow) mg_ns();
  if (!t) return fail(MG_ENOMEM, "host allocation failed");
  t->hp = pressure;
  t->n_v = in->n_v;
  t->n_p = in->n_p;
  t->nu = in->nu;
  t->dt = in->dt;
  int rc;
  try {
    rc = ns_setup(t, *in, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    rc = fail(MG_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete t;
    return rc;
  }
  *out = t;
  return MG_OK;
}

int mg_ns_momentum(mg_ns* t, const double* u, const double* p, const double* q, const double* f, double* u_out,
                   void* stream) {
  if (!t || !u || !p || !q || !u_out) return fail(MG_EINVAL, "null argument");
  if (u_out == u) return fail(MG_EINVAL, "u_out must not alias u");
  MG_HIP(launch_ns_momentum(t->V, t->G, u, p, q, f, t->m_v, t->dmask, t->dval, t->nu, t->dt, u_out,
                            static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_ns_divergence(mg_ns* t, const double* u, double* du, double* rhs, void* stream) {
  if (!t || !u || !du || !rhs) return fail(MG_EINVAL, "null argument");
  if (du == rhs) return fail(MG_EINVAL, "du and rhs must differ");
  MG_HIP(launch_ns_divergence(t->D, u, t->hp->lv[t->hp->L].mask, t->dt, du, rhs, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_ns_pressure_update(mg_ns* t, double* p, const double* q, const double* du, void* stream) {
  if (!t || !p || !q || !du) return fail(MG_EINVAL, "null argument");
  MG_HIP(launch_ns_pressure(t->n_p, p, q, du, t->m_p, t->nu, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

int mg_ns_run(mg_ns* t, int32_t steps, double* u, double* p, double* q, const double* f, mg_solve_stats* stats,
              void* stream) {
  if (!t || !u || !p || !q || steps < 0) return fail(MG_EINVAL, "null argument or negative step count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nu3 = size_t(t->n_v) * 3;
  for (int32_t k = 0; k < steps; ++k) {
    MG_HIP(launch_ns_momentum(t->V, t->G, u, p, q, f, t->m_v, t->dmask, t->dval, t->nu, t->dt, t->ubuf, s));
    MG_HIP(hipMemcpyAsync(u, t->ubuf, nu3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    MG_HIP(launch_ns_divergence(t->D, u, t->hp->lv[t->hp->L].mask, t->dt, t->du, t->rhs, s));
    const int rc = solve_impl(t->hp, t->rhs, q, stats ? stats + k : nullptr, s, 0);
    if (rc) return rc;
    MG_HIP(launch_ns_pressure(t->n_p, p, q, t->du, t->m_p, t->nu, s));
  }
  return MG_OK;
}

void mg_ns_destroy(mg_ns* t) { delete t; }

struct mg_asm : AsmDev {};

int mg_asm_setup(const mg_asm_in* in, void* stream, mg_asm** out) {
  if (!in || !out) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if ((in->dim != 2 && in->dim != 3) || (in->block != 1 && in->block != in->dim))
    return fail(MG_EINVAL, "dim must be 2 or 3 and block 1 or dim");
  if (in->n_nodes < 1 || in->n_cells < 1 || in->nnzb < 1 || !in->cell_corner || !in->cell_size || !in->dof_mask ||
      !in->A_rowptr || !in->A_col || in->n_hanging < 0 || (in->n_hanging > 0 && (!in->hang_node || !in->hang_master ||
                                                                               !in->hang_weight)))
    return fail(MG_EINVAL, "empty mesh or missing array");
  mg_asm* a = new (std::nothrow) mg_asm();
  if (!a) return fail(MG_ENOMEM, "host allocation failed");
  int rc;
  try {
    rc = asm_setup(a, *in, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    rc = fail(MG_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete a;
    return rc;
  }
  *out = a;
  return MG_OK;
}

int mg_asm_values(mg_asm* a, const mg_asm_coef* coef, double* val, void* stream) {
  if (!a || !coef || !val) return fail(MG_EINVAL, "null argument");
  const bool scalar = coef->pde == MG_ASM_POISSON || coef->pde == MG_ASM_TD;
  if ((coef->pde != MG_ASM_POISSON && coef->pde != MG_ASM_TD && coef->pde != MG_ASM_ELASTICITY) ||
      (scalar ? a->B != 1 : a->B != a->dim))
    return fail(MG_EINVAL, "pde does not match the block size");
  if (coef->pde == MG_ASM_TD && !(coef->eps > 0.0)) return fail(MG_EINVAL, "diffusion must be positive");
  AsmCoef c;
  c.pde = coef->pde;
  c.eps = coef->eps;
  for (int k = 0; k < 3; ++k) c.bvec[k] = coef->bvec[k];
  c.supg = coef->supg;
  c.lam = coef->lam;
  c.mu = coef->mu;
  c.mass_coef = coef->mass_coef;
  hipStream_t s = static_cast<hipStream_t>(stream);
  MG_HIP(launch_asm_table(c, a->dim, a->B, a->nd, a->sizes, a->table, s));
  MG_HIP(launch_asm_gather(a->nnzb, a->dim, a->B, a->nd, a->brow, a->bcol, a->cptr, a->code, a->table, a->mask, val,
                           s));
  return MG_OK;
}

void mg_asm_destroy(mg_asm* a) { delete a; }

}  // extern "C"
