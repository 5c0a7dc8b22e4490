// Internal declarations shared by the HIP kernels and the host runtime of libmgq1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgq1 {

// storage kind of matrix values
enum ValKind { VK_F64 = 0, VK_F32 = 1, VK_F16 = 2, VK_BF16 = 3, VK_DICT = 4 };
// storage kind of vectors
enum VecKind { X_F64 = 0, X_F32 = 1 };

constexpr int kWave = 64;             // wavefront width on CDNA
constexpr int kSliceWaves = 4;        // slices (one per wave) per 256-thread workgroup
constexpr int kRedThreads = 1024;
constexpr int kMaxRedBlocks = 2048;   // grid (= partial count) of the vector reductions

// Sliced ELL of a block matrix: one slice = 64 lanes = R = 64/B nodes x B components;
// lane = r*B + c handles scalar row (node slice*R + r, component c).  For block slot k of
// the slice, the value of column component cc for lane `ln` sits at
// val[(k*B + cc)*64 + ln] and the column node of row r at col[k*R + r] (k counts from
// sptr[slice]).  Padding slots hold value 0 and the row's own node as column.
struct SellDev {
  int32_t n = 0, B = 1, R = 64, nslices = 0;
  int32_t ell = 0;                  // > 0: every slice has this width (sptr[s] = s * ell), so
                                    // the kernels need no load for the slot range
  int64_t slots = 0;
  const int32_t* sptr = nullptr;    // nslices + 1
  const int32_t* col = nullptr;     // slots * R
  const void* val = nullptr;        // slots * B * 64 values of `kind`
  const int8_t* rexp = nullptr;     // nslices * 64 power-of-two row exponents (F16 / BF16)
  int kind = VK_F64;
  int kb = 0;                       // block slots per load batch (0: the default for B)
  const uint16_t* col16 = nullptr;  // col - colbase[slot] as 16 bits where the slot's columns
  const int32_t* colbase = nullptr; // span less than 2^16 (NULL: the kernels read col)
  const uint32_t* wide = nullptr;   // with col16: bit s set = slice s reads col instead
                                    // (some slot spans 2^16 or more); NULL: no such slice
  const int32_t* perm = nullptr;    // node at row position slice*R + r (NULL: the position
                                    // itself); rows sorted by length inside windows of slices
  int nt = 1;                       // 1: values and indices read with non-temporal loads
  // kind VK_DICT: the block of node row r in slot k is dtab[didx[k * R + r]] (ndict
  // distinct B x B FP64 blocks, row-major); val is not read
  const uint16_t* didx = nullptr;
  const double* dtab = nullptr;
  int32_t ndict = 0;
  int dlds = 0;                     // VK_DICT: every workgroup first copies dtab into LDS
};

// the two slot-batch sizes the slice kernels are built for (default, alternative)
void slot_batch_choices(int B, int* kb_def, int* kb_other);

// scalar CSR (transfer matrices); weights stored as float when every weight is exact in
// FP32 (dyadic), else as double
struct CsrDev {
  int32_t nrows = 0, ncols = 0;
  int64_t nnz = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const void* val = nullptr;
  int f32 = 1;
};

// the same scalar transfer matrix as a sliced ELL over node rows (the layout the grid
// kernels use): a slice holds R = 64 / (B * NR) rows, one lane per (row, component, rhs);
// slot k of row r of slice s sits at col / w[k * R + r] with k in [sptr[s], sptr[s+1]),
// padded slots carry weight 0 and a column of their own row
struct TSellDev {
  int32_t nrows = 0, ncols = 0, R = 64, nslices = 0;
  int32_t ell = 0;                  // > 0: uniform slice width, as in SellDev
  int nt = 1;                       // 1: indices and weights read with non-temporal loads
  const int32_t* sptr = nullptr;
  const int32_t* col = nullptr;
  const void* w = nullptr;
  int f32 = 1;
  // node form (single right-hand side, dyadic weights): slices of R = 64 nodes, one lane per
  // node computing its B components; per slot entry ent[k * 64 + r] = column offset from
  // colbase[k] | weight code (w * 128) << 16 | mask bits of the column's B DoFs << 24, and
  // rmask[node] = mask bits of the row's B DoFs
  int node = 0;
  const uint32_t* ent = nullptr;
  const int32_t* colbase = nullptr;
  const uint8_t* rmask = nullptr;
};

// d = M_c P~^T M_f r (rows = coarse nodes; mask_f may be NULL) and x += M_f P~ M_c y
// (rows = fine nodes), single right-hand side, with the sliced transfer matrices
hipError_t launch_restrict_s(const TSellDev& R, int B, const void* r, void* d, const uint8_t* mask_c,
                             const uint8_t* mask_f, int xk, hipStream_t s);
hipError_t launch_prolong_s(const TSellDev& P, int B, const void* y, void* x, const uint8_t* mask_f,
                            const uint8_t* mask_c, int xk, hipStream_t s);

// one level of the single-workgroup tail of the V-cycle (device-resident array)
struct TailLevel {
  SellDev A;                        // cycle operator
  const void* S = nullptr;          // smoother blocks (lane layout, cycle precision)
  const uint8_t* mask = nullptr;    // constrained DoFs
  CsrDev P, R;                      // from level l-1 (unused on level 0)
  void *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;
};

struct TailParams {
  int top = 0;                      // highest level handled by the tail
  int nu1 = 2, nu2 = 2;
  double omega = 1.0;
  const double* Ainv = nullptr;     // coarse inverse, row-major FP64
  int n0 = 0;
  int coarse_mode = 0, coarse_sweeps = 1;
};

// ------------------------------------------------------------------ launchers
// y = A x (mode 0), y = b - A x (mode 1), y = M (b - A x) with M zeroing constrained
// DoFs (mode 2); with `partials` != NULL every block also writes the sum of squares of
// its y entries to partials[block] (spmv_grid(A) entries).  xk / yk: vector kinds.
hipError_t launch_spmv(const SellDev& A, const void* b, const void* x, void* y, const uint8_t* mask,
                       int xk, int yk, int mode, double* partials, hipStream_t s,
                       const double* dotv = nullptr);
int spmv_grid(const SellDev& A);
// x_out = x + omega S (b - A x); S in lane layout, same kind as the vectors.  pmode 1:
// also + beta (x - x_prev) with x_prev read from xo before it is overwritten (three-term
// Chebyshev step); pmode 2: + beta x (x_prev = 0)
hipError_t launch_sweep(const SellDev& A, const void* S, const void* b, const void* x, void* xo,
                        double omega, int xk, hipStream_t s, double beta = 0.0, int pmode = 0);
// x_out = omega S b
// two sweeps from x = 0 in one pass (block size 1): xo = x1 + omega S (b - A x1), x1 = omega S b
hipError_t launch_sweep2z(const SellDev& A, const void* S, const void* b, void* xo, double omega, int xk,
                          hipStream_t s);
hipError_t launch_sweep0(const SellDev& A, const void* S, const void* b, void* xo, double omega,
                         int xk, hipStream_t s);
// x = Ainv b with the FP64 inverse stored row-major; b / x of kind xk
hipError_t launch_coarse_gemv(int n, const double* Ainv, const void* b, void* x, int xk, hipStream_t s);
// Gauss-Jordan with partial pivoting on the n x 2n augmented matrix M = [A | I]
// (row-major, FP64); writes the inverse (row-major) to Ainv; flag != 0 if singular
hipError_t launch_coarse_invert(int n, double* M, double* Ainv, double* pivbuf, int* flag,
                                hipStream_t s);
// levels p.top .. 1 and the coarse solve of one V-cycle in one workgroup
hipError_t launch_tail(const TailLevel* lv, int B, int kind, int xk, const TailParams& p, hipStream_t s);
// nodal block inverses of the diagonal blocks of A (FP64 SELL) into S (lane layout,
// double or float per sk); flag != 0 if a block is singular
hipError_t launch_block_invert(const SellDev& A, void* S, int sk, int* flag, int NR, hipStream_t s);

// vector kernels (n elements)
hipError_t launch_fill(int64_t n, void* y, int yk, double v, hipStream_t s);
hipError_t launch_convert(int64_t n, const void* x, int xk, void* y, int yk, hipStream_t s);
hipError_t launch_axpy(int64_t n, void* y, int yk, const void* x, int xk, double sign,
                       const double* alpha, hipStream_t s);          // y += sign * (*alpha) * x
// y = x / *denom (if != 0), and in FP32 to yc when given
hipError_t launch_scale_div(int64_t n, double* y, const double* x, const double* denom,
                            hipStream_t s, float* yc = nullptr);
// deterministic reductions without atomics: producers write one partial per block
// (reduction_grid(n) of them); consumers re-sum them in a fixed order
int reduction_grid(int64_t n);
hipError_t launch_dot_partials(int64_t n, const double* a, const double* b, double* partials, hipStream_t s);
hipError_t launch_finish(const double* partials, int g, double* out, int sqrt_out, hipStream_t s);
// MGS step: h = sum(pin) -> *hout; w -= h vi; partials of (w, vnext) (vnext NULL: (w, w));
// gin = number of partials in pin (0: reduction_grid(n))
hipError_t launch_mgs_step(int64_t n, double* w, const double* vi, const double* vnext, const double* pin,
                           double* pout, double* hout, hipStream_t s, int gin = 0);
// nrm = sqrt(sum(pin)) -> *hout; w /= nrm unless nrm == 0.  With H given, Givens step gj
// of GMRES on the (m+1) x m Hessenberg H (column-major, ld = m+1) follows in the same
// kernel: rotate column gj by the previous rotations, form rotation gj, update g;
// st[0] = |g[gj+1]|, st[1] = 1 if H[gj+1][gj] was 0 before the rotation.  With wc given,
// w is also written there in FP32.
hipError_t launch_mgs_normalize(int64_t n, double* w, const double* pin, double* hout, hipStream_t s, int gj = 0,
                                int gm = 0, double* H = nullptr, double* cs = nullptr, double* sn = nullptr,
                                double* gg = nullptr, double* st = nullptr, float* wc = nullptr);
// x += sum_{i<k} y[i] Z_i, Z_i = Z + i*ldz of kind zk
hipError_t launch_update_x(int64_t n, double* x, const void* Z, int zk, int64_t ldz, const double* y,
                           int k, hipStream_t s);
// y = H[:k,:k]^{-1} g[:k] (upper triangular)
hipError_t launch_backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t s);
// g = (beta, 0, ..., 0), beta read from the device
hipError_t launch_init_g(int m, double* g, const double* beta, hipStream_t s);

// ------------------------------------------------------------------ Chebyshev setup
// v_i = frac(i g) - 1/2, g = (sqrt(5) - 1) / 2 (Weyl sequence), in vector kind xk
hipError_t launch_weyl(int64_t n, void* v, int xk, hipStream_t s);
// per-workgroup partial sums of v_i^2 (reduction_grid(n) of them)
hipError_t launch_sumsq_partials(int64_t n, const void* v, int xk, double* partials, hipStream_t s);
// v = w / *d
hipError_t launch_scale_inv(int64_t n, void* v, const void* w, int xk, const double* d, hipStream_t s);

// ------------------------------------------------------------------ time stepping
// b = R [theta / dt + f ; g] (R: n rows of a scalar CSR over n + n_g columns; columns
// below n address theta / dt + f, the others g)
hipError_t launch_time_rhs(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                           const double* theta, const double* f, const double* g, double dt, double* b,
                           hipStream_t s);
// theta = H x (scalar CSR, n x n), then theta_i = g[gpos[i]] where gpos[i] >= 0
hipError_t launch_time_theta(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                             const int32_t* gpos, const double* x, const double* g, double* theta,
                             hipStream_t s);

// ------------------------------------------------------------------ pressure correction
// Sliced ELL over rows with several FP64 value arrays on one pattern: slice s holds rows
// [64 s, 64 s + 64); its slots t in [sptr[s], sptr[s+1]) hold col[t * 64 + lane] and the
// values val[(t * V + v) * 64 + lane], v < V (V = 4 for K, C_x, C_y, C_z; 3 for G_a and
// D_a); padding slots carry a valid column and zero values.
struct NsEll {
  int64_t nrows = 0, nslices = 0;
  const int32_t* sptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
};
// Step 1: u_out (n_v x 3) from u, s = p + q, optional forcing f (NULL = 0)
hipError_t launch_ns_momentum(const NsEll& V, const NsEll& G, const double* u, const double* p, const double* q,
                              const double* f, const double* m_v, const uint8_t* dmask, const double* dval, double nu,
                              double k, double* uo, hipStream_t s);
// du = D u, rhs = -du / k (0 where pin)
hipError_t launch_ns_divergence(const NsEll& D, const double* u, const uint8_t* pin, double k, double* du, double* rhs,
                                hipStream_t s);
// Step 3: p = p + q - nu du / m_p
hipError_t launch_ns_pressure(int64_t n, double* p, const double* q, const double* du, const double* m_p, double nu,
                              hipStream_t s);

// ------------------------------------------------------------------ GPU assembly
enum { kAsmPoisson = 0, kAsmTD = 1, kAsmElasticity = 2 };
struct AsmCoef {
  int pde = kAsmPoisson;
  double eps = 1.0, bvec[3] = {0.0, 0.0, 0.0};
  int supg = 0;
  double lam = 0.0, mu = 0.0, mass_coef = 0.0;
};
// element matrices of nd cell sizes: table[((d nb + a) nb + b) B^2 + ci B + cj]
hipError_t launch_asm_table(const AsmCoef& c, int dim, int B, int nd, const double* sizes, double* table,
                            hipStream_t s);
// val[k] (B x B, row-major) of every stored block k = (brow[k], bcol[k]) from its
// contributions code[cptr[k] .. cptr[k+1]) (d | a << 5 | b << 8 | e << 11, weight 2^-e),
// then identity rows / zero columns of the masked DoFs
hipError_t launch_asm_gather(int64_t nnzb, int dim, int B, int nd, const int32_t* brow, const int32_t* bcol,
                             const uint32_t* cptr, const uint16_t* code, const double* table, const uint8_t* mask,
                             double* val, hipStream_t s);

// ------------------------------------------------------------------ batched form
// Many independent problems (same block size) with NR right-hand sides each.  Vectors
// of one problem are stored [node][component][rhs]; the problems' vectors are
// concatenated.  A batched launch covers one step of the V-cycle (or of the outer loop)
// for every problem at once: entry e of the launch's table describes one problem and owns
// blocks [first_e, first_{e+1}).
enum BKind {
  BK_SWEEP0 = 0,   // out = omega S in0
  BK_SWEEP = 1,    // out = in1 + omega S (in0 - A in1)
  BK_DEFECT = 2,   // out = M (in0 - A in1)
  BK_RESTRICT = 3, // out = M_c T in0           (T = P~^T)
  BK_PROLONG = 4,  // out += M T M_c in0         (T = P~)
  BK_COARSE = 5,   // out = Ainv in0
  BK_SPMV64 = 6,   // out (FP64) = A64 in1 (cycle precision)
  BK_DEFECT64 = 7, // out = in0 - A64 in1 (all FP64), partial sums of squares per (block, rhs)
  BK_FILL0 = 8     // out = 0
};

struct BEntry {
  SellDev A;
  const void* S = nullptr;
  const uint8_t* mask = nullptr;
  TSellDev Ts;                       // transfer from the next coarser level (restrict / prolong)
  const uint8_t* mask_c = nullptr;
  const void* in0 = nullptr;
  const void* in1 = nullptr;
  void* out = nullptr;
  const double* Ainv = nullptr;
  int n0 = 0;
  int prob = 0;
  int first = 0;
};

// blocks of an entry for a launch kind
int batched_blocks(int kind, const SellDev& A, const TSellDev& Ts, int n0, int NR);
// one batched step; `active[prob] == 0` skips a problem; `partials` for BK_DEFECT64
// kb: slot batch of the slice kernels (sweep, defect, SpMV64, defect64); 0 = default;
// negative: -kb with the 16-bit column format (all entries of the launch must have it)
hipError_t launch_batched(int kind, const BEntry* entries, int n_entries, int n_blocks, int B, int NR, int vkind,
                          int xk, double omega, const int* active, double* partials, int kb, hipStream_t s);

// vector segments of the concatenated batch vectors: problem p owns elements
// [off[p], off[p] + len[p]) and vector blocks [vfirst[p], vfirst[p] + vcount[p])
struct BSegs {
  const int64_t* off = nullptr;
  const int64_t* len = nullptr;
  const int* vfirst = nullptr;
  const int* vcount = nullptr;
  const int* blk_prob = nullptr;   // vector block -> problem
  const int* on = nullptr;         // per-problem flags (NULL: all problems take part)
  int n_blocks = 0;
  int NR = 1;
};
constexpr int kSegBlocksMax = 1024;  // vector blocks per problem (partials re-summed per block)

// partial sums per (vector block, rhs) of a.b (b == NULL: a.a)
hipError_t launch_bdot(const BSegs& g, const double* a, const double* b, double* partials, hipStream_t s);
// per-instance sum (sqrt) of partials over the instance's blocks: out[p*NR + q]
// (pfirst / pcount: blocks per problem of the producing launch)
hipError_t launch_bfinish(const double* partials, const int* pfirst, const int* pcount, int n_inst, int NR,
                          double* out, int sqrt_out, hipStream_t s);
// batched modified Gram-Schmidt step / normalisation; per-instance Hessenberg entries are
// written to H[inst * hstride] (H points at the entry's offset inside each instance block)
hipError_t launch_bmgs_step(const BSegs& g, double* w, const double* vi, const double* vnext, const double* pin,
                            double* pout, double* H, int64_t hstride, hipStream_t s);
hipError_t launch_bmgs_normalize(const BSegs& g, double* w, const double* pin, double* H, int64_t hstride,
                                 hipStream_t s, float* wc = nullptr);
// y = x / beta[inst] (0 where beta == 0 or the instance is inactive)
hipError_t launch_bscale(const BSegs& g, double* y, const double* x, const double* beta, const int* iact,
                         hipStream_t s, float* yc = nullptr);
// x += sum_{i < kk[inst]} yv[inst][i] Z_i   (Z_i = Z + i * ldz of kind zk)
hipError_t launch_bupdate(const BSegs& g, double* x, const void* Z, int zk, int64_t ldz, const double* yv, int m,
                          const int* kk, hipStream_t s);
// per-instance Givens step j, then kk[inst] = j + 1 when |g_{j+1}| <= tol[inst] or breakdown
hipError_t launch_bgivens(int j, int m, int n_inst, double* H, double* cs, double* sn, double* g, double* st,
                          const double* tol, int* kk, const int* iact, hipStream_t s);
hipError_t launch_bbacksolve(int m, int n_inst, const double* H, const double* g, double* yv, const int* kk,
                             hipStream_t s);
// g[inst] = (beta, 0, ...), kk = 0
hipError_t launch_binit(int m, int n_inst, double* g, const double* beta, int* kk, hipStream_t s);
// kk[inst] = j + 1 where still 0 (end of a lockstep restart cycle of j + 1 steps)
hipError_t launch_bclose(int j, int n_inst, int* kk, const int* iact, hipStream_t s);

}  // namespace mgq1
