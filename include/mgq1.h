/*
 * mgq1.h - geometric multigrid V-cycle for nodal-block Q1 operators on MI355X (gfx950).
 *
 * The solver follows the paper's Algorithm "Geometric multigrid solver" (Sec. 2.2):
 * GMG(l, x, b) = coarse solve on level 0; otherwise pre-smooth, restrict the residual,
 * recurse from 0, prolongate and add, post-smooth.  The smoother is the fixed-matrix
 * iteration x <- x + omega S (b - A x) with S the inverse of the nodal diagonal blocks
 * (damped Jacobi for one component, nodal block-Jacobi / point-Vanka for systems), and
 * transfers are sparse matrices with R = P^T (Sec. 4.1 "Geometric Multigrid CUDA").
 * The V-cycle is used as a solver (defect correction) or as the preconditioner of a
 * restarted GMRES with modified Gram-Schmidt and Givens rotations (Sec. 4.2).
 *
 * Data layout (Sec. 2.1, Sec. 4.1 "Storage"): vectors are node-major / component-minor,
 * x[node * b + c]; matrices are block CSR with b x b blocks stored row-major.
 *
 * Levels are numbered 0 (coarsest) .. L (finest).  Level l >= 1 brings the scalar
 * prolongation P~_l (n_l x n_{l-1}) and the constrained-DoF mask M; the library applies
 * P = M_l (P~_l (x) I_b) M_{l-1} and R = P^T.
 *
 * Ownership: setup deep-copies every input (host or device) into library-owned device
 * memory; the caller may free its arrays afterwards.  Vector arguments of the solve
 * entry points are caller-owned device pointers (FP64, contiguous).  All device work is
 * enqueued on the caller's HIP stream; mg_solve synchronises that stream only to read
 * the convergence scalars.  No entry point aborts the process; errors are negative
 * return codes with a message in mg_last_error() (thread-local).  A handle must not be
 * used from two threads (or two streams) at once.
 */
#ifndef MGQ1_H
#define MGQ1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MG_OK = 0,
  MG_EINVAL = -1,      /* malformed input: sizes, indices, pattern, mask rows, NaN/Inf */
  MG_ENOMEM = -2,      /* device or host allocation failed */
  MG_EDEVICE = -3,     /* a HIP call failed */
  MG_ESINGULAR = -4,   /* a nodal diagonal block or the coarse matrix is singular */
  MG_ENOCONV = -5,     /* mg_solve reached maxit (statistics are still filled) */
  MG_ENUMERIC = -6,    /* NaN/Inf or divergence (residual > 1e6 x initial) in mg_solve */
  MG_EUNSUPPORTED = -7 /* valid request the library does not implement (e.g. block > 4) */
};

enum { MG_COARSE_EXACT = 0, MG_COARSE_SMOOTH = 1 };
enum { MG_OUTER_IR = 0, MG_OUTER_FGMRES = 1 };
/* smoother on levels >= 1 (the coarse MG_COARSE_SMOOTH variant always uses damped sweeps) */
enum { MG_SMOOTH_JACOBI = 0, MG_SMOOTH_CHEBYSHEV = 1 };
/* precision of the V-cycle; the outer defect, the update and the coarse solve are FP64.
 * MG_PREC_FP64_DICT: FP64 throughout with every level's stored blocks kept as a
 * dictionary (the distinct b x b FP64 blocks once, a 16-bit index per stored block) where
 * a level has at most 65,535 distinct blocks, else as plain FP64 values; lossless, so
 * every result is bitwise that of MG_PREC_FP64 (single-problem handles only). */
enum { MG_PREC_FP64 = 0, MG_PREC_FP32 = 1, MG_PREC_FP32_F16VAL = 2, MG_PREC_FP32_BF16VAL = 3,
       MG_PREC_FP64_DICT = 4 };

/* One level of the hierarchy (Sec. 2.2: meshes Omega_0 .. Omega_L and their spaces). */
typedef struct {
  int32_t n_nodes;            /* nodes on this level */
  int32_t block;              /* components per node, 1..4 */
  int64_t nnzb;               /* stored b x b blocks */
  const int32_t* A_rowptr;    /* n_nodes + 1, A_rowptr[0] = 0, non-decreasing */
  const int32_t* A_col;       /* nnzb node indices, sorted and unique per row, diagonal present */
  const double* A_val;        /* nnzb * b * b values, block row-major */
  int32_t p_cols;             /* nodes of level l-1 (ignored on level 0) */
  int64_t p_nnz;
  const int32_t* P_rowptr;    /* scalar P~: n_nodes + 1 (NULL on level 0) */
  const int32_t* P_col;       /* p_nnz coarse node indices, sorted and unique per row */
  const double* P_val;        /* p_nnz weights (without the masks) */
  const uint8_t* dof_mask;    /* n_nodes * b; 1 = constrained DoF: its row and column of A
                                 must be the identity row / column */
  const double* smoother_blocks; /* optional fixed smoother S (Sec. 4.1: x <- x + omega S
                                 (b - A x) with S a fixed matrix): n_nodes b x b blocks,
                                 row-major, node i's block applied to node i's defect;
                                 NULL = the inverses of A's nodal diagonal blocks, computed
                                 on the device.  Values must be finite. */
} mg_level_in;

typedef struct {
  double omega;               /* smoother damping */
  int32_t nu1, nu2;           /* pre- / post-smoothing sweeps */
  int32_t coarse_mode;        /* MG_COARSE_EXACT (dense inverse) or MG_COARSE_SMOOTH */
  int32_t coarse_sweeps;      /* sweeps on level 0 in MG_COARSE_SMOOTH mode */
  int32_t precision;          /* MG_PREC_* */
  int32_t outer;              /* MG_OUTER_IR or MG_OUTER_FGMRES */
  int32_t gmres_m;            /* restart length, 1..64 */
  int32_t maxit;              /* maximum number of V-cycles in mg_solve */
  double rtol;                /* stop when ||b - A x||_2 <= rtol ||b||_2 */
  int32_t use_graph;          /* 1: mg_solve replays one captured HIP graph per Krylov step
                                 (V-cycle, SpMV, Gram-Schmidt, Givens) instead of launching
                                 every kernel; 0: plain launches.  Results are identical. */
  int32_t slot_batch;         /* block slots whose loads the slice kernels issue together:
                                 0 = autotune (setup times both built sizes on every level's
                                 sweep and keeps the faster), or a fixed size: 8 or 16 for
                                 block sizes 1-2, 4 or 8 for 3-4.  Results are identical. */
  int32_t smoother;           /* MG_SMOOTH_JACOBI: x <- x + omega S (b - A x) (Sec. 4.1).
                                 MG_SMOOTH_CHEBYSHEV: the nu sweeps of a smoothing phase form
                                 the Chebyshev polynomial of S A on [cheb_lo, cheb_hi] *
                                 lambda, lambda estimated per level at setup by power_its
                                 steps of power iteration from a fixed Weyl-sequence vector;
                                 a stronger smoother of the fixed-matrix family (Sec. 6 names
                                 stronger smoothers as the next step).  omega is then unused
                                 on levels >= 1. */
  int32_t power_its;          /* power-iteration steps (Chebyshev only), 1..1000 */
  double cheb_lo, cheb_hi;    /* Chebyshev interval as fractions of lambda, 0 < lo < hi */
} mg_config;

typedef struct {
  int32_t iters;              /* V-cycles applied */
  int32_t restarts;           /* outer restarts (FGMRES) */
  int32_t status;             /* MG_OK, MG_ENOCONV or MG_ENUMERIC */
  int32_t converged;
  double res0, res_final;     /* ||b - A x0||_2, ||b - A x||_2 (FP64, all rows) */
  double t_solve_ms;          /* wall time of mg_solve including the final synchronisation */
} mg_solve_stats;

typedef struct mg_handle mg_handle;

/* Copy a hierarchy to the device and prepare smoother blocks, R = P~^T, the coarse
 * inverse and reduced-precision copies.  `lv[0]` is the coarsest level.  The hierarchy is
 * that of Sec. 2.2 (global coarsening of the adaptive mesh, one Q1 space per level, the
 * constrained operator A_l of each level), with the transfers of Sec. 4.1 ("Geometric
 * Multigrid CUDA": prolongation matrices assembled once, restriction as their transpose).
 * inputs_on_device: 0 = host pointers, 1 = device pointers.  stream: hipStream_t or NULL.
 * Every level is validated as by mg_validate_level; on any error nothing is kept and *out
 * is NULL. */
int mg_setup_hierarchy(const mg_level_in* lv, int32_t n_levels, const mg_config* cfg,
                       int32_t inputs_on_device, void* stream, mg_handle** out);

/* One V-cycle on the finest level (Algorithm "Geometric multigrid solver"):
 * x_is_zero != 0: x = GMG(L, 0, b) (the input value of x is not read);
 * x_is_zero == 0: x = GMG(L, x, b) with the input x as the initial iterate (nu1 full
 * pre-sweeps from it).  b, x: device FP64, n_L * b each; x must not alias b (MG_EINVAL).
 * On a mixed-precision handle b and x are rounded to FP32 for the cycle and x is
 * returned in FP64. */
int mg_vcycle(mg_handle* h, const double* b, double* x, int32_t x_is_zero, void* stream);

/* Solve A_L x = b to rtol (x is the initial guess on entry, the result on exit).
 * MG_OUTER_IR: x <- x + V(b - A x) (the MG iteration of Algorithm "Geometric multigrid
 * solver"); MG_OUTER_FGMRES: restarted flexible GMRES(m) right-preconditioned by one
 * V-cycle (Sec. 4.2).  `stats` may be NULL.  Returns MG_OK, MG_ENOCONV or MG_ENUMERIC. */
int mg_solve(mg_handle* h, const double* b, double* x, mg_solve_stats* stats, void* stream);

/* Same as mg_solve with the outer loop fixed to exactly `iters` V-cycles (FGMRES restarts
 * every m); the tolerance is not tested.  Used for step-by-step comparisons. */
int mg_solve_fixed(mg_handle* h, const double* b, double* x, int32_t iters,
                   mg_solve_stats* stats, void* stream);

/* The outer defect of the finest level in FP64 for every precision (the first step of
 * the MG iteration and of each GMRES restart, Sec. 4.2): r = b - A_L x and
 * *norm = ||r||_2.  b, x, r: device FP64 (n_L * b), r must not alias b or x;
 * norm: one device double.  Enqueued on `stream`, nothing is synchronised; uses the
 * handle's partial-sum buffer, so calls on one handle must not overlap. */
int mg_outer_defect(mg_handle* h, const double* b, const double* x, double* r, double* norm, void* stream);

/* mg_outer_defect for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same result, but the per-workgroup partial sums of the norm live in a static device
 * array of the library (65,536 doubles, 512 KiB, held by each GPU the library runs on
 * until the process ends) instead of the handle's buffer, and the call allocates nothing.
 * Finest levels whose SpMV needs more partial sums than the array holds (above about
 * 16.7 million scalar rows) are refused with MG_EUNSUPPORTED before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller. */
int mg_outer_defect_noalloc(mg_handle* h, const double* b, const double* x, double* r, double* norm,
                            void* stream);

/* The V-cycle steps one at a time on level `level`, with the operator and vectors of the
 * cycle precision: device FP64 vectors on MG_PREC_FP64 handles, device FP32 vectors (and
 * FP32 / FP16 x 2^e / BF16 x 2^e stored values, FP32 arithmetic) on the others:
 *   mg_level_defect   r = b - A_l x            (masked = 1: r = 0 on constrained DoFs)
 *   mg_level_spmv     y = A_l x
 *   mg_level_sweep    x_out = x + omega S_l (b - A_l x)      (Sec. 4.1 smoother)
 *   mg_level_sweep0   x_out = omega S_l b                    (first sweep from 0)
 *   mg_level_restrict d_{l-1} = R_{l-1} r = M_{l-1} P~^T M_l r  (Sec. 4.1 transfers)
 *   mg_level_prolong  x_l += M_l P~ M_{l-1} y_{l-1}
 *   mg_coarse_solve   x_0 = A_0^{-1} b_0 (FP64 inverse; or coarse_sweeps sweeps from 0)
 * Outputs must not alias inputs (MG_EINVAL); prolongation updates x_fine in place. */
int mg_level_defect(mg_handle* h, int32_t level, const void* b, const void* x, void* r,
                    int32_t masked, void* stream);
int mg_level_spmv(mg_handle* h, int32_t level, const void* x, void* y, void* stream);
int mg_level_sweep(mg_handle* h, int32_t level, const void* b, const void* x, void* x_out,
                   void* stream);
int mg_level_sweep0(mg_handle* h, int32_t level, const void* b, void* x_out, void* stream);
/* The level's smoother (Sec. 4.1; with MG_SMOOTH_CHEBYSHEV the three-term Chebyshev
 * steps) applied `sweeps` times to b from x (x_is_zero = 0) or from 0 (x not read), as a
 * pre- or post-smoothing phase of the V-cycle does; result in x_out.  Vectors of the cycle
 * precision; x_out must not alias b or x; uses the level's work buffer, so calls on one
 * handle must not overlap.  Chebyshev phases may have at most max(nu1, nu2) steps. */
int mg_level_smooth(mg_handle* h, int32_t level, const void* b, const void* x, void* x_out, int32_t x_is_zero,
                    int32_t sweeps, void* stream);
/* The power-iteration estimate of the largest eigenvalue of S_l A_l (Chebyshev handles,
 * levels >= 1; MG_EUNSUPPORTED otherwise). */
int mg_level_eigen_estimate(const mg_handle* h, int32_t level, double* lambda_max);
int mg_level_restrict(mg_handle* h, int32_t level, const void* r_fine, void* d_coarse,
                      void* stream);
int mg_level_prolong(mg_handle* h, int32_t level, const void* y_coarse, void* x_fine,
                     void* stream);
int mg_coarse_solve(mg_handle* h, const void* b, void* x, void* stream);

/* The stored cycle operator of level `level` in the input's BSR order (the encoding of
 * the reduced-precision form: values rounded to FP32, or a_ij / 2^e_i rounded to FP16 /
 * BF16 with e_i the smallest integer with max_j |a_ij| <= 2^e_i per scalar row).
 * values: host buffer of nnzb * b * b entries of the storage type (double, float or
 * uint16 codes), block row-major; row_exp: host buffer of n_nodes * b exponents e_i,
 * required for FP16 / BF16 handles, ignored (may be NULL) otherwise.  Synchronous.
 * MG_EUNSUPPORTED on a block-dictionary handle (MG_PREC_FP64_DICT), which keeps no
 * per-block values. */
int mg_level_export(const mg_handle* h, int32_t level, void* values, int8_t* row_exp);

/* Sizes of level `level`: nodes, block size, stored blocks. */
int mg_level_info(const mg_handle* h, int32_t level, int32_t* n_nodes, int32_t* block,
                  int64_t* nnzb);
int32_t mg_num_levels(const mg_handle* h);

/* Slot batch used on level `level`, the bytes per stored column index of its operators
 * (2 when the kernels read 16-bit offsets from a per-slot base: in every slice whose block
 * slots each span less than 2^16 columns, the others, at most 1/8 of the slots, reading
 * 32-bit indices; else 4), and the sweep times (microseconds per
 * launch) that the setup measured for the default and the other slot batch (0 when
 * slot_batch was fixed).  Any output pointer may be NULL. */
int mg_level_tuning(const mg_handle* h, int32_t level, int32_t* slot_batch, int32_t* col_bytes,
                    double* us_default, double* us_other);

/* Storage of the transfers between level `level` - 1 and `level` (level >= 1) on a
 * single-problem handle: bytes per stored column index of P~ and of R = P~^T, and bytes
 * per weight of P~.  (2, 2, 1): the node form (one lane per node; 16-bit column offsets
 * from a per-slot base and the weight code w * 128 packed with the column mask bits into
 * 32 bits), used when every weight is a multiple of 1/128 up to 255/128 (the weights of
 * nested box meshes) and every slot's columns span less than 2^16; else, level by level,
 * 4-byte columns and FP32 (4) weights when FP32 holds every weight exactly, FP64 (8)
 * otherwise.  Every form gives the same bits (Sec. 4.1:
 * prolongation and restriction as sparse products).  Any output pointer may be NULL. */
int mg_level_transfer_format(const mg_handle* h, int32_t level, int32_t* p_col_bytes, int32_t* r_col_bytes,
                             int32_t* weight_bytes);

/* Distinct blocks of level `level`'s operator in the dictionary form (MG_PREC_FP64_DICT
 * handles), or 0 when its values are stored plainly. */
int mg_level_dictionary(const mg_handle* h, int32_t level, int32_t* n_blocks);

/* Host-only structural validation of one level (and its coarser neighbour for P~);
 * no device is touched.  Returns MG_OK or MG_EINVAL with a message. */
int mg_validate_level(const mg_level_in* lv, const mg_level_in* coarser);

void mg_destroy(mg_handle* h);

/* ---- batched form: many independent problems, 1 or 8 right-hand sides each ----------
 * Every problem brings its own hierarchy (same block size for all).  Vectors of the batch
 * are the problems' vectors concatenated; inside problem p they are node-major with the
 * right-hand sides innermost: v[off[p] + (node * b + c) * nrhs + q], off from
 * mg_batch_offsets (n_problems + 1 entries).  Each step of the V-cycle runs as one launch
 * over all problems (levels aligned by depth below each problem's finest level); the
 * n_problems * nrhs FGMRES(m) instances run in lockstep, each with its own Hessenberg
 * matrix, Givens rotations and stopping test ||b_i - A x_i|| <= rtol ||b_i||; with
 * use_graph each Krylov step of the whole batch is one captured HIP graph.
 * Requirements: outer = MG_OUTER_FGMRES, coarse_mode = MG_COARSE_EXACT, smoother =
 * MG_SMOOTH_JACOBI, nrhs in {1, 8}
 * (8 for block size 1 only).  Mathematically every instance is the single-problem solve
 * of mg_solve (Algorithm "Geometric multigrid solver" inside GMRES, Sec. 4.2). */
typedef struct mg_batch mg_batch;
int mg_setup_batch(const mg_level_in* const* problems, const int32_t* n_levels, int32_t n_problems,
                   int32_t nrhs, const mg_config* cfg, int32_t inputs_on_device, void* stream,
                   mg_batch** out);
int mg_batch_offsets(const mg_batch* h, int64_t* offsets);
/* b, x: device FP64 batch vectors; x is the initial guess on entry.  stats: NULL or an
 * array of n_problems * nrhs entries (instance p * nrhs + q).  Returns MG_OK when every
 * instance converged, else MG_ENOCONV / MG_ENUMERIC (stats still filled). */
int mg_solve_batch(mg_batch* h, const double* b, double* x, mg_solve_stats* stats, void* stream);
void mg_destroy_batch(mg_batch* h);
/* ---- time stepping: Algorithm "Nonstationary Linear Problem" (Sec. 4) -------------
 * The operators of a handle are reused for every step; each step forms its right-hand
 * side on the device, solves with mg_solve from the previous solution, and maps the
 * solution back to nodal values.  For backward Euler with the lumped mass of eq.
 * mass_lumping (m_i = integral of phi_i) on the finest level,
 *   b_n = R [theta_{n-1} / dt + f_n ; g_n],  R = [Z H^T M_l | -Z H^T A_full E_g],
 *   A_L x_n = b_n (the handle's operator, which must hold the M_l / dt term),
 *   theta_n = H x_n, and theta_n = g_n on the Dirichlet DoFs,
 * with f_n the nodal source values, g_n the Dirichlet values of step n, H the
 * hanging-node interpolation, Z the mask of constrained DoFs, A_full the unconstrained
 * operator (mass term included) and E_g the injection of the Dirichlet DoFs.
 * mg_time_setup: n = n_L * b rows; R is scalar CSR with n rows over n + n_g columns
 * (columns < n address theta / dt + f, column n + k the k-th Dirichlet value), H is
 * scalar CSR n x n, g_idx the n_g Dirichlet DoFs (distinct, ascending not required).
 * Host arrays, deep-copied; the handle must outlive the time object and is used
 * by it (do not run other work on the handle concurrently).  MG_EINVAL for malformed
 * CSR, out-of-range indices, duplicate Dirichlet DoFs or dt <= 0. */
typedef struct mg_time mg_time;
int mg_time_setup(mg_handle* h, int32_t n_g, const int32_t* R_rowptr, const int32_t* R_col,
                  const double* R_val, const int32_t* H_rowptr, const int32_t* H_col,
                  const double* H_val, const int32_t* g_idx, double dt, void* stream, mg_time** out);
/* b = R [theta / dt + f ; g] (device FP64: theta, f, b of n entries, g of n_g; b must not
 * alias the inputs). */
int mg_time_rhs(mg_time* t, const double* theta, const double* f, const double* g, double* b, void* stream);
/* theta = H x, then theta[g_idx[k]] = g[k] (device FP64; theta must not alias x or g). */
int mg_time_theta(mg_time* t, const double* x, const double* g, double* theta, void* stream);
/* `steps` backward-Euler steps: F holds f_1 .. f_steps (steps * n, device), G holds
 * g_1 .. g_steps (steps * n_g, device); theta (n, device) is theta_0 on entry and
 * theta_steps on exit; x (n, device) is the initial guess of the first solve on entry
 * (each later solve starts from the previous solution) and x_steps on exit.  history:
 * NULL or steps * n device doubles receiving theta_1 .. theta_steps.  stats: NULL or
 * `steps` entries.  Stops at the first step whose solve fails (its code is returned,
 * the stats of that step are filled). */
int mg_time_run(mg_time* t, int32_t steps, double* theta, const double* F, const double* G, double* x,
                double* history, mg_solve_stats* stats, void* stream);
void mg_time_destroy(mg_time* t);

/* ---- explicit pressure correction: Algorithm "The fully discrete solution procedure for
 * the Navier-Stokes equations" (Sec. 5.3) ------------------------------------------------
 * Velocity Q1 on n_v nodes (3 components, node-major), pressure Q1 on n_p nodes; lumped
 * masses m_v, m_p (eq. mass_lumping).  Per step, with k = dt and s = p + q:
 *   Step 1: u_ic <- k / m_i (m_i (f_ic + u_ic / k) - nu (K u_c)_i + sum_a (C_a (u_a u_c))_i
 *           + (G_c s)_i) on free DoFs, the Dirichlet value on the others (eq. tp gives the
 *           nodal products u_a u_c, eq. multC their C_a products);
 *   Step 2: q solves K_p q = -(1/k) D u (GMRES + V-cycle on the caller's pressure
 *           hierarchy, from the previous q; zero right-hand side on its constrained
 *           nodes), D u = sum_a D_a u_a;
 *   Step 3: p <- p + q - nu D u / m_p.
 * Matrices (host CSR, deep-copied at setup): K and C_a = (phi_j, d_a phi_i) on one
 * n_v x n_v pattern; G_a = (phi^p_q, d_a phi^v_i) (n_v x n_p) on one pattern; D_a = G_a^T
 * (n_p x n_v) on one pattern.  dir_mask / dir_val: n_v * 3.  The pressure handle must be
 * an FP64 scalar hierarchy with n_p finest nodes; it stays owned by the caller and must
 * outlive the object. */
typedef struct {
  int32_t n_v, n_p;
  const int32_t *V_rowptr, *V_col;
  const double* K_val;
  const double* C_val[3];
  const int32_t *G_rowptr, *G_col;
  const double* G_val[3];
  const int32_t *D_rowptr, *D_col;
  const double* D_val[3];
  const double *m_v, *m_p;
  const uint8_t* dir_mask;
  const double* dir_val;
  double nu, dt;
} mg_ns_in;
typedef struct mg_ns mg_ns;
int mg_ns_setup(const mg_ns_in* in, mg_handle* pressure, void* stream, mg_ns** out);
/* Step 1 into u_out (device, n_v * 3; must not alias u); f: n_v * 3 or NULL (no forcing) */
int mg_ns_momentum(mg_ns* t, const double* u, const double* p, const double* q, const double* f, double* u_out,
                   void* stream);
/* du = D u and rhs = -(1/k) du (0 on the pressure hierarchy's constrained nodes) */
int mg_ns_divergence(mg_ns* t, const double* u, double* du, double* rhs, void* stream);
/* Step 3 in place: p <- p + q - nu du / m_p */
int mg_ns_pressure_update(mg_ns* t, double* p, const double* q, const double* du, void* stream);
/* `steps` time steps: u, p, q (device) in/out; stats: NULL or `steps` entries (the
 * pressure solves).  Stops at the first failing solve and returns its code. */
int mg_ns_run(mg_ns* t, int32_t steps, double* u, double* p, double* q, const double* f, mg_solve_stats* stats,
              void* stream);
void mg_ns_destroy(mg_ns* t);

/* ---- GPU-side assembly of the constrained Q1 operators on adaptive meshes -----------
 * A = Z (H^T A_full H) Z + I_C (Sec. 2.2: hanging nodes through the interpolation H,
 * constrained DoFs eliminated with identity rows / columns), the assembly the paper keeps
 * on the CPU ("init", Sec. 5.1; Sec. 6).  mg_asm_setup takes the mesh once: the leaves
 * (2^dim corner nodes each, bit k of the corner index = offset along axis k, and the
 * edge length), the hanging nodes with up to 4 masters and weights (powers of two, as on
 * box meshes: 1/2 on edges, 1/4 on faces), the DoF mask and the BSR pattern of A (sorted
 * columns per row; blocks the mesh does not reach stay zero); at most 32 distinct cell
 * sizes.  mg_asm_values then fills the nnzb * b * b block values (device FP64, block
 * row-major) for the given coefficients entirely on the GPU: element matrices of every
 * cell size from the tensor-product formulas, then one gather per stored block in a fixed
 * order (no atomics; repeated calls are bitwise identical).  Host inputs, deep-copied. */
enum { MG_ASM_POISSON = 0, MG_ASM_TD = 1, MG_ASM_ELASTICITY = 2 };
typedef struct {
  int32_t pde;                /* MG_ASM_*: (grad u, grad v); eps (grad u, grad v) + (b.grad u, v)
                                 [+ streamline term]; 2 mu (eps(u), eps(v)) + lam (div u, div v) */
  int32_t supg;               /* transport-diffusion: 1 = streamline stabilisation tau_K (b.grad u,
                                 b.grad v), tau_K = h_K/(2|b|)(coth Pe - 1/Pe), Pe = |b| h_K/(2 eps) */
  double eps, bvec[3];
  double lam, mu;
  double mass_coef;           /* c of a lumped-mass term c M_l (eq. mass_lumping); 0 = none */
} mg_asm_coef;
typedef struct {
  int32_t dim, block;         /* 2 or 3; 1 (Laplace / transport-diffusion) or dim (elasticity) */
  int32_t n_nodes, n_cells;
  const int32_t* cell_corner; /* n_cells * 2^dim */
  const double* cell_size;    /* n_cells */
  int32_t n_hanging;
  const int32_t* hang_node;   /* n_hanging */
  const int32_t* hang_master; /* n_hanging * 4, -1 = unused */
  const double* hang_weight;  /* n_hanging * 4 */
  const uint8_t* dof_mask;    /* n_nodes * block, 1 = constrained */
  int64_t nnzb;
  const int32_t* A_rowptr;    /* n_nodes + 1 */
  const int32_t* A_col;       /* nnzb */
} mg_asm_in;
typedef struct mg_asm mg_asm;
int mg_asm_setup(const mg_asm_in* in, void* stream, mg_asm** out);
/* val: device, nnzb * block * block doubles; enqueued on `stream`, nothing synchronised */
int mg_asm_values(mg_asm* a, const mg_asm_coef* coef, double* val, void* stream);
void mg_asm_destroy(mg_asm* a);

const char* mg_status_string(int status);
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
