/*
 * mggen.h - native problem generator for the adaptive-Q1 multigrid library (host only).
 *
 * Builds, from a seeded workload description, everything the solver library's
 * mg_setup_hierarchy() consumes: per level l = 0 (coarsest) .. L (finest) the
 * constrained nodal-block operator A_l (BSR), the scalar prolongation P~_l from level
 * l-1 (CSR), the constrained-DoF mask, and the finest right-hand side.
 *
 * What it computes (paper, Sec. 2.1 and 2.2):
 *   - adaptive quadrilateral / hexahedral meshes on a box of coarse cells, a refined
 *     cell replaced by 2^d children, one level jump between neighbours (read over
 *     shared vertices), hanging nodes on edges (2 masters, 1/2) and faces (4 masters,
 *     1/4) replaced by interpolation through the square matrix H;
 *   - the multigrid hierarchy by global coarsening (families whose 2^d children are all
 *     leaves are coarsened together unless that breaks the one-level-jump rule);
 *   - Q1 operators A = Z (H^T A_full H) Z + I_C and loads b = Z H^T f, Z masking the
 *     constrained set C (hanging nodes, Dirichlet components);
 *   - P~ = Q H_coarse with Q_ij the coarse nodal basis at the fine nodes (Sec. 4.1,
 *     eq. "prolongation"); weights are exact dyadic numbers.
 * Node numbers follow the lexicographic (z, y, x) order of the lattice points.
 *
 * Ownership: mggen_build() returns a problem object that owns every array; views
 * returned by mggen_level() stay valid until mggen_free().  No function aborts: errors
 * are negative return codes with a message in mggen_last_error() (thread-local).
 */
#ifndef MGGEN_H
#define MGGEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MGGEN_OK = 0, MGGEN_EINVAL = -1, MGGEN_ENOMEM = -2, MGGEN_EINTERNAL = -3 };
enum { MGGEN_ROUND_UNIFORM = 0, MGGEN_ROUND_BAND = 1, MGGEN_ROUND_CORNER = 2 };
enum { MGGEN_PDE_POISSON = 0, MGGEN_PDE_TD = 1, MGGEN_PDE_ELASTICITY = 2, MGGEN_PDE_OSEEN = 3 };
enum { MGGEN_RHS_SINSIN = 0, MGGEN_RHS_DISK = 1, MGGEN_RHS_CONST = 2, MGGEN_RHS_FIELD = 3,
       MGGEN_RHS_NOISE = 4, MGGEN_RHS_NONE = 5 };

/* One refinement round.  UNIFORM: every leaf.  BAND (2D): every leaf whose closed box
 * meets the open annulus p[2]-p[3] < |x - (p[0],p[1])| < p[2]+p[3].  CORNER: every leaf of
 * the current maximum depth whose box lies in {x_a <= p[0] for every axis a in `axes`}.
 * Every round is followed by 2:1 balancing. */
typedef struct {
  int32_t kind;
  int32_t axes;
  double p[4];
} mggen_round;

typedef struct {
  int32_t dim;                 /* 2 or 3 */
  int32_t coarse[3];           /* coarse cells per axis (x, y, z) */
  double h0;                   /* coarse cell edge */
  int32_t n_rounds;
  const mggen_round* rounds;
  int32_t pde;                 /* MGGEN_PDE_* */
  int32_t block;               /* components per node: 1, 3 (elasticity) or 4 (p,u,v,w) */
  double eps;                  /* transport-diffusion: diffusion */
  double bvec[3];              /* transport-diffusion: constant convection */
  double lam, mu;              /* elasticity */
  double nu, dt, pspg_alpha;   /* flow step */
  int32_t dir_faces;           /* bit 2a: face x_a = 0, bit 2a+1: face x_a = max */
  int32_t dir_comps;           /* components constrained on Dirichlet faces */
  int32_t rhs;                 /* MGGEN_RHS_* */
  double rhs_const[4];
  /* flow-step fields: beta = scale * sum_k a_k 2 pi cos(2 pi kappa_k.x + phi_k) (kappa_k x e_{j_k}),
   * forcing = sum_m fc_m sin(2 pi fk_m.x + fphi_m) e_{fi_m} */
  double kappa[8][3], a[8], phi[8], scale;
  int32_t j[8];
  double fk[4][3], fc[4], fphi[4];
  int32_t fi[4];
  int32_t no_supg;             /* 1: no streamline stabilisation in the TD operator */
  double mass_coef;            /* c of a lumped mass term c M_l added to every level's
                                  operator (eq. mass_lumping: m_i = int phi_i); 0 = none */
  int32_t time_ops;            /* 1: also build the right-hand-side operators of a
                                  time-stepping run on the finest level (mggen_time_ops) */
} mggen_config;

typedef struct {
  int32_t n_nodes, block;
  int64_t nnzb;
  const int32_t* rowptr;       /* n_nodes + 1 */
  const int32_t* col;          /* nnzb, sorted per row */
  const double* val;           /* nnzb * block * block, block row-major */
  int32_t p_cols;              /* nodes of level l-1 (0 on level 0) */
  int64_t p_nnz;
  const int32_t* p_rowptr;     /* n_nodes + 1, or NULL on level 0 */
  const int32_t* p_col;
  const double* p_val;
  const uint8_t* dof_mask;     /* n_nodes * block, 1 = constrained */
  int32_t n_hanging;
  const int32_t* hang_node;    /* n_hanging */
  const int32_t* hang_master;  /* n_hanging * 4, -1 = unused */
  const double* hang_weight;   /* n_hanging * 4 */
  const int32_t* node_lattice; /* n_nodes * 3 lattice coordinates (x, y, z) */
  int32_t max_depth;
} mggen_level_view;

typedef struct mggen_problem mggen_problem;

int mggen_build(const mggen_config* cfg, mggen_problem** out);
int32_t mggen_num_levels(const mggen_problem* p);
int mggen_level(const mggen_problem* p, int32_t level, mggen_level_view* out);
/* finest right-hand side b = Z H^T f (n_nodes * block); NULL for MGGEN_RHS_NOISE */
const double* mggen_rhs(const mggen_problem* p);
/* b = Z H^T (m (*) xi) for nodal noise xi (n_nodes * nrhs, node-major), m the lumped mass
 * (block must be 1); out: n_nodes * nrhs, node-major */
int mggen_rhs_noise(const mggen_problem* p, const double* xi, int32_t nrhs, double* out);
/* Operators of a backward-Euler run with the lumped mass (Algorithm "Nonstationary Linear
 * Problem", Sec. 4; eq. mass_lumping), finest level, DoF = node * block + component:
 *   R (n_dofs x (n_dofs + n_g)) = [Z H^T M_l | -Z H^T A_full E_g], so that the right-hand
 *     side of a step is b = R [theta_old / dt + f ; g] (f nodal source values, g the
 *     Dirichlet values of the step); A_full is the unconstrained operator with its mass
 *     term, E_g injects the n_g Dirichlet DoFs g_idx;
 *   H (n_dofs x n_dofs): theta = H x (hanging DoFs interpolated; identity rows else);
 *   coords: n_nodes * dim node coordinates.
 * Available when the problem was built with time_ops = 1; views stay valid until
 * mggen_free(). */
typedef struct {
  int32_t n_dofs;
  int32_t n_g;
  int64_t r_nnz, h_nnz;
  const int32_t* R_rowptr;
  const int32_t* R_col;
  const double* R_val;
  const int32_t* H_rowptr;
  const int32_t* H_col;
  const double* H_val;
  const int32_t* g_idx;
  const double* coords;
} mggen_time_view;
int mggen_time_ops(const mggen_problem* p, mggen_time_view* out);
/* The leaves of level `level`: corner node numbers (n_cells * corners, corners = 2^dim;
 * bit k of the corner index is the offset along axis k) and edge lengths. */
typedef struct {
  int32_t n_cells, corners;
  const int32_t* corner;
  const double* size;
} mggen_cells_view;
int mggen_level_cells(const mggen_problem* p, int32_t level, mggen_cells_view* out);
void mggen_free(mggen_problem* p);
const char* mggen_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
