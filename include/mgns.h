/*
 * mgns.h - native generator of the explicit pressure-correction workload (host only).
 *
 * Sec. 5.3 (Navier-Stokes equations), Algorithm "The fully discrete solution procedure
 * for the Navier-Stokes equations": driven cavity on (0,L0) x (0,L1) x (0,L2), pressure
 * Q1 on a graded tensor grid Omega_h, velocity Q1 on its equidistant refinement
 * Omega_{h/2} (the Q1-iso-Q2 / Q1 pair), lumped masses (eq. mass_lumping), the
 * convective term through the matrices C_a = (phi_j, d_a phi_i) (eq. multC).
 *
 * Grading (Sec. 5.3, ascending order): x_i = L0 (1 - cos(i pi / N0)) / 2, likewise y;
 * z_k = L2 (1 + sin((k - N2) pi / (2 N2))).  Node numbers are lexicographic with x
 * fastest: node (i, j, k) = (k ny + j) nx + i.  Every matrix is exact for Q1 on boxes:
 * sums of Kronecker products of the one-dimensional P1 mass, stiffness and derivative
 * matrices, and G_a = C_a P with P the nodal interpolation of the pressure hat
 * functions in the velocity hat functions.
 *
 * Built:
 *   velocity (n_v nodes, one CSR pattern): K = (grad phi_j, grad phi_i), C_x, C_y, C_z;
 *     lumped mass m_v; Dirichlet mask / values of the 3 components on every boundary node
 *     (u = (0, 1, 0) on the face x = L0, 0 elsewhere); node coordinates;
 *   coupling: G_a (n_v x n_p) = (phi^p_q, d_a phi^v_i) and D_a = G_a^T (n_p x n_v);
 *   pressure: lumped mass m_p and the multigrid hierarchy of the pressure Laplacian
 *     (levels by uniform coarsening of the tensor grid, every other coordinate), node 0
 *     pinned on every level (identity row and column: the Neumann problem fixes the
 *     pressure increment up to a constant), scalar prolongations by tensor-product
 *     nodal interpolation; the level views are those of mggen.h.
 *
 * Ownership and errors as in mggen.h: the problem owns every array; views stay valid
 * until mgns_free(); errors are negative MGGEN_* codes with a message in
 * mgns_last_error().
 */
#ifndef MGNS_H
#define MGNS_H

#include <stdint.h>

#include "mggen.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t cells[3];            /* pressure-mesh cells per axis (each divisible by 2^(n_levels-1)) */
  double length[3];            /* domain edge lengths */
  int32_t n_levels;            /* pressure multigrid levels, >= 1 */
} mgns_config;

typedef struct {
  int32_t n_v, n_p;            /* velocity nodes, pressure nodes */
  int64_t v_nnz;
  const int32_t* V_rowptr;     /* n_v + 1 */
  const int32_t* V_col;        /* v_nnz, sorted per row */
  const double* K_val;         /* velocity Laplacian */
  const double* C_val[3];      /* C_x, C_y, C_z */
  int64_t g_nnz;
  const int32_t* G_rowptr;     /* n_v + 1 */
  const int32_t* G_col;        /* pressure nodes, sorted */
  const double* G_val[3];
  int64_t d_nnz;
  const int32_t* D_rowptr;     /* n_p + 1 */
  const int32_t* D_col;        /* velocity nodes, sorted */
  const double* D_val[3];
  const double* m_v;           /* n_v */
  const double* m_p;           /* n_p */
  const uint8_t* dir_mask;     /* n_v * 3, 1 = Dirichlet velocity DoF */
  const double* dir_val;       /* n_v * 3 */
  const double* coords_v;      /* n_v * 3 */
} mgns_view;

typedef struct mgns_problem mgns_problem;

int mgns_build(const mgns_config* cfg, mgns_problem** out);
int mgns_operators(const mgns_problem* p, mgns_view* out);
int32_t mgns_num_levels(const mgns_problem* p);
/* pressure level `level` (0 = coarsest) in the mggen level layout (block 1; the
 * hanging-node and lattice fields are empty) */
int mgns_pressure_level(const mgns_problem* p, int32_t level, mggen_level_view* out);
void mgns_free(mgns_problem* p);
const char* mgns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
