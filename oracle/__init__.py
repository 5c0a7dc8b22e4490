"""Plain FP64 CPU oracle for the adaptive-Q1 geometric multigrid hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports, calls or links this
package; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
do.  It shares no code with the native generator or the HIP kernels: the two sides meet
only through the seeded inputs in `workloads`.

Modules, in the order the method uses them:
  mesh       forest of quad/hex cells, refinement, 2:1 balance, nodes, hanging nodes,
             the hanging-node matrix H, global coarsening          (Sec. 2.2)
  fem        Q1 element matrices by Gauss quadrature, assembly, constraint elimination
             A = Z (H^T A_full H) Z + I_C, load vectors             (Sec. 2.1, 2.2)
  transfer   prolongation P~ = Q H_c from the coarse nodal basis, masks, R = P^T
             (Sec. 4.1 "Geometric Multigrid CUDA", eq. "prolongation")
  hierarchy  the level hierarchy of one workload
  multigrid  damped Jacobi / nodal block-Jacobi smoother, coarse solve, V-cycle
             (Algorithm "Geometric multigrid solver"), MG iteration, FGMRES with
             modified Gram-Schmidt and Givens rotations (Sec. 4.2)
  codec      FP16 / BF16 storage of matrix values with power-of-two row scales
Every function states the passage it follows.  Parity pins: see tests/test_oracle_*.py.
"""
