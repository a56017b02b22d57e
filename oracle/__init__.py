"""Plain FP64 CPU oracle for the matrix-free multigrid hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never calls it and shares no code
with it; the only common module is ``synth`` (seeded inputs, no arithmetic).

What it computes (paper: Munch, Heister, Prieto Saavedra, Kronbichler,
"Efficient distributed matrix-free multigrid methods on locally refined meshes
for FEM computations", arXiv 2203.12292):

* ``octree``  — the test meshes (Section 4 "Examples"), the one-irregularity
  closure, and the global-coarsening level sequence (Section 2.2).
* ``fe``      — Q_k Lagrange elements on Gauss-Lobatto nodes, Gauss
  quadrature with (k+1)^3 points (Section 5 set-up), element matrices.
* ``space``   — free DoFs, hanging-node and Dirichlet constraints
  x_i = sum_j c_ij x_j (Section 3.1), the condensed stiffness matrix
  A = sum_e C_e^T A_e C_e (the plain definition behind Eq. (impl:mf)), load
  vectors, and the prolongation P (Section 3.5) with R = P^T.
* ``solvers`` — Chebyshev-Jacobi smoothing (Section 3.3), the V-cycle of
  Algorithms 1-2 (global-coarsening branch), CG preconditioned by one V-cycle
  (Section 2), direct solves.
* ``local_smoothing`` — the local-smoothing levels (all cells of one
  refinement level), their refinement-edge split, the copy to and from the
  levels, and the local-smoothing branch of Algorithms 1-2 (Section 2.1).
* ``mlp``     — the per-coarse-cell network of the learned coarse correction
  (forward, backward, Adam) in FP64.

Every function is written for clarity, not speed: dense or scipy sparse
matrices, Python loops over cells.  Pins that tie it to the paper and to
mathematics other than itself live in ``tests/test_oracle_*.py``.
"""
