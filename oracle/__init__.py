"""CPU FP64 oracle for the deflated-CG pseudo-stress Stokes solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code, header, table or
layout with the HIP library; the two meet only through the seeded input
generators in ``dcg_workloads``.

Layout: the paper's component-major ordering (Section 3.1, the d = 2 block
structure): a tensor vector is ``[sigma_11 | sigma_12 | sigma_21 | sigma_22]``,
each block a scalar DG-Q1 vector of length ``4 * n * n`` indexed ``4 e + j``
with ``e = ey * n + ex`` and local corner ``j = ix + 2 iy``.

Modules
-------
discretisation  DG-Q1 assembly of M, the div-div SIPG form A, A* = M + alpha A,
                the deflation basis V and an independently written scalar SIPG
                Laplacian (Sections 2.2-3.3, eq. (Vmatrix), Corollary 1).
multigrid       nested 2x2-agglomeration transfers, Galerkin hierarchy, RAS
                smoother, W-cycle and the Multigrid iteration
                (Section 4.2, Algorithms 3 and 4).
discretisation3d  the d = 3 forms on hexahedra (Section 3.1 for d = 3, Corollary 1).
multigrid3d     the three-dimensional hierarchy (2x2x2 agglomeration, trilinear
                transfers, RAS blocks of a cube and its face neighbours) for the
                same W-cycle (Section 4.2, the 3D case).
krylov          CG, deflated CG and FCG(m) (Section 4.1, eqs. (x_defl),
                (defl_sys), (fixed_tol), (tol), Algorithms 1 and 2), with an
                optional preconditioner in the flexible form.
precond         multigrid on A* itself (tensor Galerkin hierarchy, RAS blocks of
                a square and its edge neighbours) as that preconditioner: the
                outer multigrid the paper's conclusions leave to future work.
timestep        BDF2 right-hand side for a time-stepping run (Section 2.3).

Every function cites the passage it follows.  Parity status of each function
(pinned / unpinned) is listed in the module docstrings.
"""
