"""Multigrid on A* as the preconditioner of the outer iteration (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's conclusions name a multigrid preconditioner for the outer
iteration, to make its count independent of h, as future work.  This module
writes that idea out with the paper's own ingredients: the W-cycle of
Algorithm 4 with the RAS smoother of Section 4.2, applied to the full
operator A* = M + alpha A (eq. (pb_study)) instead of the inner Laplacian,
and used as B ~ (A*)^{-1} inside the flexible CG of Algorithm 1 on the
deflated system (``krylov.dcg(..., outer='fcg', precond=B)``: the direction
is built from z_i = B(r_i) in place of r_i).

Readings (the paper prints none of this):
* Hierarchy: a level's tensor DG-Q1 space is four copies of the scalar one,
  so the prolongation is I_4 (x) P in the component-major order of the
  oracle (each stress component injected as in the scalar hierarchy), and
  A*_{k-1} = P^T A*_k P (the Galerkin rule of Algorithm 2).  The coarsest
  level has ``coarsest`` x ``coarsest`` squares (8 by default) and is solved
  exactly by a dense Cholesky factorisation.
* RAS blocks: the definition of Section 4.2 applied to A*'s unknowns, one
  block per square: all four components on the square and on its edge
  neighbours, D = 1 / (number of blocks holding the dof).
* B(r) is one W-cycle from zero with m pre- and m post-smoothing steps.  The
  RAS smoother is not symmetric, so B enters the flexible form of the outer
  iteration only.

Parity status: pinned.  The tensor prolongation against the scalar one and
on bilinear fields, the Galerkin products of M and A against direct coarse
assembly (fine penalty), the partition of unity and block sizes, the
two-grid W-cycle against its error-propagation matrix, the flexible outer
iteration with the exact inverse as B (one iteration) and with the identity
(the unpreconditioned iterates), and the multigrid-preconditioned solve
against the direct solution are checked in tests/test_oracle_precond.py.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import multigrid
from .discretisation import element_index

N_COMP = 4
COARSEST_N = 8


def prolongation(n_coarse):
    """I_4 (x) P: the scalar injection of each stress component."""
    return sp.kron(sp.identity(N_COMP), multigrid.prolongation(n_coarse)).tocsr()


def ras_blocks(n_k):
    """One block per square (Section 4.2): the four components on the square
    and its edge neighbours.  Returns (dof index arrays, weights D_i)."""
    m = 4 * n_k * n_k
    blocks = []
    for ey in range(n_k):
        for ex in range(n_k):
            squares = [(ex, ey)] + [(ex + dx, ey + dy) for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1))
                                    if 0 <= ex + dx < n_k and 0 <= ey + dy < n_k]
            blocks.append(np.array([c * m + 4 * element_index(n_k, x, y) + j
                                    for c in range(N_COMP) for x, y in squares for j in range(4)]))
    count = np.zeros(N_COMP * m)
    for dofs in blocks:
        count[dofs] += 1.0
    return blocks, [1.0 / count[dofs] for dofs in blocks]


class Hierarchy:
    """A*_J given, A*_{k-1} = P_k^T A*_k P_k, RAS smoothers on levels k >= 2
    and a Cholesky factor on level 1: the attributes the W-cycle of
    ``multigrid`` reads (A, P, S, chol, J, n)."""

    def __init__(self, Astar, n, coarsest=COARSEST_N):
        self.J = multigrid.num_levels(n, coarsest)
        self.n = {self.J: n}
        self.A = {self.J: sp.csr_matrix(Astar)}
        self.P = {}
        for k in range(self.J, 1, -1):
            self.P[k] = prolongation(self.n[k] // 2)
            self.n[k - 1] = self.n[k] // 2
            self.A[k - 1] = (self.P[k].T @ self.A[k] @ self.P[k]).tocsr()
        self.S = {k: multigrid.RAS(self.A[k], *ras_blocks(self.n[k])) for k in range(2, self.J + 1)}
        self.chol = sla.cho_factor(self.A[1].toarray(), lower=True)


def preconditioner(H, m=2):
    """B(r) = Wcycle_J(r, 0) on the hierarchy of A* (Algorithm 4)."""
    def apply(r):
        return multigrid.wcycle(H, r, np.zeros_like(r), H.J, m, m)
    return apply
