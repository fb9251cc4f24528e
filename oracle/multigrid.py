"""W-cycle multigrid with a Restricted Additive Schwarz smoother (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 4.2 and Algorithms 3 (Multigrid) and 4 (Wcycle), with the
Galerkin hierarchy of Algorithm 2 (each coarse operator is the fine one
multiplied by the prolongation on the right and its transpose on the left).
The W-cycle is written from its definition: smoothing by the Schwarz
operator, a coarse-grid correction made of gamma = 2 cycles of the next
coarser level, smoothing again; the exact solve on level 1.

Readings where the paper is silent or written for other meshes:
* Levels: the finest grid has n x n squares, each coarser level agglomerates
  2 x 2 squares, and the coarsest level k = 1 has 16 x 16 squares by default,
  so J = log2(n / 16) + 1; a shorter hierarchy (the four levels of the
  paper's experiments, Section 5) stops at a larger coarsest grid
  (``coarsest``), J = log2(n / coarsest) + 1, still solved exactly.
* Coarse spaces are DG-Q1 on the agglomerated squares.  They are nested, so
  the L2-projection prolongation of Section 4.2 is the exact injection of a
  coarse Q1 function into the four fine squares (coefficients in
  {1, 1/2, 1/4, 0}); for nested spaces its L2 adjoint acts on residual
  vectors as P^T, and the Galerkin product is P^T Z P.
* RAS blocks: 4 x 4-square cores extended by every square sharing an edge
  with the core (one layer of overlap, Section 4.2 "element and its
  immediate neighbours"), clipped at the boundary.  D_i = 1 / (number of
  blocks containing the dof), as in Section 4.2.
* The local problems (A_k)_i z_i = R_i r are solved with the explicit inverse
  of (A_k)_i (a library inverse), mathematically identical to any other
  exact local solve.
* The coarsest problem is solved exactly by a dense Cholesky factorisation.

Parity status: pinned.  Prolongation exactness on Q1 functions, the Galerkin
identity against direct coarse assembly, the partition of unity, the RAS
special cases (one block = exact solve; 1x1 non-overlapping blocks = block
Jacobi), the coarsest Cholesky and the two- and three-level W-cycles
against their dense error-propagation matrices are checked in
tests/test_oracle_multigrid.py.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .discretisation import element_index

COARSEST_N = 16


def num_levels(n, coarsest=COARSEST_N):
    """J such that level k has n / 2^(J-k) squares per side and level 1 has
    ``coarsest`` (16 unless a test asks for a smaller hierarchy)."""
    if n < coarsest or n % coarsest:
        raise ValueError("n must be 16 times a power of two")
    ratio = n // coarsest
    if ratio & (ratio - 1):
        raise ValueError("n must be 16 times a power of two")
    return int(np.log2(ratio)) + 1


def prolongation(n_coarse):
    """I_{k-1}^k: DG-Q1 on n_coarse^2 squares -> DG-Q1 on (2 n_coarse)^2.

    Fine corner (ix, iy) of child (cx, cy) sits at reference point
    ((cx + ix)/2, (cy + iy)/2) of its parent, so its coefficient is the
    parent's bilinear function evaluated there."""
    nf = 2 * n_coarse
    rows, cols, vals = [], [], []
    for EY in range(n_coarse):
        for EX in range(n_coarse):
            E = element_index(n_coarse, EX, EY)
            for cy in range(2):
                for cx in range(2):
                    e = element_index(nf, 2 * EX + cx, 2 * EY + cy)
                    for j in range(4):
                        xi, eta = (cx + j % 2) / 2.0, (cy + j // 2) / 2.0
                        for J in range(4):
                            JX, JY = J % 2, J // 2
                            v = (xi if JX else 1.0 - xi) * (eta if JY else 1.0 - eta)
                            if v != 0.0:
                                rows.append(4 * e + j)
                                cols.append(4 * E + J)
                                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(4 * nf * nf, 4 * n_coarse * n_coarse))


def ras_blocks(n_k, tile=4, layer=True):
    """Blocks B_i of the RAS smoother on an n_k x n_k grid (Section 4.2).

    Returns (list of dof index arrays, list of weight arrays D_i)."""
    if n_k % tile:
        raise ValueError("grid not divisible into tiles")
    blocks = []
    for b in range(n_k // tile):
        for a in range(n_k // tile):
            elems = [(ex, ey) for ey in range(tile * b, tile * b + tile)
                     for ex in range(tile * a, tile * a + tile)]
            if layer:
                ring = []
                for ey in range(tile * b, tile * b + tile):
                    ring += [(tile * a - 1, ey), (tile * a + tile, ey)]
                for ex in range(tile * a, tile * a + tile):
                    ring += [(ex, tile * b - 1), (ex, tile * b + tile)]
                elems += [(ex, ey) for ex, ey in ring if 0 <= ex < n_k and 0 <= ey < n_k]
            dofs = np.array([4 * element_index(n_k, ex, ey) + j for ex, ey in elems for j in range(4)])
            blocks.append(dofs)
    count = np.zeros(4 * n_k * n_k)
    for dofs in blocks:
        count[dofs] += 1.0
    weights = [1.0 / count[dofs] for dofs in blocks]
    return blocks, weights


class RAS:
    """S_k = sum_i R_i^T D_i (A_k)_i^{-1} R_i (Section 4.2)."""

    def __init__(self, A, blocks, weights):
        A = sp.csr_matrix(A)
        self.size = A.shape[0]
        # blocks of equal size are stacked so that the local solves run as one
        # batched product; the arithmetic per block is unchanged
        self.groups = []
        sizes = sorted({len(d) for d in blocks})
        for s in sizes:
            sel = [i for i, d in enumerate(blocks) if len(d) == s]
            idx = np.stack([blocks[i] for i in sel])
            w = np.stack([weights[i] for i in sel])
            local = np.stack([A[blocks[i]][:, blocks[i]].toarray() for i in sel])
            self.groups.append((idx, w, np.linalg.inv(local)))

    def apply(self, r):
        z = np.zeros(self.size)
        for idx, w, inv in self.groups:
            y = w * np.matmul(inv, r[idx][..., None])[..., 0]       # D_i (A_k)_i^{-1} R_i r
            z += np.bincount(idx.ravel(), weights=y.ravel(), minlength=self.size)  # sum R_i^T
        return z


class Hierarchy:
    """{Z_k}: Z_J given, Z_{k-1} = P_k^T Z_k P_k (Algorithm 2), with RAS
    smoothers on levels k >= 2 and a Cholesky factor on level 1."""

    def __init__(self, ZJ, n, tile=4, layer=True, coarsest=COARSEST_N):
        self.J = num_levels(n, coarsest)
        self.n = {self.J: n}
        self.A = {self.J: sp.csr_matrix(ZJ)}
        self.P = {}
        for k in range(self.J, 1, -1):
            nk = self.n[k]
            self.P[k] = prolongation(nk // 2)
            self.n[k - 1] = nk // 2
            self.A[k - 1] = (self.P[k].T @ self.A[k] @ self.P[k]).tocsr()
        self.S = {k: RAS(self.A[k], *ras_blocks(self.n[k], tile, layer)) for k in range(2, self.J + 1)}
        self.chol = sla.cho_factor(self.A[1].toarray(), lower=True)


def smooth(H, k, f, z, steps):
    """``steps`` RAS smoothing steps z <- z + S_k (f - A_k z) on level k
    (Section 4.2: the smoother is the Schwarz operator S_k applied to the
    current residual)."""
    for _ in range(steps):
        z = z + H.S[k].apply(f - H.A[k] @ z)
    return z


def coarse_correction(H, k, residual, m1, m2, gamma=2):
    """Correction from level k - 1 for the level-k residual (Section 4.2).

    The residual is restricted with P_k^T, the coarse problem
    A_{k-1} c = P_k^T residual is approximated by ``gamma`` successive
    level-(k-1) cycles started from c = 0 (gamma = 2: the W-cycle), and the
    result is prolongated with P_k.  On level 1 a cycle is the exact solve,
    so every repetition returns the same vector."""
    rhs = H.P[k].T @ residual
    c = np.zeros_like(rhs)
    for _ in range(gamma):
        c = wcycle(H, rhs, c, k - 1, m1, m2)
    return H.P[k] @ c


def wcycle(H, f, z0, k, m1=2, m2=2):
    """One W-cycle for A_k z = f from the guess z0 (Algorithm 4): the exact
    solve on level 1, otherwise m1 smoothing steps, the coarse-grid
    correction with two coarse cycles, and m2 smoothing steps."""
    if k == 1:
        return sla.cho_solve(H.chol, f)
    z = smooth(H, k, f, z0.copy(), m1)
    z = z + coarse_correction(H, k, f - H.A[k] @ z, m1, m2)
    return smooth(H, k, f, z, m2)


def multigrid(H, f, z0=None, m1=2, m2=2, tol=1e-10, n_max=100):
    """Multigrid iteration (Algorithm 3): W-cycles while n < n_max and
    ||f - A_J z_n|| / ||f|| > tol.  Returns (z, n).  A zero right-hand side
    returns the zero vector after 0 cycles."""
    A = H.A[H.J]
    z = np.zeros_like(f) if z0 is None else z0.copy()
    fnorm = np.linalg.norm(f)
    if fnorm == 0.0:
        return np.zeros_like(f), 0
    n = 0
    while n < n_max and np.linalg.norm(f - A @ z) / fnorm > tol:
        z = wcycle(H, f, z, H.J, m1, m2)
        n += 1
    return z, n
