"""W-cycle multigrid with a Restricted Additive Schwarz smoother in three
dimensions (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The inner system of the d = 3 deflated CG, V^T A* V = (alpha/3) L with L the
scalar SIPG Laplacian of the hexahedral DG-Q1 space (Corollary 1), solved by
the Multigrid iteration of Algorithm 3 with the W-cycle of Algorithm 4 and a
RAS smoother (Section 4.2); the 3D runs of Section 4.2 use m = 10 pre- and
post-smoothing steps on three nested levels.  The cycle itself is the one of
the two-dimensional oracle (``multigrid.wcycle`` / ``multigrid.multigrid``:
smoothing, a coarse correction of gamma = 2 cycles, smoothing, an exact
solve on level 1); this module supplies the three-dimensional hierarchy.

Readings (the paper's 3D hierarchy nests tetrahedral meshes in a finite
element package; this module takes the hexahedral analogue):
* Levels: the finest grid has n^3 cubes, each coarser level agglomerates
  2 x 2 x 2 cubes, level 1 has ``coarsest``^3 cubes (2 by default: the
  coarsest of the paper's three nested meshes refines the unit cube twice
  per direction), J = log2(n / coarsest) + 1.
* Coarse spaces are DG-Q1 on the agglomerated cubes.  They are nested, so the
  L2-projection prolongation is the exact injection of a coarse trilinear
  function into its eight children (coefficients products of {1, 1/2, 0}
  per axis) and the Galerkin operators are P^T A P.
* RAS blocks: one block per cube, the cube and every cube sharing a face
  with it (Section 4.2: an element with its immediate neighbours, one layer
  of overlap), clipped at the boundary; ``core`` > 1 groups core^3 cubes
  around which the face layer is taken (the two-dimensional build's tiles).
  D_i = 1 / (number of blocks holding the dof).
* The local problems and the coarsest problem are solved exactly (a library
  inverse; a dense Cholesky factorisation on level 1).

Parity status: pinned.  Prolongation exactness on trilinear functions and
its injection of single-cube coarse functions, the Galerkin identity against
direct coarse assembly with the fine penalty, the partition of unity and the
block sizes, the RAS special cases (one block = exact solve; single cubes
without overlap = block Jacobi), the coarsest Cholesky, the two- and
three-level W-cycles against their dense error-propagation matrices, and the
Multigrid iteration reaching its tolerance are checked in
tests/test_oracle_multigrid3d.py.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .discretisation3d import element_index
from .multigrid import RAS

NB = 8
COARSEST_N = 2
FACE_NEIGHBOURS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


def num_levels(n, coarsest=COARSEST_N):
    """J such that level k has n / 2^(J-k) cubes per side, level 1 ``coarsest``."""
    if coarsest < 1 or n < coarsest or n % coarsest:
        raise ValueError("n must be coarsest times a power of two")
    ratio = n // coarsest
    if ratio & (ratio - 1):
        raise ValueError("n must be coarsest times a power of two")
    return int(np.log2(ratio)) + 1


def prolongation(n_coarse):
    """I_{k-1}^k: DG-Q1 on n_coarse^3 cubes -> DG-Q1 on (2 n_coarse)^3.

    Fine corner (ix, iy, iz) of child (cx, cy, cz) sits at the reference point
    ((cx + ix)/2, (cy + iy)/2, (cz + iz)/2) of its parent; its coefficient is
    the parent's trilinear function evaluated there."""
    nf = 2 * n_coarse
    rows, cols, vals = [], [], []
    for EZ in range(n_coarse):
        for EY in range(n_coarse):
            for EX in range(n_coarse):
                E = element_index(n_coarse, EX, EY, EZ)
                for c in range(8):
                    cx, cy, cz = c % 2, (c // 2) % 2, c // 4
                    e = element_index(nf, 2 * EX + cx, 2 * EY + cy, 2 * EZ + cz)
                    for j in range(NB):
                        p = ((cx + j % 2) / 2.0, (cy + (j // 2) % 2) / 2.0, (cz + j // 4) / 2.0)
                        for J in range(NB):
                            bits = (J % 2, (J // 2) % 2, J // 4)
                            v = 1.0
                            for t, b in zip(p, bits):
                                v *= t if b else 1.0 - t
                            if v != 0.0:
                                rows.append(NB * e + j)
                                cols.append(NB * E + J)
                                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(NB * nf ** 3, NB * n_coarse ** 3))


def ras_blocks(n_k, core=1, layer=True):
    """Blocks B_i of the RAS smoother on an n_k^3 grid (Section 4.2): core^3
    cubes plus, with ``layer``, every cube outside the core that shares a
    face with it.  Returns (list of dof index arrays, list of weights D_i)."""
    if n_k % core:
        raise ValueError("grid not divisible into cores")
    blocks = []
    for bz in range(0, n_k, core):
        for by in range(0, n_k, core):
            for bx in range(0, n_k, core):
                cubes = [(x, y, z) for z in range(bz, bz + core) for y in range(by, by + core)
                         for x in range(bx, bx + core)]
                inside = set(cubes)
                ring = []
                if layer:
                    for x, y, z in cubes:
                        for dx, dy, dz in FACE_NEIGHBOURS:
                            q = (x + dx, y + dy, z + dz)
                            if q in inside or q in ring:
                                continue
                            if all(0 <= c < n_k for c in q):
                                ring.append(q)
                dofs = np.array([NB * element_index(n_k, *q) + j for q in cubes + ring
                                 for j in range(NB)])
                blocks.append(dofs)
    count = np.zeros(NB * n_k ** 3)
    for dofs in blocks:
        count[dofs] += 1.0
    return blocks, [1.0 / count[dofs] for dofs in blocks]


class Hierarchy:
    """{Z_k}: Z_J given, Z_{k-1} = P_k^T Z_k P_k (Algorithm 2), RAS smoothers
    on levels k >= 2 and a Cholesky factor on level 1 -- the attributes the
    W-cycle of ``multigrid`` reads (A, P, S, chol, J, n)."""

    def __init__(self, ZJ, n, coarsest=COARSEST_N, core=1, layer=True):
        self.J = num_levels(n, coarsest)
        self.n = {self.J: n}
        self.A = {self.J: sp.csr_matrix(ZJ)}
        self.P = {}
        for k in range(self.J, 1, -1):
            nk = self.n[k]
            self.P[k] = prolongation(nk // 2)
            self.n[k - 1] = nk // 2
            self.A[k - 1] = (self.P[k].T @ self.A[k] @ self.P[k]).tocsr()
        self.S = {k: RAS(self.A[k], *ras_blocks(self.n[k], min(core, self.n[k]), layer))
                  for k in range(2, self.J + 1)}
        self.chol = sla.cho_factor(self.A[1].toarray(), lower=True)
