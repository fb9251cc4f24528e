"""Pins of the oracle's three-dimensional multigrid hierarchy and RAS
smoother (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import discretisation3d as d3
from oracle import krylov
from oracle import multigrid as mg
from oracle import multigrid3d as mg3

PEN = d3.DEFAULT_PENALTY


def test_num_levels():
    assert [mg3.num_levels(n) for n in (2, 4, 8, 32, 64)] == [1, 2, 3, 5, 6]
    assert [mg3.num_levels(n, c) for n, c in ((16, 4), (12, 3), (8, 8))] == [3, 3, 1]
    for n, c in ((6, 2), (3, 2), (2, 4)):
        with pytest.raises(ValueError):
            mg3.num_levels(n, c)


@pytest.mark.parametrize("fun", [lambda x, y, z: 1.0, lambda x, y, z: x, lambda x, y, z: z,
                                 lambda x, y, z: x * y * z,
                                 lambda x, y, z: 2 - x + 3 * y * z - 0.5 * x * z + 4 * x * y * z])
def test_prolongation_reproduces_trilinear_functions(fun):
    # nested Q1: a function trilinear on the whole domain is reproduced exactly
    nc = 3
    P = mg3.prolongation(nc)
    assert np.allclose(P @ d3.interpolate(nc, fun), d3.interpolate(2 * nc, fun), atol=1e-14)


def test_prolongation_evaluates_the_coarse_function_at_fine_nodes():
    # a random coarse DG-Q1 function, evaluated with the Q1 basis at the
    # reference point of each fine node inside its parent
    nc = 2
    rng = np.random.default_rng(7)
    q = rng.standard_normal(8 * nc ** 3)
    fine = mg3.prolongation(nc) @ q
    h_f = 1.0 / (2 * nc)
    for e, xyz in enumerate(d3.node_coordinates(2 * nc).reshape(-1, 8, 3)):
        for j, p in enumerate(xyz):
            centre = p - 0.5 * h_f * (np.array(d3.corner(j)) - 0.5)   # inside the fine cube
            E = d3.element_index(nc, *(np.floor(centre * nc).astype(int)))
            ref_pt = p * nc - np.floor(centre * nc)
            val = sum(q[8 * E + J] * d3.q1_value(J, ref_pt) for J in range(8))
            assert abs(fine[8 * e + j] - val) <= 1e-14


def test_prolongation_injects_single_cube_functions():
    nc = 3
    P = mg3.prolongation(nc).toarray()
    E = d3.element_index(nc, 1, 2, 0)
    col = P[:, 8 * E:8 * E + 8]
    children = [d3.element_index(2 * nc, 2 + cx, 4 + cy, cz)
                for cz in range(2) for cy in range(2) for cx in range(2)]
    rows = np.concatenate([8 * e + np.arange(8) for e in children])
    mask = np.ones(P.shape[0], bool)
    mask[rows] = False
    assert np.all(col[mask] == 0.0)
    assert np.allclose(col[rows].sum(axis=1), 1.0)        # partition of unity inside
    assert set(np.unique(P)) <= {0.0, 0.125, 0.25, 0.5, 1.0}


def test_galerkin_product_equals_direct_coarse_assembly():
    # P^T L_h P is the SIPG Laplacian of the 2h grid with the fine penalty:
    # jumps of a coarse Q1 function vanish on fine faces inside a coarse cube,
    # coarse faces (and the outflow face) are unions of fine faces, and the
    # consistency terms of a coarse function are the same on either grid.
    nf = 8
    gamma_f = PEN * nf
    Lf = d3.sipg_laplacian(nf)
    P = mg3.prolongation(nf // 2)
    Lc = (P.T @ Lf @ P).toarray()
    direct = d3.sipg_laplacian(nf // 2, gamma=gamma_f).toarray()
    assert np.abs(Lc - direct).max() <= 1e-12 * np.abs(direct).max()
    P2 = mg3.prolongation(nf // 4)
    Lcc = (P2.T @ sp.csr_matrix(Lc) @ P2).toarray()
    direct2 = d3.sipg_laplacian(nf // 4, gamma=gamma_f).toarray()
    assert np.abs(Lcc - direct2).max() <= 1e-12 * np.abs(direct2).max()


@pytest.mark.parametrize("n_k", [4, 6])
def test_ras_partition_of_unity_and_block_sizes(n_k):
    blocks, weights = mg3.ras_blocks(n_k)
    assert len(blocks) == n_k ** 3
    total = np.zeros(8 * n_k ** 3)
    for dofs, w in zip(blocks, weights):
        total[dofs] += w
    assert np.allclose(total, 1.0, atol=1e-15)
    # a block is a cube and its face neighbours: 7 cubes inside, 4 at a corner
    assert sorted({len(b) // 8 for b in blocks}) == [4, 5, 6, 7]
    # a dof lies in the blocks of its cube and of each face neighbour
    inv = np.round(1.0 / np.concatenate(weights)).astype(int)
    assert set(inv) == {4, 5, 6, 7}
    corner = blocks[d3.element_index(n_k, 0, 0, 0)]
    assert set(corner // 8) == {d3.element_index(n_k, *c) for c in
                                ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1))}
    # cores of 2 x 2 x 2 cubes with their face layer: 8 + 24 cubes inside
    blocks2, _ = mg3.ras_blocks(n_k, core=2)
    assert max(len(b) for b in blocks2) == 8 * (8 + 24 if n_k >= 6 else 8 + 12)


def test_ras_single_block_is_exact_solve():
    n = 4
    L = d3.sipg_laplacian(n)
    S = mg.RAS(L, *mg3.ras_blocks(n, core=n))
    r = np.random.default_rng(1).standard_normal(L.shape[0])
    assert np.allclose(S.apply(r), np.linalg.solve(L.toarray(), r), rtol=1e-12, atol=1e-12)


def test_ras_single_cube_without_overlap_is_block_jacobi():
    n = 3
    L = d3.sipg_laplacian(n).toarray()
    S = mg.RAS(sp.csr_matrix(L), *mg3.ras_blocks(n, layer=False))
    r = np.random.default_rng(2).standard_normal(L.shape[0])
    ref = np.concatenate([np.linalg.solve(L[8 * e:8 * e + 8, 8 * e:8 * e + 8], r[8 * e:8 * e + 8])
                          for e in range(n ** 3)])
    assert np.allclose(S.apply(r), ref, atol=1e-13)


def test_ras_block_solve_is_the_local_dirichlet_problem():
    # the local solve of the block of cube c: the restriction of L to the
    # block's dofs, inverted (values outside the block held at zero)
    n = 4
    L = d3.sipg_laplacian(n).toarray()
    blocks, weights = mg3.ras_blocks(n)
    c = d3.element_index(n, 1, 2, 1)
    dofs = blocks[c]
    r = np.random.default_rng(3).standard_normal(L.shape[0])
    one = mg.RAS(sp.csr_matrix(L), [dofs], [weights[c]]).apply(r)
    y = np.linalg.solve(L[np.ix_(dofs, dofs)], r[dofs])
    assert np.allclose(one[dofs], weights[c] * y, atol=1e-13)
    assert np.allclose(np.delete(one, dofs), 0.0)
    assert np.allclose(weights[c][:8], 1.0 / 7.0)


def test_coarsest_cholesky_reconstructs_operator():
    n = 8
    H = mg3.Hierarchy(d3.sipg_laplacian(n), n)
    assert H.J == 3 and H.n == {3: 8, 2: 4, 1: 2}
    C = np.tril(H.chol[0])
    A1 = H.A[1].toarray()
    assert np.abs(C @ C.T - A1).max() <= 1e-13 * np.abs(A1).max()


def _dense_smoother(H, k):
    N = H.A[k].shape[0]
    S = np.zeros((N, N))
    for idx, w, inv in H.S[k].groups:
        for dofs, wi, Ai in zip(idx, w, inv):
            S[np.ix_(dofs, dofs)] += wi[:, None] * Ai
    return S


@pytest.mark.parametrize("m", [2, 10])
def test_two_grid_wcycle_equals_error_propagation_matrix(m):
    # J = 2: z -> z + (I - E_TG) A^{-1} (f - A z) with
    # E_TG = (I - S A)^m (I - P A_1^{-1} P^T A) (I - S A)^m  (Algorithm 4)
    n = 4
    H = mg3.Hierarchy(d3.sipg_laplacian(n), n)
    assert H.J == 2
    A = H.A[2].toarray()
    I = np.eye(len(A))
    smooth = np.linalg.matrix_power(I - _dense_smoother(H, 2) @ A, m)
    P = H.P[2].toarray()
    E = smooth @ (I - P @ np.linalg.solve(H.A[1].toarray(), P.T @ A)) @ smooth
    rng = np.random.default_rng(4)
    f, z = rng.standard_normal(len(A)), rng.standard_normal(len(A))
    ref = z + (I - E) @ np.linalg.solve(A, f - A @ z)
    out = mg.wcycle(H, f, z, 2, m, m)
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref)
    # a convergent cycle, contracting faster with more smoothing (0.85 and 0.52)
    assert max(abs(np.linalg.eigvals(E))) < (0.9 if m == 2 else 0.6)


def test_three_level_wcycle_equals_recursive_error_propagation():
    # gamma = 2: E_k = (I - S_k A_k)^m (I - P_k (I - E_{k-1}^2) A_{k-1}^{-1}
    # P_k^T A_k) (I - S_k A_k)^m, E_1 = 0 (Algorithm 4)
    n, m = 4, 2
    H = mg3.Hierarchy(d3.sipg_laplacian(n), n, coarsest=1)
    assert H.J == 3
    E_prev = np.zeros((H.A[1].shape[0],) * 2)
    for k in (2, 3):
        A = H.A[k].toarray()
        I = np.eye(len(A))
        Ic = np.eye(H.A[k - 1].shape[0])
        smooth = np.linalg.matrix_power(I - _dense_smoother(H, k) @ A, m)
        P = H.P[k].toarray()
        coarse = (Ic - E_prev @ E_prev) @ np.linalg.solve(H.A[k - 1].toarray(), P.T @ A)
        E_prev = smooth @ (I - P @ coarse) @ smooth
    A = H.A[3].toarray()
    rng = np.random.default_rng(5)
    f, z = rng.standard_normal(len(A)), rng.standard_normal(len(A))
    ref = z + (np.eye(len(A)) - E_prev) @ np.linalg.solve(A, f - A @ z)
    out = mg.wcycle(H, f, z, 3, m, m)
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref)


def test_multigrid_converges_and_stops_at_tolerance():
    # the inner system of the d = 3 deflated CG, (dt/3) L, with the paper's
    # m = 10 on three levels: every cycle contracts, the iteration stops at
    # the first iterate under the tolerance
    n, dt = 8, 1e-3
    H = mg3.Hierarchy(dt / 3 * d3.sipg_laplacian(n), n)
    f = np.random.default_rng(6).standard_normal(8 * n ** 3)
    z, cycles = mg.multigrid(H, f, m1=10, m2=10, tol=1e-10)
    A = H.A[H.J]
    rel = np.linalg.norm(f - A @ z) / np.linalg.norm(f)
    assert rel <= 1e-10 and 10 <= cycles <= 60
    z1, c1 = mg.multigrid(H, f, m1=10, m2=10, tol=1e-10, n_max=cycles - 1)
    assert np.linalg.norm(f - A @ z1) / np.linalg.norm(f) > 1e-10
    z0, c0 = mg.multigrid(H, np.zeros_like(f))
    assert c0 == 0 and not z0.any()


def test_deflated_cg_with_the_multigrid_inner_solve():
    # Algorithm 2 on the d = 3 system with the W-cycle inner solve (m = 10):
    # the same solution as with the exact inner solve, within the tolerance,
    # and the outer count of the exact inner solve within a few iterations;
    # the adaptive rule of eq. (tol) spends fewer W-cycles (Table 5, right)
    n, dt, tol = 4, 1e-2, 1e-8
    As = d3.operator(n, dt, nu=0.5)
    V = d3.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = np.random.default_rng(8).standard_normal(As.shape[0])
    exact = krylov.dcg(As, V, f, krylov.exact_inner(E), tol=tol)
    H = mg3.Hierarchy(E, n)
    fixed = krylov.dcg(As, V, f, krylov.mg_inner(H, 10, 10), tol=tol, c_F=0.01)
    adaptive = krylov.dcg(As, V, f, krylov.mg_inner(H, 10, 10), tol=tol, c_A=0.02)
    for res in (fixed, adaptive):
        assert res.rel_res_true <= 2 * tol
        assert abs(res.iterations - exact.iterations) <= 3
        assert np.linalg.norm(res.x - exact.x) <= 1e-6 * np.linalg.norm(exact.x)
    assert adaptive.total_cycles < fixed.total_cycles
