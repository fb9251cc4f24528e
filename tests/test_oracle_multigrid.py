"""Pins of the oracle's multigrid and RAS smoother (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import discretisation as d
from oracle import multigrid as mg


def test_num_levels():
    assert [mg.num_levels(n) for n in (16, 32, 128, 512, 1024)] == [1, 2, 4, 6, 7]
    # shortened hierarchies: the four levels of Section 5 at n = 512 stop at 64 x 64
    assert [mg.num_levels(n, c) for n, c in ((512, 64), (64, 32), (32, 32), (1024, 128))] == [4, 2, 1, 4]
    for bad in (8, 48, 100):
        with pytest.raises(ValueError):
            mg.num_levels(bad)


@pytest.mark.parametrize("fun", [lambda x, y: 1.0, lambda x, y: x, lambda x, y: y,
                                 lambda x, y: x * y, lambda x, y: 3 - 2 * x + 0.5 * y + 7 * x * y])
def test_prolongation_reproduces_bilinear_functions(fun):
    # nested Q1: a function bilinear on the whole domain is reproduced exactly
    nc = 4
    P = mg.prolongation(nc)
    assert np.allclose(P @ d.interpolate(nc, fun), d.interpolate(2 * nc, fun), atol=1e-14)


def test_prolongation_injects_discontinuous_coarse_functions():
    # a coarse function living on one coarse square only stays on its 4 children
    nc = 3
    P = mg.prolongation(nc).toarray()
    E = d.element_index(nc, 1, 2)
    col = P[:, 4 * E:4 * E + 4]
    children = [d.element_index(2 * nc, 2 + cx, 4 + cy) for cy in range(2) for cx in range(2)]
    rows = np.concatenate([4 * e + np.arange(4) for e in children])
    mask = np.ones(P.shape[0], bool)
    mask[rows] = False
    assert np.all(col[mask] == 0.0)
    assert np.allclose(col[rows].sum(axis=1), 1.0)       # partition of unity inside
    assert set(np.unique(P)) <= {0.0, 0.25, 0.5, 1.0}


def test_galerkin_product_equals_direct_coarse_assembly():
    # P^T L_h P is the SIPG Laplacian of the 2h grid with the fine penalty:
    # jumps of a coarse Q1 function vanish on fine faces inside a coarse
    # square, coarse faces are unions of fine faces, and consistency terms of
    # a coarse function are the same on either grid.
    nf = 16
    gamma_f = 10.0 * nf
    Lf = d.sipg_laplacian(nf)
    P = mg.prolongation(nf // 2)
    Lc = (P.T @ Lf @ P).toarray()
    direct = d.sipg_laplacian(nf // 2, gamma=gamma_f).toarray()
    assert np.abs(Lc - direct).max() <= 1e-12 * np.abs(direct).max()
    # two levels down
    P2 = mg.prolongation(nf // 4)
    Lcc = P2.T @ sp.csr_matrix(Lc) @ P2
    direct2 = d.sipg_laplacian(nf // 4, gamma=gamma_f).toarray()
    assert np.abs(Lcc.toarray() - direct2).max() <= 1e-12 * np.abs(direct2).max()


@pytest.mark.parametrize("n_k", [8, 16, 32])
def test_ras_partition_of_unity(n_k):
    blocks, weights = mg.ras_blocks(n_k)
    total = np.zeros(4 * n_k * n_k)
    for dofs, w in zip(blocks, weights):
        total[dofs] += w
    assert np.allclose(total, 1.0, atol=1e-15)
    # interior tiles hold 32 squares (128 dofs); multiplicities 1, 2, 3
    sizes = sorted({len(b) for b in blocks})
    assert sizes[-1] == (128 if n_k >= 12 else 96) and sizes[0] == 4 * 24
    assert set(np.round(1.0 / np.concatenate(weights)).astype(int)) <= {1, 2, 3}


def test_ras_single_block_is_exact_solve():
    n = 8
    L = d.sipg_laplacian(n)
    S = mg.RAS(L, *mg.ras_blocks(n, tile=n))
    r = np.random.default_rng(1).standard_normal(L.shape[0])
    assert np.allclose(S.apply(r), np.linalg.solve(L.toarray(), r), rtol=1e-12, atol=1e-12)


def test_ras_one_square_no_overlap_is_block_jacobi():
    n = 4
    L = d.sipg_laplacian(n).toarray()
    S = mg.RAS(sp.csr_matrix(L), *mg.ras_blocks(n, tile=1, layer=False))
    r = np.random.default_rng(2).standard_normal(L.shape[0])
    ref = np.concatenate([np.linalg.solve(L[4 * e:4 * e + 4, 4 * e:4 * e + 4], r[4 * e:4 * e + 4])
                          for e in range(n * n)])
    assert np.allclose(S.apply(r), ref, atol=1e-13)


def test_coarsest_cholesky_reconstructs_operator():
    n = 32
    L = d.sipg_laplacian(n)
    H = mg.Hierarchy(L, n)
    C = np.tril(H.chol[0])
    A1 = H.A[1].toarray()
    assert np.abs(C @ C.T - A1).max() <= 1e-13 * np.abs(A1).max()


def test_two_grid_wcycle_equals_error_propagation_matrix():
    # J = 2: one W-cycle maps z to z + (I - E_TG) A^{-1} (f - A z) with
    # E_TG = (I - S A)^m2 (I - P A_1^{-1} P^T A) (I - S A)^m1  (Algorithm 4).
    n = 32
    L = d.sipg_laplacian(n)
    H = mg.Hierarchy(L, n)
    A = H.A[2].toarray()
    N = A.shape[0]
    S = np.zeros((N, N))
    for idx, w, inv in H.S[2].groups:
        for dofs, wi, Ai in zip(idx, w, inv):
            S[np.ix_(dofs, dofs)] += wi[:, None] * Ai
    P = H.P[2].toarray()
    I = np.eye(N)
    smooth = I - S @ A
    cgc = I - P @ np.linalg.solve(H.A[1].toarray(), P.T @ A)
    E = smooth @ smooth @ cgc @ smooth @ smooth
    rng = np.random.default_rng(3)
    f = rng.standard_normal(N)
    z = rng.standard_normal(N)
    ref = z + (I - E) @ np.linalg.solve(A, f - A @ z)
    out = mg.wcycle(H, f, z, 2)
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref)
    v = rng.standard_normal(N)                     # spectral radius < 1
    for _ in range(30):
        v = E @ v
    assert np.linalg.norm(v) ** (1.0 / 30) < 0.5


def _dense_smoother(H, k):
    N = H.A[k].shape[0]
    S = np.zeros((N, N))
    for idx, w, inv in H.S[k].groups:
        for dofs, wi, Ai in zip(idx, w, inv):
            S[np.ix_(dofs, dofs)] += wi[:, None] * Ai
    return S


def test_three_level_wcycle_equals_recursive_error_propagation():
    # gamma = 2 cycle: the coarse problem is approximated by two coarse
    # W-cycles from zero, so E_k = (I - S_k A_k)^m2 (I - P_k (I - E_{k-1}^2)
    # A_{k-1}^{-1} P_k^T A_k) (I - S_k A_k)^m1 with E_1 = 0 (Algorithm 4).
    n = 16
    L = d.sipg_laplacian(n)
    H = mg.Hierarchy(L, n, coarsest=4)
    assert H.J == 3
    E_prev = np.zeros((H.A[1].shape[0],) * 2)
    for k in (2, 3):
        A = H.A[k].toarray()
        I = np.eye(A.shape[0])
        Ic = np.eye(H.A[k - 1].shape[0])
        smooth = I - _dense_smoother(H, k) @ A
        P = H.P[k].toarray()
        coarse = (Ic - E_prev @ E_prev) @ np.linalg.solve(H.A[k - 1].toarray(), P.T @ A)
        E_prev = smooth @ smooth @ (I - P @ coarse) @ smooth @ smooth
    A = H.A[3].toarray()
    rng = np.random.default_rng(6)
    f = rng.standard_normal(A.shape[0])
    z = rng.standard_normal(A.shape[0])
    ref = z + (np.eye(len(A)) - E_prev) @ np.linalg.solve(A, f - A @ z)
    out = mg.wcycle(H, f, z, 3)
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref)


def test_multigrid_converges_and_stops_at_tolerance():
    n = 64
    dt = 1e-3
    L = d.sipg_laplacian(n)
    H = mg.Hierarchy(dt / 2 * L, n)
    f = np.random.default_rng(4).standard_normal(L.shape[0])
    z, cycles = mg.multigrid(H, f, tol=1e-10)
    rel = np.linalg.norm(f - H.A[H.J] @ z) / np.linalg.norm(f)
    assert rel <= 1e-10 and 3 <= cycles <= 20
    z0, c0 = mg.multigrid(H, np.zeros_like(f))
    assert c0 == 0 and not z0.any()
