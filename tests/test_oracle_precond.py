"""Pins of the oracle's multigrid preconditioner on A* for the outer
iteration (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import discretisation as d
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import precond as pc


def test_tensor_prolongation_is_the_scalar_one_per_component():
    nc = 4
    P, Ps = pc.prolongation(nc), mg.prolongation(nc)
    m, mf = 4 * nc * nc, 4 * (2 * nc) ** 2
    for c in range(4):
        for c2 in range(4):
            blk = P[c * mf:(c + 1) * mf, c2 * m:(c2 + 1) * m]
            assert abs(blk - (Ps if c == c2 else 0 * Ps)).max() == 0.0
    # a field bilinear on the whole domain in every component is reproduced
    funs = [lambda x, y: 1.0, lambda x, y: x, lambda x, y: x * y - 2 * y, lambda x, y: 3 + y]
    coarse = np.concatenate([d.interpolate(nc, f) for f in funs])
    fine = np.concatenate([d.interpolate(2 * nc, f) for f in funs])
    assert np.allclose(P @ coarse, fine, atol=1e-14)


def test_galerkin_products_equal_direct_coarse_assembly():
    # nested tensor spaces: P^T M_h P is the coarse mass matrix, P^T A_h P the
    # coarse div-div form with the fine penalty (coarse faces are unions of
    # fine faces, jumps of coarse fields vanish inside coarse squares)
    nf, pen = 8, 10.0
    P = pc.prolongation(nf // 2)
    Mc = (P.T @ d.dev_mass(nf, nu=0.7) @ P).toarray()
    assert np.abs(Mc - d.dev_mass(nf // 2, nu=0.7).toarray()).max() <= 1e-15
    Ac = (P.T @ d.divdiv(nf, pen) @ P).toarray()
    direct = d.divdiv(nf // 2, B=d.scalar_forms(nf // 2, gamma=pen * nf)).toarray()
    assert np.abs(Ac - direct).max() <= 1e-12 * np.abs(direct).max()


@pytest.mark.parametrize("n_k", [4, 8])
def test_ras_blocks_partition_of_unity_and_sizes(n_k):
    blocks, weights = pc.ras_blocks(n_k)
    assert len(blocks) == n_k * n_k
    total = np.zeros(16 * n_k * n_k)
    for dofs, w in zip(blocks, weights):
        total[dofs] += w
    assert np.allclose(total, 1.0, atol=1e-15)
    # a square and its edge neighbours: 5 inside, 3 at a corner, 16 dofs each
    assert sorted({len(b) // 16 for b in blocks}) == [3, 4, 5]
    assert set(np.round(1.0 / np.concatenate(weights)).astype(int)) == {3, 4, 5}


def test_two_grid_wcycle_equals_error_propagation_matrix():
    n, dt, m = 8, 1e-2, 2
    As = d.operator(n, dt)
    H = pc.Hierarchy(As, n, coarsest=4)
    assert H.J == 2
    A = H.A[2].toarray()
    N = len(A)
    S = np.zeros((N, N))
    for idx, w, inv in H.S[2].groups:
        for dofs, wi, Ai in zip(idx, w, inv):
            S[np.ix_(dofs, dofs)] += wi[:, None] * Ai
    I = np.eye(N)
    sm = np.linalg.matrix_power(I - S @ A, m)
    P = H.P[2].toarray()
    E = sm @ (I - P @ np.linalg.solve(H.A[1].toarray(), P.T @ A)) @ sm
    r = np.random.default_rng(3).standard_normal(N)
    ref = (I - E) @ np.linalg.solve(A, r)
    out = pc.preconditioner(H, m)(r)
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref)
    assert max(abs(np.linalg.eigvals(E))) < 1.0


def _system(n, dt):
    As = d.operator(n, dt)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = np.random.default_rng(5).standard_normal(As.shape[0])
    return As, V, E, f


def test_exact_inverse_as_preconditioner_converges_in_one_iteration():
    # V^T r_i = 0 for every deflated residual, so M_D (A*)^{-1} r_i = r_i and
    # the first step with z_0 = (A*)^{-1} r_0 lands on the solution
    n, dt = 8, 1e-2
    As, V, E, f = _system(n, dt)
    lu = spla.splu(As.tocsc())
    res = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-10, outer='fcg', m_max=None, precond=lu.solve)
    assert res.iterations == 1
    assert np.linalg.norm(res.x - lu.solve(f)) <= 1e-10 * np.linalg.norm(res.x)


def test_identity_preconditioner_gives_the_unpreconditioned_iterates():
    n, dt = 8, 1e-2
    As, V, E, f = _system(n, dt)
    a = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8, outer='fcg', m_max=8)
    b = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8, outer='fcg', m_max=8, precond=lambda r: r.copy())
    assert a.iterations == b.iterations and np.array_equal(a.x, b.x)
    with pytest.raises(ValueError):
        kr.dcg(As, V, f, kr.exact_inner(E), outer='cg', precond=lambda r: r)


def test_multigrid_preconditioned_solve():
    # the W-cycle on A* cuts the outer count of the deflated iteration several
    # times and reaches the direct solution; the count still grows with n on
    # this discretisation (23 -> 45 at dt = 1e-2, n = 16 -> 32)
    n, dt, tol = 16, 1e-2, 1e-8
    As, V, E, f = _system(n, dt)
    B = pc.preconditioner(pc.Hierarchy(As, n), m=2)
    res = kr.dcg(As, V, f, kr.exact_inner(E), tol=tol, outer='fcg', m_max=8, precond=B)
    plain = kr.dcg(As, V, f, kr.exact_inner(E), tol=tol, outer='fcg', m_max=8)
    x_direct = spla.spsolve(As.tocsc(), f)
    assert res.rel_res_true <= 2 * tol
    assert np.linalg.norm(res.x - x_direct) <= 1e-6 * np.linalg.norm(x_direct)
    assert 4 * res.iterations < plain.iterations


@pytest.mark.parametrize("dt", [1e-4, 1e-1])
def test_window_rows_reproduce_the_hierarchy_levels(dt):
    # the test-side window (tests/window2d.py) that evaluates the level
    # operators of large grids square by square rests on the exact h-scaling
    # of the forms and on the Galerkin levels keeping the fine penalty; both
    # are checked here against the oracle's own hierarchy at n = 32 (levels
    # 32 and 16, every distance class from the sides)
    from layout import comp_to_elem, tensor_perm
    from window2d import Window, sample_squares
    n = 32
    H = pc.Hierarchy(d.operator(n, dt), n)
    rng = np.random.default_rng(3)
    for k in (H.J, H.J - 1):
        nk = H.n[k]
        W = Window(nk, n, dt)
        pe = tensor_perm(nk)
        f, z = rng.standard_normal(16 * nk * nk), rng.standard_normal(16 * nk * nk)
        Az = comp_to_elem(H.A[k] @ z[pe], nk)
        Sf = comp_to_elem(H.S[k].apply(f[pe]), nk)
        Sz = comp_to_elem(z[pe] + H.S[k].apply(f[pe] - H.A[k] @ z[pe]), nk)
        for x, y in sample_squares(nk, count=30, seed=k):
            e = y * nk + x
            sl = slice(16 * e, 16 * e + 16)
            assert np.abs(W.rows(z, x, y) - Az[sl]).max() <= 1e-12 * np.abs(Az).max(), (k, x, y)
            assert np.abs(W.ras(f, x, y) - Sf[sl]).max() <= 1e-11 * np.abs(Sf).max(), (k, x, y)
            assert np.abs(W.ras(f, x, y, z) - Sz[sl]).max() <= 1e-11 * np.abs(Sz).max(), (k, x, y)
