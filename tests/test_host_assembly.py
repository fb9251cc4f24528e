"""Host-side setup of the library (C++ assembly, Galerkin hierarchy, RAS
tile inverses, coarsest inverse) against the oracle.  CPU only: the
library's dcg_host_assemble runs the same host code dcg_setup uploads."""
import numpy as np
import pytest
import scipy.sparse as sp

from layout import block_ell_to_csr, tensor_perm
from oracle import discretisation as d
from oracle import multigrid as mg

lib = pytest.importorskip("paper_2606_13429_amd._binding")


def _mesh(n):
    m, _ = lib.dcg_defaults()
    m.n = n
    return m


def _rel(a, b):
    if sp.issparse(a) or sp.issparse(b):
        diff = sp.csr_matrix(a) - sp.csr_matrix(b)
        return abs(diff).max() / abs(sp.csr_matrix(b)).max()
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


@pytest.mark.parametrize("n", [16, 32])
def test_divdiv_blocks_match_oracle(n):
    vals, cols = lib.dcg_host_assemble(_mesh(n), 0)
    A_elem = block_ell_to_csr(vals, cols, n * n, 16, 16)
    perm = tensor_perm(n)
    A_lib = A_elem[perm][:, perm]
    assert _rel(A_lib, d.divdiv(n)) < 1e-13


def test_divdiv_on_identity_matches_oracle():
    n = 32
    vals, cols = lib.dcg_host_assemble(_mesh(n), 1)
    AZ = block_ell_to_csr(vals, cols, n * n, 16, 4)
    AZ_lib = AZ[tensor_perm(n)]
    assert _rel(AZ_lib, d.divdiv_on_identity(n)) < 1e-13


def test_element_mass_matches_oracle():
    n = 16
    vals, _ = lib.dcg_host_assemble(_mesh(n), 2)
    M1 = sp.block_diag([vals.reshape(n * n, 4, 4)[e] for e in range(n * n)])
    assert _rel(M1, d.scalar_mass(n)) < 1e-14


@pytest.mark.parametrize("n", [32, 64])
def test_galerkin_hierarchy_matches_oracle(n):
    # the library keeps L_k = (2/dt) Z_k; with dt = 2 the oracle's Z_J = V^T A* V is L_J
    As = d.operator(n, 2.0)
    V = d.deflation_basis(n)
    H = mg.Hierarchy((V.T @ As @ V).tocsr(), n)
    for k in range(1, H.J + 1):
        nk = H.n[k]
        vals, cols = lib.dcg_host_assemble(_mesh(n), 3, k)
        Lk = block_ell_to_csr(vals, cols, nk * nk, 4, 4)
        assert _rel(Lk, H.A[k]) < 1e-12, k


def test_ras_tile_inverses_match_oracle():
    n = 64
    As = d.operator(n, 2.0)
    V = d.deflation_basis(n)
    H = mg.Hierarchy((V.T @ As @ V).tocsr(), n)
    for k in range(2, H.J + 1):
        vals, squares = lib.dcg_host_assemble(_mesh(n), 4, k)
        T = vals.size // (128 * 128)
        F = vals.reshape(T, 128, 128)
        squares = squares.reshape(T, 32)
        blocks, weights = mg.ras_blocks(H.n[k])
        assert len(blocks) == T
        Ak = H.A[k].tocsr()
        for t in range(T):
            dofs = blocks[t]
            W = weights[t][:, None] * np.linalg.inv(Ak[dofs][:, dofs].toarray())   # D_i A_i^{-1}
            # library local order: 4 * slot + j over its 32 square slots
            pos = {dof: i for i, dof in enumerate(dofs)}
            lib_dofs = [4 * e + j for e in squares[t] if e >= 0 for j in range(4)]
            lib_idx = [4 * s + j for s, e in enumerate(squares[t]) if e >= 0 for j in range(4)]
            o_idx = [pos[x] for x in lib_dofs]
            Ft = F[t][np.ix_(lib_idx, lib_idx)]                 # F[j][i] = (D A^{-1})[i][j]
            ref = W[np.ix_(o_idx, o_idx)].T
            assert np.abs(Ft - ref).max() <= 1e-12 * np.abs(ref).max(), (k, t)
            # padded slots carry no weight
            pad = [4 * s + j for s, e in enumerate(squares[t]) if e < 0 for j in range(4)]
            if pad:
                assert not F[t][:, pad].any()


def test_coarsest_inverse_matches_oracle():
    n = 32
    vals, _ = lib.dcg_host_assemble(_mesh(n), 5)
    As = d.operator(n, 2.0)
    V = d.deflation_basis(n)
    H = mg.Hierarchy((V.T @ As @ V).tocsr(), n)
    ref = np.linalg.inv(H.A[1].toarray())
    assert _rel(vals.reshape(1024, 1024), ref) < 1e-10


def test_invalid_mesh_rejected():
    for bad in (0, 8, 48, 4096):
        with pytest.raises(lib.DCGError) as ei:
            lib.dcg_host_assemble(_mesh(bad), 0)
        assert ei.value.status == lib.DCG_EINVAL
    assert [lib.dcg_num_levels(n) for n in (16, 32, 512, 1024, 12)] == [1, 2, 6, 7, -1]


def test_divdiv_blocks_act_on_each_stress_row_alike():
    # the div-div form couples sigma_k1 with sigma_k2 of the same row k only,
    # with the same matrix for k = 1, 2 (Section 3.3.2): every 16 x 16 block is
    # diag(C, C); the device stores C alone and A_div Z follows from its
    # sigma_11 / sigma_22 columns
    lib = pytest.importorskip("paper_2606_13429_amd._binding")
    mesh, _ = lib.dcg_defaults()
    mesh.n = 16
    A, _ = lib.dcg_host_assemble(mesh, 0)
    A = A.reshape(-1, 5, 16, 16)
    assert not A[:, :, :8, 8:].any() and not A[:, :, 8:, :8].any()
    assert np.array_equal(A[:, :, :8, :8], A[:, :, 8:, 8:])
    AZ, _ = lib.dcg_host_assemble(mesh, 1)
    AZ = AZ.reshape(-1, 5, 16, 4)
    C = A[:, :, :8, :8]
    assert np.allclose(AZ[:, :, :8], C[..., :4] / np.sqrt(2), atol=1e-15, rtol=0)
    assert np.allclose(AZ[:, :, 8:], C[..., 4:] / np.sqrt(2), atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [16, 32])
def test_fast_diagonalisation_inverts_the_2d_laplacian(n):
    # the exact inner solve: with the host's 1D eigenvectors V and eigenvalues l
    # (K V = M V diag(l)), (V (x) V) diag(1 / (l_i + l_k)) (V (x) V)^T on the
    # tensor index (Iy, Ix) must invert the oracle's SIPG Laplacian, which also
    # checks the separable reading L = M (x) K + K (x) M
    N = 2 * n
    vals, _ = lib.dcg_host_assemble(_mesh(n), 6)
    V, lam = vals[:N * N].reshape(N, N), vals[N * N:]
    W = np.kron(V, V)
    Linv_t = W @ np.diag(1.0 / (lam[:, None] + lam[None, :]).reshape(-1)) @ W.T
    perm = np.zeros(4 * n * n, dtype=int)        # element-major 4 e + j -> (Iy, Ix)
    for e in range(n * n):
        ex, ey = e % n, e // n
        for j in range(4):
            perm[4 * e + j] = (2 * ey + (j >> 1)) * N + 2 * ex + (j & 1)
    Linv = Linv_t[np.ix_(perm, perm)]
    L = d.sipg_laplacian(n).toarray()
    assert np.abs(L @ Linv - np.eye(4 * n * n)).max() < 1e-9
    assert lam.min() > 0


@pytest.mark.parametrize("n,levels", [(64, 2), (64, 3), (32, 1)])
def test_coarse_level_fast_diagonalisation_inverts_galerkin_operator(n, levels):
    # the exact coarsest solve of a shortened hierarchy: the host's axis factors
    # of the coarsest level of ``levels`` levels must invert the oracle's own
    # Galerkin coarsest operator P^T ... L ... P (dense products of its sparse
    # hierarchy), which checks that the Galerkin product keeps the form
    # M_c (x) K_c + K_c (x) M_c with the one-dimensional injection
    nc = n >> (levels - 1)
    N = 2 * nc
    vals, _ = lib.dcg_host_assemble(_mesh(n), 7, levels)
    assert vals.size == N * N + N
    V, lam = vals[:N * N].reshape(N, N), vals[N * N:]
    W = np.kron(V, V)
    Linv_t = W @ np.diag(1.0 / (lam[:, None] + lam[None, :]).reshape(-1)) @ W.T
    perm = np.zeros(4 * nc * nc, dtype=int)
    for e in range(nc * nc):
        ex, ey = e % nc, e // nc
        for j in range(4):
            perm[4 * e + j] = (2 * ey + (j >> 1)) * N + 2 * ex + (j & 1)
    Linv = Linv_t[np.ix_(perm, perm)]
    As = d.operator(n, 2.0)                       # dt = 2: Z_J = V^T A* V = L_J
    Vd = d.deflation_basis(n)
    H = mg.Hierarchy((Vd.T @ As @ Vd).tocsr(), n, coarsest=nc)
    assert H.J == levels and H.n[1] == nc
    Lc = H.A[1].toarray()
    assert np.abs(Lc @ Linv - np.eye(4 * nc * nc)).max() < 1e-9
    assert lam.min() > 0


def test_coarse_level_factors_reject_bad_levels():
    with pytest.raises(lib.DCGError):
        lib.dcg_host_assemble(_mesh(64), 7, 0)
    with pytest.raises(lib.DCGError):
        lib.dcg_host_assemble(_mesh(64), 7, 4)       # J = 3 at n = 64
    with pytest.raises(lib.DCGError):
        lib.dcg_host_assemble(_mesh(1024), 7, 2)     # coarsest 512 > 256


def _square_class(ex, ey, n):
    cx = 0 if ex == 0 else (2 if ex == n - 1 else 1)
    cy = 0 if ey == 0 else (2 if ey == n - 1 else 1)
    return 3 * cy + cx


def test_level_operator_blocks_depend_only_on_the_square_class():
    # the device keeps one set of the five 4 x 4 blocks of L_k per class of
    # squares (left / interior / right times bottom / interior / top); the
    # library's host blocks must be bit-identical within a class (setup refuses
    # otherwise), and the oracle's own Galerkin hierarchy must show the same
    # structure (translation invariance of the uniform grid and of P^T L P)
    n = 64
    As = d.operator(n, 2.0)
    V = d.deflation_basis(n)
    H = mg.Hierarchy((V.T @ As @ V).tocsr(), n)
    steps = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    for k in range(1, H.J + 1):
        nk = H.n[k]
        vals, cols = lib.dcg_host_assemble(_mesh(n), 3, k)
        blocks = vals.reshape(nk * nk, 5, 4, 4)
        A = H.A[k].tocsr()
        rep_lib, rep_orc = {}, {}
        for e in range(nk * nk):
            ex, ey = e % nk, e // nk
            c = _square_class(ex, ey, nk)
            orc = np.zeros((5, 4, 4))
            for s, (dx, dy) in enumerate(steps):
                if 0 <= ex + dx < nk and 0 <= ey + dy < nk:
                    f = e + dx + dy * nk
                    orc[s] = A[4 * e:4 * e + 4, 4 * f:4 * f + 4].toarray()
            if c not in rep_lib:
                rep_lib[c], rep_orc[c] = blocks[e].copy(), orc
                continue
            assert np.array_equal(blocks[e], rep_lib[c]), (k, e)
            assert np.abs(orc - rep_orc[c]).max() <= 1e-12 * np.abs(rep_orc[c]).max(), (k, e)
        assert sorted(rep_lib) == list(range(9))
        for c in range(9):          # and the library's class blocks are the oracle's
            assert np.abs(rep_lib[c] - rep_orc[c]).max() <= 1e-12 * np.abs(rep_orc[c]).max()


def test_tile_inverses_fall_into_nine_position_classes():
    # the device stores one inverse per class of tiles; on the uniform grid the
    # local problem (L_k)_i and its weights D_i depend only on whether the tile
    # touches the left / right and bottom / top sides
    n = 64
    for k in (2, 3):
        vals, cols = lib.dcg_host_assemble(_mesh(n), 4, k)
        T = vals.size // (128 * 128)
        inv = vals.reshape(T, 128, 128)
        side = int(round(T ** 0.5))
        rep = {}
        for t in range(T):
            c = _square_class(t % side, t // side, side)
            if c in rep:
                assert np.array_equal(inv[t], inv[rep[c]]), (k, t)
            else:
                rep[c] = t
        assert len(rep) == 9
        distinct = {inv[t].tobytes() for t in rep.values()}
        assert len(distinct) == 9
