"""Host-side assembly of the 3D path (C++ element and face blocks, the
block-Jacobi inverses) against the oracle.  CPU only: dcg3d_host_blocks runs
the same host code that dcg3d_setup uploads."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import discretisation3d as d3

lib = pytest.importorskip("paper_2606_13429_amd._binding")

PEN = 40.0


def _neighbours(n):
    """nb[e, s]: element in face slot s of e (0 itself, 1/2 -x/+x, 3/4 -y/+y,
    5/6 -z/+z), -1 outside the cube."""
    ne = n ** 3
    e = np.arange(ne)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    nb = np.full((ne, 7), -1)
    nb[:, 0] = e
    for s, (ax, step) in enumerate([(ex, -1), (ex, 1), (ey, -1), (ey, 1), (ez, -1), (ez, 1)], start=1):
        stride = [1, 1, n, n, n * n, n * n][s - 1]
        ok = (ax + step >= 0) & (ax + step < n)
        nb[ok, s] = e[ok] + step * stride
    return nb


def _divdiv_from_blocks(n, cd):
    """Component-major sparse A_div from the [7][ne][24][24] column-major blocks."""
    ne = n ** 3
    m = 8 * ne
    nb = _neighbours(n)
    blk = cd.reshape(7, ne, 24, 24)          # [slot][e][column][row]
    rows, cols, vals = [], [], []
    for s in range(7):
        for e in range(ne):
            f = nb[e, s]
            if f < 0:
                assert not blk[s, e].any()
                continue
            for k in range(3):
                for j in range(3):
                    for i in range(3):
                        sub = blk[s, e, 8 * i:8 * i + 8, 8 * j:8 * j + 8].T   # [a][b]
                        r = (3 * k + j) * m + 8 * e + np.arange(8)
                        c = (3 * k + i) * m + 8 * f + np.arange(8)
                        rows.append(np.repeat(r, 8))
                        cols.append(np.tile(c, 8))
                        vals.append(sub.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(9 * m, 9 * m))


def _scalar_from_blocks(n, ld):
    ne = n ** 3
    nb = _neighbours(n)
    blk = ld.reshape(7, ne, 8, 8)            # [slot][e][b][a]
    rows, cols, vals = [], [], []
    for s in range(7):
        for e in range(ne):
            f = nb[e, s]
            if f < 0:
                assert not blk[s, e].any()
                continue
            rows.append(np.repeat(8 * e + np.arange(8), 8))
            cols.append(np.tile(8 * f + np.arange(8), 8))
            vals.append(blk[s, e].T.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(8 * ne, 8 * ne))


def _rel(a, b):
    diff = sp.csr_matrix(a) - sp.csr_matrix(b)
    return abs(diff).max() / abs(sp.csr_matrix(b)).max()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_divdiv_blocks_match_oracle(n):
    cd = lib.dcg3d_host_blocks(n, PEN, 1e-3, 0)
    assert _rel(_divdiv_from_blocks(n, cd), d3.divdiv(n, PEN)) < 1e-13


@pytest.mark.parametrize("n", [2, 3])
def test_laplacian_blocks_match_oracle(n):
    ld = lib.dcg3d_host_blocks(n, PEN, 1e-3, 1)
    assert _rel(_scalar_from_blocks(n, ld), d3.sipg_laplacian(n, PEN)) < 1e-13


def test_block_jacobi_inverses_and_mass():
    n, dt = 3, 0.25
    dinv = lib.dcg3d_host_blocks(n, PEN, dt, 2).reshape(n ** 3, 8, 8)     # [e][b][a]
    L = d3.sipg_laplacian(n, PEN).toarray()
    for e in range(n ** 3):
        blk = dt / 3.0 * L[8 * e:8 * e + 8, 8 * e:8 * e + 8]
        assert np.abs(dinv[e].T @ blk - np.eye(8)).max() < 1e-12
    me = lib.dcg3d_host_blocks(n, PEN, dt, 3).reshape(8, 8)
    assert np.abs(me - d3.element_mass(1.0 / n)).max() < 1e-17


@pytest.mark.parametrize("n", [2, 3, 4])
def test_fast_diagonalisation_inverts_the_laplacian(n):
    # the exact inner solve: with the host's per-axis eigenvectors V_d and
    # eigenvalues l_d, V diag(1 / (lx + ly + lz)) V^T (V = V_z (x) V_y (x) V_x on
    # the tensor index (Iz, Iy, Ix), V_z = V_y) must be the inverse of the
    # oracle's 3D SIPG Laplacian, which checks the Kronecker-sum reading too
    N = 2 * n
    f = lib.dcg3d_host_blocks(n, PEN, 1e-3, 4)
    Vx, lx = f[:N * N].reshape(N, N), f[N * N:N * N + N]
    Vy, ly = f[N * N + N:2 * N * N + N].reshape(N, N), f[2 * N * N + N:]
    V = np.kron(np.kron(Vy, Vy), Vx)
    lam = (lx[None, None, :] + ly[None, :, None] + ly[:, None, None]).reshape(-1)
    Linv_t = V @ np.diag(1.0 / lam) @ V.T                 # tensor order
    perm = np.zeros(8 * n ** 3, dtype=int)                # element-major -> tensor
    for e in range(n ** 3):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        for a in range(8):
            perm[8 * e + a] = ((2 * ez + (a >> 2)) * N + 2 * ey + ((a >> 1) & 1)) * N + 2 * ex + (a & 1)
    Linv = Linv_t[np.ix_(perm, perm)]
    L = d3.sipg_laplacian(n, PEN).toarray()
    assert np.abs(L @ Linv - np.eye(8 * n ** 3)).max() < 1e-9
    assert lx.min() > 0 and ly.min() > -1e-9 * ly.max()   # x carries the outflow face, y and z are Neumann


def test_host_blocks_rejects_bad_arguments():
    with pytest.raises(lib.DCGError):
        lib.dcg3d_host_blocks(1, PEN, 1e-3, 0)
    with pytest.raises(lib.DCGError):
        lib.dcg3d_host_blocks(3, -1.0, 1e-3, 0)
    with pytest.raises(KeyError):
        lib.dcg3d_host_blocks(3, PEN, 1e-3, 7)
    out = np.empty(64)
    assert lib._lib.dcg3d_host_blocks(3, PEN, 1e-3, 5, out.ctypes.data_as(lib._P(lib.ctypes.c_double))) < 0
