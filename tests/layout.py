"""Test-side conversions between the library's element-major layout and the
oracle's component-major layout, and block-ELL -> scipy.sparse."""
import numpy as np
import scipy.sparse as sp


def elem_to_comp(v, n):
    """[16 e + 4 c + j] -> [c * 4 n^2 + 4 e + j]."""
    return np.asarray(v).reshape(n * n, 4, 4).transpose(1, 0, 2).reshape(-1)


def comp_to_elem(v, n):
    """[c * 4 n^2 + 4 e + j] -> [16 e + 4 c + j]."""
    return np.asarray(v).reshape(4, n * n, 4).transpose(1, 0, 2).reshape(-1)


def tensor_perm(n):
    """perm such that x_comp = x_elem[perm]."""
    return elem_to_comp(np.arange(16 * n * n), n)


def block_ell_to_csr(vals, cols, ne, rows, ncols, ne_cols=None):
    """vals [ne][5][rows][ncols] with column squares cols [ne][5] (-1 = none)
    -> scipy CSR of shape (ne*rows, ne_cols*ncols) in the element-major order."""
    ne_cols = ne if ne_cols is None else ne_cols
    v = np.asarray(vals).reshape(ne, 5, rows, ncols)
    c = np.asarray(cols).reshape(ne, 5)
    R, C, V = [], [], []
    for s in range(5):
        ok = c[:, s] >= 0
        e = np.nonzero(ok)[0]
        col_e = c[ok, s]
        rr = (e[:, None, None] * rows + np.arange(rows)[None, :, None]) + 0 * np.arange(ncols)[None, None, :]
        cc = (col_e[:, None, None] * ncols + np.arange(ncols)[None, None, :]) + 0 * np.arange(rows)[None, :, None]
        R.append(rr.ravel())
        C.append(cc.ravel())
        V.append(v[ok, s].ravel())
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                         shape=(ne * rows, ne_cols * ncols))


def elem_to_comp3(v, n):
    """3D tensor vector [72 e + 8 c + a] -> [c * 8 n^3 + 8 e + a]."""
    return np.asarray(v).reshape(n ** 3, 9, 8).transpose(1, 0, 2).reshape(-1)


def comp_to_elem3(v, n):
    """[c * 8 n^3 + 8 e + a] -> [72 e + 8 c + a]."""
    return np.asarray(v).reshape(9, n ** 3, 8).transpose(1, 0, 2).reshape(-1)
