"""Host construction of the outer multigrid preconditioner's hierarchy of A*
(class tables of the level operators, Galerkin products, RAS update tables,
coarsest inverse) against the oracle's (oracle/precond.py).  CPU only:
dcg_host_outer_mg runs the same host code that dcg_setup uploads."""
import numpy as np
import pytest
import scipy.sparse as sp

from layout import tensor_perm
from oracle import discretisation as d
from oracle import precond as pc

lib = pytest.importorskip("paper_2606_13429_amd._binding")

SLOTS = ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))
DIAMOND = [(dx, dy) for dy in range(-2, 3) for dx in range(-2, 3) if abs(dx) + abs(dy) <= 2]


def _op_class(x, n):
    return np.where(x == 0, 0, np.where(x == n - 1, 2, 1))


def _ras_class(x, n):
    return np.where(x < 3, x, np.where(n - 1 - x < 3, 6 - (n - 1 - x), 3))


def _dense_from_op(n, op):
    """The element-major level operator from its class table (9, 5, 16, 16)."""
    e = np.arange(n * n)
    x, y = e % n, e // n
    cls = _op_class(x, n) + 3 * _op_class(y, n)
    R, C, V = [], [], []
    for s, (dx, dy) in enumerate(SLOTS):
        ok = (x + dx >= 0) & (x + dx < n) & (y + dy >= 0) & (y + dy < n)
        for c in e[ok]:
            f = c + dx + dy * n
            R.append(np.repeat(16 * c + np.arange(16), 16))
            C.append(np.tile(16 * f + np.arange(16), 16))
            V.append(op[cls[c], s].ravel())
    m = 16 * n * n
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(m, m))


def _ras_apply(n, ras, r):
    e = np.arange(n * n)
    x, y = e % n, e // n
    cls = e if n < 6 else _ras_class(x, n) + 7 * _ras_class(y, n)
    rv = r.reshape(-1, 16)
    out = np.zeros_like(rv)
    for dd, (dx, dy) in enumerate(DIAMOND):
        ok = (x + dx >= 0) & (x + dx < n) & (y + dy >= 0) & (y + dy < n)
        c = e[ok]
        f = c + dx + dy * n
        out[c] += np.einsum("cab,cb->ca", ras[cls[c]][:, :, 16 * dd:16 * dd + 16], rv[f])
    return out.ravel()


@pytest.mark.parametrize("n,dt,nu", [(16, 1e-2, 1.0), (32, 1e-4, 0.7), (64, 1e-3, 1.0)])
def test_tables_match_the_oracle_hierarchy(n, dt, nu):
    pen = 10.0
    As = d.operator(n, dt, nu=nu, penalty=pen)
    H = pc.Hierarchy(As, n)
    rng = np.random.default_rng(n)
    for k in range(1, H.J + 1):
        nk = H.n[k]
        perm = tensor_perm(nk)                      # x_comp = x_elem[perm]
        A_elem = H.A[k][np.argsort(perm)][:, np.argsort(perm)]
        op = lib.dcg_host_outer_mg(n, pen, dt, nu, k, 0)
        got = _dense_from_op(nk, op)
        assert abs(got - A_elem).max() <= 1e-12 * abs(A_elem).max(), k
        if k >= 2:
            ras = lib.dcg_host_outer_mg(n, pen, dt, nu, k, 1)
            r = rng.standard_normal(16 * nk * nk)
            ref = H.S[k].apply(r[perm])[np.argsort(perm)]
            assert np.linalg.norm(_ras_apply(nk, ras, r) - ref) <= 1e-12 * np.linalg.norm(ref), k
    inv = lib.dcg_host_outer_mg(n, pen, dt, nu, 1, 2)
    perm = tensor_perm(8)
    ref = np.linalg.inv(H.A[1].toarray())[np.argsort(perm)][:, np.argsort(perm)]
    assert abs(inv - ref).max() <= 1e-9 * abs(ref).max()


@pytest.mark.parametrize("n,level,which", [(24, 1, 0), (128, 1, 0), (16, 1, 1), (16, 2, 2), (16, 3, 0), (16, 1, 4)])
def test_bad_arguments_are_rejected(n, level, which):
    with pytest.raises(lib.DCGError):
        lib.dcg_host_outer_mg(n, 10.0, 1e-3, 1.0, level, which)


def _from_operand_order(tm):
    """The class matrices as the MFMA kernels read them: at step s lane l
    supplies row l % 16, column 4 s + l / 16."""
    ncls, steps, _ = tm.shape
    out = np.empty((ncls, 16, 4 * steps))
    for s in range(steps):
        for l in range(64):
            out[:, l % 16, 4 * s + l // 16] = tm[:, s, l]
    return out


@pytest.mark.parametrize("n,dt", [(16, 1e-2), (32, 1e-4)])
def test_operand_order_tables_hold_the_same_matrices(n, dt):
    pen, nu = 10.0, 1.0
    J = {16: 2, 32: 3}[n]
    rng = np.random.default_rng(n)
    for k in range(1, J + 1):
        nk = n >> (J - k)
        op = lib.dcg_host_outer_mg(n, pen, dt, nu, k, 0)
        opm = _from_operand_order(lib.dcg_host_outer_mg(n, pen, dt, nu, k, 3))
        assert np.array_equal(opm, op.transpose(0, 2, 1, 3).reshape(9, 16, 80))
        # the same level product through the reordered table
        op_back = opm.reshape(9, 16, 5, 16).transpose(0, 2, 1, 3)
        z = rng.standard_normal(16 * nk * nk)
        assert np.array_equal(_dense_from_op(nk, op_back) @ z, _dense_from_op(nk, op) @ z)
        if k >= 2:
            ras = lib.dcg_host_outer_mg(n, pen, dt, nu, k, 1)
            rasm = _from_operand_order(lib.dcg_host_outer_mg(n, pen, dt, nu, k, 4))
            assert np.array_equal(rasm, ras)
