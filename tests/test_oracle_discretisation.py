"""Pins of the oracle's discretisation against what the paper and the
mathematics fix (no GPU)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from conftest import GOLDEN, read_golden_matrix
from oracle import discretisation as d

GP = d.GAUSS_POINTS
GW = d.GAUSS_WEIGHTS


# ---------------------------------------------------------------- closed forms
def test_q1_element_mass_closed_form():
    # int_K phi_a phi_b for bilinear corner functions on a square of side h:
    # h^2/36 * [[4,2,2,1],[2,4,1,2],[2,1,4,2],[1,2,2,4]] (exact integration)
    h = 0.37
    ref = h * h / 36.0 * np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]])
    assert np.allclose(d.element_mass(h), ref, rtol=0, atol=1e-15)


def test_q1_element_stiffness_closed_form():
    # int_K grad phi_a . grad phi_b is independent of h in 2D:
    # 1/6 * [[4,-1,-1,-2],[-1,4,-2,-1],[-1,-2,4,-1],[-2,-1,-1,4]]
    G = d.element_grad_grad(0.25)
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(G[0, 0] + G[1, 1], ref, atol=1e-14)
    # the mixed blocks are transposes of each other (B_ij = B_ji^T, Section 3.1)
    assert np.allclose(G[0, 1], G[1, 0].T, atol=1e-15)


# ---------------------------------------------------------------- printed data
def test_dev_coefficients_match_printed_matrices():
    for dim, name in ((2, "dev_coefficients_2d.txt"), (3, "dev_coefficients_3d.txt")):
        assert np.allclose(d.dev_coefficients(dim), read_golden_matrix(name), atol=1e-15)


def test_deflation_vector_matches_printed_basis():
    with open(os.path.join(GOLDEN, "deflation_vectors.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for tag, *vals in rows:
        dim = int(tag[1:])
        v = np.array([float(x) for x in vals])
        assert np.allclose(d.deflation_vector(dim), v / np.sqrt(dim), atol=1e-15)


def test_dev_mass_is_kronecker_of_scalar_mass():
    n = 4
    M = d.dev_mass(n, nu=2.0).toarray()
    C = read_golden_matrix("dev_coefficients_2d.txt")
    assert np.allclose(M, np.kron(C, d.scalar_mass(n).toarray()) / 2.0, atol=1e-16)


# ---------------------------------------------------------------- kernel of M
def test_M_V_is_zero_and_kernel_dimension():
    n = 4
    M = d.dev_mass(n)
    V = d.deflation_basis(n)
    assert abs(M @ V).max() <= 1e-16 * abs(M).max()
    # dim ker M = number of scalar dofs exactly (the sigma = qI modes)
    rank = np.linalg.matrix_rank(M.toarray(), tol=1e-12 * abs(M).max())
    assert rank == 3 * 4 * n * n


def test_Astar_V_equals_alpha_divdiv_on_identity():
    n, dt = 6, 3e-3
    B = d.scalar_forms(n)
    As = d.dev_mass(n) + dt * d.divdiv(n, B=B)
    lhs = As @ d.deflation_basis(n)
    rhs = dt * d.divdiv_on_identity(n, B=B)
    assert abs(lhs - rhs).max() <= 1e-14 * abs(rhs).max()


def test_corollary1_reduced_matrix_is_scaled_sipg_laplacian():
    for n, dt in ((4, 1e-1), (8, 1e-5)):
        As = d.operator(n, dt)
        V = d.deflation_basis(n)
        E = (V.T @ As @ V).toarray()
        L = d.sipg_laplacian(n).toarray()
        assert np.abs(E - dt / 2.0 * L).max() <= 1e-13 * np.abs(dt / 2.0 * L).max()


# ------------------------------------------------- consistency of the SIPG forms
def _gamma_d_load_scalar(n, dudn_right, dudn_top):
    """F(v) = int_{x=1} dudn_right(y) v dy + int_{y=1} dudn_top(x) v dx."""
    h = 1.0 / n
    f = np.zeros(4 * n * n)
    for ey in range(n):          # right side x = 1: element (n-1, ey), xi = 1
        e = d.element_index(n, n - 1, ey)
        for g, w in zip(GP, GW):
            y = (ey + g) * h
            for j in range(4):
                f[4 * e + j] += w * h * dudn_right(y) * d.q1_value(j, 1.0, g)
    for ex in range(n):          # top side y = 1: element (ex, n-1), eta = 1
        e = d.element_index(n, ex, n - 1)
        for g, w in zip(GP, GW):
            x = (ex + g) * h
            for j in range(4):
                f[4 * e + j] += w * h * dudn_top(x) * d.q1_value(j, g, 1.0)
    return f


def test_sipg_laplacian_consistency_on_bilinear_field():
    # u = xy lies in DG-Q1, is continuous, vanishes on Gamma_N and is harmonic,
    # so integration by parts gives L u = int_{Gamma_D} du/dn v exactly.
    n = 5
    u = d.interpolate(n, lambda x, y: x * y)
    rhs = _gamma_d_load_scalar(n, lambda y: y, lambda x: x)
    L = d.sipg_laplacian(n)
    assert np.allclose(L @ u, rhs, atol=1e-13)
    # the component forms sum to the same Laplacian (Corollary 1)
    B = d.scalar_forms(n)
    assert np.allclose((B[0][0] + B[1][1]) @ u, rhs, atol=1e-13)


@pytest.mark.parametrize("cell,expected_faces", [((2, 2), 4), ((0, 0), 4), ((4, 4), 2), ((0, 4), 3)])
def test_sipg_laplacian_penalty_energy(cell, expected_faces):
    # For a piecewise constant q (indicator of one square) only the penalty
    # term survives: L(q, q) = gamma * sum_F |F| = (10/h) * h * #faces in F^I u F^N.
    n = 5
    q = np.zeros(4 * n * n)
    e = d.element_index(n, *cell)
    q[4 * e:4 * e + 4] = 1.0
    assert np.isclose(q @ (d.sipg_laplacian(n) @ q), 10.0 * expected_faces, rtol=1e-13)


def _divdiv_rhs(n, a, b):
    """A(sigma, tau) for sigma_k = (a_k xy, b_k xy): div sigma_k = a_k y + b_k x
    is smooth, sigma_k . n = 0 on Gamma_N and [[sigma_k]]_n = 0 inside, so
    A(sigma, tau) = sum_k [ -int grad(div sigma_k) . tau_k
                            + int_{Gamma_D} div sigma_k tau_k . n ]
    with grad(div sigma_k) = (b_k, a_k); component-major vector."""
    h = 1.0 / n
    m = 4 * n * n
    out = np.zeros(4 * m)
    cell_int = h * h / 4.0        # int_K phi_j
    for k in range(2):
        f1 = np.full(m, -b[k] * cell_int)        # tested against tau_k1
        f2 = np.full(m, -a[k] * cell_int)        # tested against tau_k2
        f1 += _gamma_d_load_scalar(n, lambda y: a[k] * y + b[k] * 1.0, lambda x: 0.0)
        f2 += _gamma_d_load_scalar(n, lambda y: 0.0, lambda x: a[k] * 1.0 + b[k] * x)
        out[d.comp(k, 0) * m:(d.comp(k, 0) + 1) * m] = f1
        out[d.comp(k, 1) * m:(d.comp(k, 1) + 1) * m] = f2
    return out


def test_divdiv_consistency_on_bilinear_fields():
    n = 4
    m = 4 * n * n
    a, b = (1.0, -2.0), (0.5, 3.0)
    xy = d.interpolate(n, lambda x, y: x * y)
    sigma = np.zeros(4 * m)
    for k in range(2):
        sigma[d.comp(k, 0) * m:(d.comp(k, 0) + 1) * m] = a[k] * xy
        sigma[d.comp(k, 1) * m:(d.comp(k, 1) + 1) * m] = b[k] * xy
    A = d.divdiv(n)
    assert np.allclose(A @ sigma, _divdiv_rhs(n, a, b), atol=1e-13)


def test_divdiv_penalty_energy():
    # sigma_11 = 1 on one interior square: div = 0 inside, the normal jump of
    # row 1 is +-1 on the two vertical faces and 0 on the horizontal ones, so
    # A(sigma, sigma) = gamma * 2h = 20; likewise sigma_12 on horizontal faces.
    n = 5
    m = 4 * n * n
    e = d.element_index(n, 2, 2)
    A = d.divdiv(n)
    s11 = np.zeros(4 * m)
    s11[d.comp(0, 0) * m + 4 * e:d.comp(0, 0) * m + 4 * e + 4] = 1.0
    s12 = np.zeros(4 * m)
    s12[d.comp(0, 1) * m + 4 * e:d.comp(0, 1) * m + 4 * e + 4] = 1.0
    s22 = np.zeros(4 * m)
    s22[d.comp(1, 1) * m + 4 * e:d.comp(1, 1) * m + 4 * e + 4] = 1.0
    assert np.isclose(s11 @ (A @ s11), 20.0, rtol=1e-13)
    assert np.isclose(s12 @ (A @ s12), 20.0, rtol=1e-13)
    assert np.isclose(s22 @ (A @ s22), 20.0, rtol=1e-13)
    assert abs(s11 @ (A @ s12)) < 1e-12       # n_x n_y = 0 on every face
    assert abs(s11 @ (A @ s22)) < 1e-12       # different rows never couple


# ---------------------------------------------------------------- SPD
def test_operator_symmetric_positive_definite():
    n = 8
    A = d.divdiv(n).toarray()
    M = d.dev_mass(n).toarray()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > -1e-12 * np.abs(A).max()    # A is PSD
    for dt in (1e-1, 1e-4, 1e-10):
        ev = np.linalg.eigvalsh(M + dt * A)
        assert ev.min() > 0.0


def test_cholesky_of_operator_succeeds_at_n16():
    n = 16
    M = d.dev_mass(n).toarray()
    A = d.divdiv(n).toarray()
    for dt in (1e-1, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        sla.cho_factor(M + dt * A, lower=True)     # raises if not SPD
