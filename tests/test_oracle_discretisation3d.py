"""Pins of the oracle's 3D discretisation against what the paper and the
mathematics fix (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from conftest import read_golden_matrix
from oracle import discretisation3d as d3
from oracle import krylov

PEN = d3.DEFAULT_PENALTY


# ---------------------------------------------------------------- closed forms
def _m1(h):
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


def _k1(h):
    return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h


def test_q1_hex_element_mass_is_tensor_product():
    # trilinear corner functions: the mass matrix is the Kronecker product of
    # three 1D P1 mass matrices h/6 [[2,1],[1,2]] (j = ix + 2 iy + 4 iz)
    h = 0.3
    ref = np.kron(np.kron(_m1(h), _m1(h)), _m1(h))
    assert np.allclose(d3.element_mass(h), ref, rtol=0, atol=1e-16)
    assert np.isclose(d3.element_mass(h).sum(), h ** 3)


def test_q1_hex_element_stiffness_is_sum_of_tensor_products():
    h = 0.2
    m, k = _m1(h), _k1(h)
    ref = np.kron(np.kron(m, m), k) + np.kron(np.kron(m, k), m) + np.kron(np.kron(k, m), m)
    G = d3.element_grad_grad(h)
    assert np.allclose(G[0, 0] + G[1, 1] + G[2, 2], ref, atol=1e-14)
    for i in range(3):
        for j in range(3):
            assert np.allclose(G[i, j], G[j, i].T, atol=1e-15)   # B_ij = B_ji^T


def test_dev_mass_is_kronecker_of_printed_coefficients():
    n = 2
    M = d3.dev_mass(n, nu=0.5).toarray()
    C = read_golden_matrix("dev_coefficients_3d.txt")
    assert np.allclose(M, np.kron(C, d3.scalar_mass(n).toarray()) / 0.5, atol=1e-16)


# ---------------------------------------------------------------- kernel of M
def test_M_V_is_zero_and_kernel_dimension():
    n = 2
    M = d3.dev_mass(n)
    V = d3.deflation_basis(n)
    assert abs(M @ V).max() < 1e-15
    # C has exactly one zero eigenvalue, so ker M = span(V) has dimension N/9
    ev = np.linalg.eigvalsh(read_golden_matrix("dev_coefficients_3d.txt"))
    assert np.sum(np.abs(ev) < 1e-12) == 1 and ev.min() > -1e-12
    assert V.shape == (9 * 8 * n ** 3, 8 * n ** 3)
    assert np.allclose((V.T @ V).toarray(), np.eye(8 * n ** 3))


def test_Astar_V_equals_alpha_divdiv_on_identity():
    n, alpha = 2, 0.37
    Astar = d3.operator(n, alpha)
    V = d3.deflation_basis(n)
    assert abs(Astar @ V - alpha * d3.divdiv_on_identity(n)).max() < 1e-11


def test_corollary1_reduced_matrix_is_scaled_sipg_laplacian():
    # V^T A* V = (alpha / 3)(B_11 + B_22 + B_33), and that sum is the SIPG
    # Laplacian written independently in normal-derivative form (Corollary 1, d = 3)
    n, alpha = 3, 0.05
    V = d3.deflation_basis(n)
    E = (V.T @ d3.operator(n, alpha) @ V).toarray()
    L = d3.sipg_laplacian(n).toarray()
    assert np.abs(E - alpha / 3.0 * L).max() < 1e-11 * np.abs(L).max()
    B = d3.scalar_forms(n)
    assert np.abs((B[0][0] + B[1][1] + B[2][2]).toarray() - L).max() < 1e-11 * np.abs(L).max()


# ---------------------------------------------------------------- consistency
def _poly_integrals(n_pts=3):
    g, w = np.polynomial.legendre.leggauss(n_pts)
    return (g + 1.0) / 2.0, w / 2.0


def _face_integral(fun, axis, side):
    """int over the face {x_axis = side} of the unit cube (3-point Gauss-Legendre
    per direction, exact for the polynomials used here)."""
    g, w = _poly_integrals()
    total = 0.0
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            p = [0.0, 0.0, 0.0]
            others = [k for k in range(3) if k != axis]
            p[axis], p[others[0]], p[others[1]] = side, a, b
            total += wa * wb * fun(*p)
    return total


def _volume_integral(fun):
    g, w = _poly_integrals()
    return sum(wa * wb * wc * fun(a, b, c) for a, wa in zip(g, w) for b, wb in zip(g, w)
               for c, wc in zip(g, w))


_TRILINEAR = {
    "1": (lambda x, y, z: 1.0, lambda x, y, z: (0.0, 0.0, 0.0)),
    "x": (lambda x, y, z: x, lambda x, y, z: (1.0, 0.0, 0.0)),
    "y": (lambda x, y, z: y, lambda x, y, z: (0.0, 1.0, 0.0)),
    "xz": (lambda x, y, z: x * z, lambda x, y, z: (z, 0.0, x)),
    "xyz": (lambda x, y, z: x * y * z, lambda x, y, z: (y * z, x * z, x * y)),
    "y+2z": (lambda x, y, z: y + 2 * z, lambda x, y, z: (0.0, 1.0, 2.0)),
}


def _a_ij_continuous(i, j, u, gu, v, gv, gamma):
    """a_ij(u, v) for continuous trilinear u, v, from the definition of the form
    (Section 3.3.2): jumps vanish on interior faces, so only the volume term and
    the Gamma_out = {x = 1} face (outward normal e_x, single traces) remain:
      int grad_i u grad_j v - [j = 0] int_F d_i u v - [i = 0] int_F d_j v u
      + gamma [i = 0][j = 0] int_F u v."""
    val = _volume_integral(lambda x, y, z: gu(x, y, z)[i] * gv(x, y, z)[j])
    if j == 0:
        val -= _face_integral(lambda x, y, z: gu(x, y, z)[i] * v(x, y, z), 0, 1.0)
    if i == 0:
        val -= _face_integral(lambda x, y, z: gv(x, y, z)[j] * u(x, y, z), 0, 1.0)
    if i == 0 and j == 0:
        val += gamma * _face_integral(lambda x, y, z: u(x, y, z) * v(x, y, z), 0, 1.0)
    return val


def test_component_forms_consistent_on_trilinear_fields():
    n = 3
    gamma = PEN * n
    B = d3.scalar_forms(n)
    names = list(_TRILINEAR)
    for un in names:
        u, gu = _TRILINEAR[un]
        uh = d3.interpolate(n, u)
        for vn in names:
            v, gv = _TRILINEAR[vn]
            vh = d3.interpolate(n, v)
            for i in range(3):
                for j in range(3):
                    got = vh @ (B[i][j] @ uh)
                    ref = _a_ij_continuous(i, j, u, gu, v, gv, gamma)
                    assert np.isclose(got, ref, rtol=1e-11, atol=1e-11), (un, vn, i, j, got, ref)


def test_sipg_laplacian_consistent_on_trilinear_fields():
    n = 3
    gamma = PEN * n
    L = d3.sipg_laplacian(n)
    for un, (u, gu) in _TRILINEAR.items():
        uh = d3.interpolate(n, u)
        for vn, (v, gv) in _TRILINEAR.items():
            vh = d3.interpolate(n, v)
            ref = sum(_a_ij_continuous(i, i, u, gu, v, gv, gamma) for i in range(3))
            assert np.isclose(vh @ (L @ uh), ref, rtol=1e-11, atol=1e-11), (un, vn)


@pytest.mark.parametrize("cell,faces", [((1, 1, 1), 6), ((0, 0, 0), 3), ((2, 0, 0), 4), ((2, 2, 2), 4),
                                        ((0, 1, 2), 4)])
def test_sipg_laplacian_penalty_energy(cell, faces):
    # q = indicator of one cube: only the penalty survives,
    # L(q, q) = gamma h^2 #(interior faces + Gamma_out faces of the cube)
    n = 3
    h = 1.0 / n
    q = np.zeros(8 * n ** 3)
    e = d3.element_index(n, *cell)
    q[8 * e:8 * e + 8] = 1.0
    assert np.isclose(q @ (d3.sipg_laplacian(n) @ q), PEN / h * h * h * faces, rtol=1e-13)


def test_divdiv_penalty_energy_selects_face_normals():
    # sigma_ki = indicator of an interior cube: div = 0 inside and the normal
    # jump of row k is nonzero only on the two faces normal to e_i, so
    # A(sigma, sigma) = gamma * 2 h^2; different rows never couple.
    n = 3
    h = 1.0 / n
    m = 8 * n ** 3
    e = d3.element_index(n, 1, 1, 1)
    A = d3.divdiv(n)
    vecs = {}
    for k in range(3):
        for i in range(3):
            s = np.zeros(9 * m)
            c = d3.comp(k, i)
            s[c * m + 8 * e:c * m + 8 * e + 8] = 1.0
            vecs[(k, i)] = s
            assert np.isclose(s @ (A @ s), 2.0 * PEN * h, rtol=1e-13)
    for (k1, i1), s1 in vecs.items():
        for (k2, i2), s2 in vecs.items():
            if (k1, i1) != (k2, i2):
                assert abs(s1 @ (A @ s2)) < 1e-12


def test_operator_symmetric_positive_definite():
    n = 2
    A = d3.divdiv(n).toarray()
    M = d3.dev_mass(n).toarray()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > -1e-12 * np.abs(A).max()
    for dt in (1.0, 1e-3, 1e-8):
        assert np.linalg.eigvalsh(M + dt * A).min() > 0.0


# ---------------------------------------------------------------- deflated CG in 3D
def test_dcg3d_with_exact_inner_solve_reaches_direct_solution():
    n, dt = 3, 1e-3
    Astar = d3.operator(n, dt)
    V = d3.deflation_basis(n)
    E = (V.T @ Astar @ V)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(Astar.shape[0])
    x_ref = spla.spsolve(Astar.tocsc(), f)
    res = krylov.dcg(Astar, V, f, krylov.exact_inner(E), tol=1e-10)
    assert np.linalg.norm(res.x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    # deflation removes the dt-dependence of the outer count (Table 5 trend):
    # plain CG needs several times more iterations at small dt
    _, it_cg, _ = krylov.cg(Astar, f, tol=1e-8)
    res8 = krylov.dcg(Astar, V, f, krylov.exact_inner(E), tol=1e-8)
    assert res8.iterations * 3 < it_cg
