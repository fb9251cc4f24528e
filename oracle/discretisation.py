"""DG-Q1 discretisation of the pseudo-stress operator A* = M + alpha A (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is assembled, and where the paper defines it
-------------------------------------------------
* ``dev_mass``      M, the dev-dev mass form written component-wise
                    (Section 2.3, eq. (component_form)); its d = 2 Kronecker
                    structure is printed in Section 3.1.
* ``scalar_forms``  the scalar SIPG forms a^h_ij of the PolyDG discretisation
                    (Section 3.3.2), specialised to DG-Q1 on a uniform square
                    grid, read component-wise: the flux term pairs the scalar
                    average {d_i sigma} with the j-th component of the vector
                    jump [[tau]] (the printed form pairs a scalar with a vector).
* ``divdiv``        A = sum_{k,i,j} a_ij(sigma_ki, tau_kj)
                    (eq. (component_form)), assembled as blockdiag(C_2, C_2)
                    (Section 3.1).
* ``deflation_basis`` V = (v (x) I)/sqrt(d), v = 1 on the diagonal components
                    (eq. (Vmatrix)).
* ``divdiv_on_identity`` the form A(q I / sqrt(2), tau) assembled directly,
                    i.e. A V without forming the product (Corollary 1, proof).
* ``sipg_laplacian`` an independently written scalar SIPG Laplacian in
                    normal-derivative form (Corollary 1: V^T A* V equals
                    (alpha/d) times the Laplacian stiffness matrix).

Discretisation choices the paper leaves open (each is a reading):
  Omega = (0,1)^2, n x n squares of side h = 1/n; discontinuous Q1 per stress
  component with corner-nodal basis phi_j, j = ix + 2 iy; 2x2 Gauss on
  elements and 2-point Gauss on faces (exact for every integrand here);
  penalty gamma = penalty / h with h the side length (p = 1); the traction
  (essential) boundary Gamma_N = {x = 0} u {y = 0} carries the SIPG face terms
  and the velocity boundary Gamma_D = {x = 1} u {y = 1} carries none
  (Section 5.1 places the velocity data on the top and right sides).

Parity status: pinned.  Closed-form element blocks, the printed dev-dev
coefficient matrix, consistency of both SIPG forms on exactly representable
fields (integration by parts), closed-form penalty energies, M V = 0,
A* V = alpha * divdiv_on_identity and V^T A* V = (alpha/2) sipg_laplacian are
checked in tests/test_oracle_discretisation.py.
"""
import numpy as np
import scipy.sparse as sp

_G = (1.0 - 1.0 / np.sqrt(3.0)) / 2.0
GAUSS_POINTS = (_G, 1.0 - _G)          # 2-point Gauss rule on [0, 1]
GAUSS_WEIGHTS = (0.5, 0.5)


# --------------------------------------------------------------------------
# reference Q1 basis on [0,1]^2, corner j = ix + 2 iy
# --------------------------------------------------------------------------
def _b(i, t):
    return t if i == 1 else 1.0 - t


def _db(i):
    return 1.0 if i == 1 else -1.0


def q1_value(j, xi, eta):
    """phi_j(xi, eta) on the reference square."""
    return _b(j % 2, xi) * _b(j // 2, eta)


def q1_grad(j, xi, eta, h):
    """Physical gradient (d/dx, d/dy) of phi_j on a square of side h."""
    ix, iy = j % 2, j // 2
    return np.array([_db(ix) * _b(iy, eta) / h, _b(ix, xi) * _db(iy) / h])


def element_index(n, ex, ey):
    return ey * n + ex


# --------------------------------------------------------------------------
# element and face matrices by quadrature
# --------------------------------------------------------------------------
def element_mass(h):
    """m(phi_b, phi_a) = int_K phi_b phi_a on one square (Section 2.3)."""
    out = np.zeros((4, 4))
    for gx, wx in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        for gy, wy in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            v = np.array([q1_value(j, gx, gy) for j in range(4)])
            out += wx * wy * h * h * np.outer(v, v)
    return out


def element_grad_grad(h):
    """G[i][j][a, b] = int_K d_i phi_b d_j phi_a (volume part of a^h_ij)."""
    out = np.zeros((2, 2, 4, 4))
    for gx, wx in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        for gy, wy in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            g = np.array([q1_grad(j, gx, gy, h) for j in range(4)])  # (4, 2)
            for i in range(2):
                for j in range(2):
                    out[i, j] += wx * wy * h * h * np.outer(g[:, j], g[:, i])
    return out


def _face_traces(side_coords, h):
    """Values and gradients of the 4 basis functions of one element at the two
    face quadrature points.  ``side_coords(g)`` maps the face parameter g in
    [0,1] to reference coordinates (xi, eta) of that element."""
    vals, grads = [], []
    for g in GAUSS_POINTS:
        xi, eta = side_coords(g)
        vals.append([q1_value(j, xi, eta) for j in range(4)])
        grads.append([q1_grad(j, xi, eta, h) for j in range(4)])
    return np.array(vals), np.array(grads)   # (2, 4), (2, 4, 2)


def face_matrices(sides, h, gamma):
    """Face contribution to every a^h_ij on one face (Section 3.3.2).

    ``sides`` lists (side_coords, outward_normal) for the one (boundary face)
    or two (interior face) elements sharing the face.  Returns F[i][j] of shape
    (4s, 4s), rows = test functions, columns = trial functions, s = #sides.

    With the component reading of the jump and average,
      a_ij gets  - {d_i sigma} [[tau]]_j - {d_j tau} [[sigma]]_i
                 + gamma [[sigma]]_i [[tau]]_j
    integrated over the face; {.} is the mean of the traces on an interior
    face and the single trace on a boundary face, [[v]] = sum_s v_s n_s.
    """
    s = len(sides)
    avg = 0.5 if s == 2 else 1.0
    traces = [_face_traces(c, h) for c, _ in sides]
    normals = [np.asarray(nrm, dtype=float) for _, nrm in sides]
    out = np.zeros((2, 2, 4 * s, 4 * s))
    for q, w in enumerate(GAUSS_WEIGHTS):
        wq = w * h
        for st in range(s):              # side of the test function
            vt, gt = traces[st][0][q], traces[st][1][q]
            nt = normals[st]
            for ss in range(s):          # side of the trial function
                vs, gs = traces[ss][0][q], traces[ss][1][q]
                ns = normals[ss]
                for i in range(2):
                    for j in range(2):
                        blk = (-avg * np.outer(vt * nt[j], gs[:, i])
                               - avg * np.outer(gt[:, j], vs * ns[i])
                               + gamma * np.outer(vt * nt[j], vs * ns[i]))
                        out[i, j, 4 * st:4 * st + 4, 4 * ss:4 * ss + 4] += wq * blk
    return out


# --------------------------------------------------------------------------
# face sets of the uniform grid
# --------------------------------------------------------------------------
def _vertical_pair():
    # left element (xi = 1 edge, normal +x), right element (xi = 0, normal -x)
    return [(lambda g: (1.0, g), (1.0, 0.0)), (lambda g: (0.0, g), (-1.0, 0.0))]


def _horizontal_pair():
    # lower element (eta = 1 edge, normal +y), upper element (eta = 0, normal -y)
    return [(lambda g: (g, 1.0), (0.0, 1.0)), (lambda g: (g, 0.0), (0.0, -1.0))]


def _left_boundary():
    return [(lambda g: (0.0, g), (-1.0, 0.0))]


def _bottom_boundary():
    return [(lambda g: (g, 0.0), (0.0, -1.0))]


def face_list(n):
    """All faces carrying SIPG terms: interior faces and Gamma_N faces.

    Returns a list of (kind, element tuple) with kind in
    {'v', 'h', 'left', 'bottom'}; Gamma_D faces (x = 1, y = 1) carry no term.
    """
    faces = []
    for ey in range(n):
        for ex in range(n - 1):
            faces.append(('v', (element_index(n, ex, ey), element_index(n, ex + 1, ey))))
    for ey in range(n - 1):
        for ex in range(n):
            faces.append(('h', (element_index(n, ex, ey), element_index(n, ex, ey + 1))))
    for ey in range(n):
        faces.append(('left', (element_index(n, 0, ey),)))
    for ex in range(n):
        faces.append(('bottom', (element_index(n, ex, 0),)))
    return faces


_FACE_GEOMETRY = {'v': _vertical_pair, 'h': _horizontal_pair,
                  'left': _left_boundary, 'bottom': _bottom_boundary}


def _scatter(rows, cols, vals, size):
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(size, size))


# --------------------------------------------------------------------------
# global scalar matrices
# --------------------------------------------------------------------------
def scalar_mass(n):
    """M_1: the scalar DG-Q1 mass matrix, block diagonal (Section 3.1)."""
    h = 1.0 / n
    me = element_mass(h)
    m = 4 * n * n
    rows, cols, vals = [], [], []
    for e in range(n * n):
        idx = 4 * e + np.arange(4)
        rows.append(np.repeat(idx, 4))
        cols.append(np.tile(idx, 4))
        vals.append(me.ravel())
    return _scatter(rows, cols, vals, m)


def scalar_forms(n, penalty=10.0, gamma=None):
    """B[i][j]: matrix of a^h_ij(sigma, tau) with rows indexed by the test
    function tau and columns by the trial function sigma (Section 3.3.2).

    gamma defaults to penalty / h (p = 1, h the side length)."""
    h = 1.0 / n
    if gamma is None:
        gamma = penalty / h
    m = 4 * n * n
    vol = element_grad_grad(h)
    parts = [[([], [], []) for _ in range(2)] for _ in range(2)]
    for e in range(n * n):
        idx = 4 * e + np.arange(4)
        for i in range(2):
            for j in range(2):
                r, c, v = parts[i][j]
                r.append(np.repeat(idx, 4))
                c.append(np.tile(idx, 4))
                v.append(vol[i, j].ravel())
    cache = {kind: face_matrices(geom(), h, gamma) for kind, geom in _FACE_GEOMETRY.items()}
    for kind, elems in face_list(n):
        fm = cache[kind]
        idx = np.concatenate([4 * e + np.arange(4) for e in elems])
        k = len(idx)
        for i in range(2):
            for j in range(2):
                r, c, v = parts[i][j]
                r.append(np.repeat(idx, k))
                c.append(np.tile(idx, k))
                v.append(fm[i, j].ravel())
    return [[_scatter(*parts[i][j], m) for j in range(2)] for i in range(2)]


# --------------------------------------------------------------------------
# tensor operators in the component-major layout
# --------------------------------------------------------------------------
D = 2
N_COMP = D * D


def comp(k, i):
    """Position of sigma_{k+1, i+1} in the unknown ordering
    [sigma_11, sigma_12, sigma_21, sigma_22] (Section 3.1)."""
    return D * k + i


def dev_coefficients(d):
    """The d^2 x d^2 matrix C with M = mu^{-1} C (x) M_1, read off the
    component form of (dev sigma, dev tau) (Section 2.3, eq. (component_form)):
      sum_k (1 - 1/d) m(s_kk, t_kk)
      + sum_{k != i} ( -1/d m(s_kk, t_ii) + m(s_ki, t_ki) ),
    unknowns ordered row by row, sigma_ki at position d k + i."""
    C = np.zeros((d * d, d * d))
    for k in range(d):
        C[d * k + k, d * k + k] += 1.0 - 1.0 / d
        for i in range(d):
            if i != k:
                C[d * i + i, d * k + k] += -1.0 / d      # test t_ii, trial s_kk
                C[d * k + i, d * k + i] += 1.0
    return C


def deflation_vector(d):
    """v / sqrt(d) with v_j = 1 for j in I_d = {(i-1) d + i} (eq. (Vmatrix))."""
    v = np.zeros(d * d)
    for i in range(d):
        v[d * i + i] = 1.0
    return v / np.sqrt(d)


def dev_mass(n, nu=1.0):
    """M = mu^{-1} C (x) M_1 with C from ``dev_coefficients`` (mu = nu)."""
    return (sp.kron(sp.csr_matrix(dev_coefficients(D)), scalar_mass(n)) / nu).tocsr()


def divdiv(n, penalty=10.0, B=None):
    """A = sum_{k,i,j} a_ij(sigma_ki, tau_kj) (eq. (component_form)).

    Row block = test component (k, j), column block = trial component (k, i),
    entry block B[i][j]; this is blockdiag(C_2, C_2) of Section 3.1."""
    if B is None:
        B = scalar_forms(n, penalty)
    size = B[0][0].shape[0]
    blocks = [[sp.csr_matrix((size, size)) for _ in range(N_COMP)] for _ in range(N_COMP)]
    for k in range(D):
        for i in range(D):
            for j in range(D):
                blocks[comp(k, j)][comp(k, i)] = B[i][j]
    return sp.bmat(blocks, format='csr')


def operator(n, alpha, nu=1.0, penalty=10.0):
    """A* = M + alpha A (eq. (pb_study)); alpha = dt for implicit Euler."""
    return (dev_mass(n, nu) + alpha * divdiv(n, penalty)).tocsr()


def deflation_basis(n):
    """V = (v (x) I)/sqrt(d), v_j = 1 for the diagonal components
    (eq. (Vmatrix)); columns span ker M."""
    m = 4 * n * n
    v = deflation_vector(D)
    return sp.kron(sp.csr_matrix(v.reshape(-1, 1)), sp.identity(m)).tocsr()


def divdiv_on_identity(n, penalty=10.0, B=None):
    """The form A(q I / sqrt(d), tau) assembled directly (no product with V):
    row block (k, j) holds a_kj(q, tau_kj)/sqrt(d), since only the diagonal
    entry sigma_kk = q/sqrt(d) of row k is nonzero (Corollary 1, proof)."""
    if B is None:
        B = scalar_forms(n, penalty)
    rows = [None] * N_COMP
    for k in range(D):
        for j in range(D):
            rows[comp(k, j)] = [B[k][j] / np.sqrt(D)]
    return sp.bmat(rows, format='csr')


# --------------------------------------------------------------------------
# independently written scalar SIPG Laplacian
# --------------------------------------------------------------------------
def sipg_laplacian(n, penalty=10.0, gamma=None):
    """Scalar SIPG Laplacian in normal-derivative form:
      L(q, r) = sum_K int grad q . grad r
              - sum_F int ( {dq/dnu} (r_a - r_b) + {dr/dnu} (q_a - q_b) )
              + gamma sum_F int (q_a - q_b)(r_a - r_b)
    over interior faces (unit normal nu from element a to element b) and
    Gamma_N faces (r_b = q_b = 0, nu outward, single trace).
    Written separately from ``scalar_forms`` so that Corollary 1 can be
    checked against it."""
    h = 1.0 / n
    if gamma is None:
        gamma = penalty / h
    m = 4 * n * n
    stiff = np.zeros((4, 4))
    for gx, wx in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        for gy, wy in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            g = np.array([q1_grad(j, gx, gy, h) for j in range(4)])
            stiff += wx * wy * h * h * (g @ g.T)
    rows, cols, vals = [], [], []

    def put(ia, ib, blk):
        rows.append(np.repeat(ia, len(ib)))
        cols.append(np.tile(ib, len(ia)))
        vals.append(blk.ravel())

    for e in range(n * n):
        idx = 4 * e + np.arange(4)
        put(idx, idx, stiff)

    def face_block(coords_a, coords_b, nu):
        # returns (2x2 grid of 4x4 blocks) [test side][trial side]
        nu = np.asarray(nu, dtype=float)
        blocks = np.zeros((2, 2, 4, 4))
        for g, w in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            sides = []
            for sign, c in ((1.0, coords_a), (-1.0, coords_b)):
                if c is None:
                    sides.append((0.0, np.zeros(4), np.zeros(4)))
                    continue
                xi, eta = c(g)
                val = np.array([q1_value(j, xi, eta) for j in range(4)])
                dn = np.array([q1_grad(j, xi, eta, h) @ nu for j in range(4)])
                sides.append((sign, val, dn))
            mean = 0.5 if coords_b is not None else 1.0
            for t in range(2):
                st, vt, dt_ = sides[t]
                for s in range(2):
                    ss, vs, ds = sides[s]
                    blocks[t, s] += w * h * (-mean * np.outer(st * vt, ds)
                                             - mean * np.outer(dt_, ss * vs)
                                             + gamma * np.outer(st * vt, ss * vs))
        return blocks

    vert = face_block(lambda g: (1.0, g), lambda g: (0.0, g), (1.0, 0.0))
    horz = face_block(lambda g: (g, 1.0), lambda g: (g, 0.0), (0.0, 1.0))
    left = face_block(lambda g: (0.0, g), None, (-1.0, 0.0))
    bottom = face_block(lambda g: (g, 0.0), None, (0.0, -1.0))
    for ey in range(n):
        for ex in range(n):
            e = element_index(n, ex, ey)
            ia = 4 * e + np.arange(4)
            if ex + 1 < n:
                ib = 4 * element_index(n, ex + 1, ey) + np.arange(4)
                for t, it in ((0, ia), (1, ib)):
                    for s, is_ in ((0, ia), (1, ib)):
                        put(it, is_, vert[t, s])
            if ey + 1 < n:
                ib = 4 * element_index(n, ex, ey + 1) + np.arange(4)
                for t, it in ((0, ia), (1, ib)):
                    for s, is_ in ((0, ia), (1, ib)):
                        put(it, is_, horz[t, s])
            if ex == 0:
                put(ia, ia, left[0, 0])
            if ey == 0:
                put(ia, ia, bottom[0, 0])
    return _scatter(rows, cols, vals, m)


# --------------------------------------------------------------------------
# nodal interpolation and load vectors used by pins and time stepping
# --------------------------------------------------------------------------
def node_coordinates(n):
    """(x, y) of every scalar dof 4 e + j (corner j of element e)."""
    h = 1.0 / n
    xy = np.zeros((4 * n * n, 2))
    for ey in range(n):
        for ex in range(n):
            e = element_index(n, ex, ey)
            for j in range(4):
                xy[4 * e + j] = ((ex + j % 2) * h, (ey + j // 2) * h)
    return xy


def interpolate(n, fun):
    """DG-Q1 nodal interpolant of fun(x, y) (exact for bilinear fun)."""
    xy = node_coordinates(n)
    return np.array([fun(x, y) for x, y in xy])
