"""DG-Q1 discretisation of A* = M + alpha A in three dimensions (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is assembled, and where the paper defines it
-------------------------------------------------
* ``dev_mass``      M = mu^{-1} C_9 (x) M_1 with the 9 x 9 coefficient matrix
                    printed for d = 3 in Section 3.1 (read off the component
                    form of (dev sigma, dev tau), Section 2.3).
* ``scalar_forms``  the scalar SIPG forms a^h_ij, i, j in {1, 2, 3}
                    (Section 3.3.2), on a uniform hexahedral grid, with the
                    same component reading of jumps and averages as in 2D.
* ``divdiv``        A = blockdiag(C_3, C_3, C_3), C_3 = [B_ij] (Section 3.1).
* ``deflation_basis`` V = (v (x) I)/sqrt(3), v = 1 on sigma_11, sigma_22,
                    sigma_33 (eq. (Vmatrix), d = 3).
* ``sipg_laplacian`` an independently written scalar SIPG Laplacian in
                    normal-derivative form (Corollary 1 for d = 3:
                    V^T A* V = (alpha/3)(B_11 + B_22 + B_33) is this matrix
                    times alpha/3).

Readings (the paper's 3D runs use tetrahedral P1 elements in a finite-element
package; this module takes the hexahedral analogue of the 2D
discretisation):
  Omega = (0,1)^3, n^3 cubes of side h = 1/n, element e = (ez n + ey) n + ex;
  discontinuous Q1 per stress component with corner-nodal basis phi_j,
  j = ix + 2 iy + 4 iz; 2x2x2 Gauss in elements and 2x2 Gauss on faces
  (exact for every integrand here); penalty gamma = penalty / h, penalty
  alpha* = 40 by default (Section 4.2); the SIPG face terms sit on interior
  faces and on Gamma_out = {x = 1}, where Section 4.2 imposes sigma n = 0;
  the rest of the boundary carries the divergence data and no face term.

Parity status: pinned.  The printed 9 x 9 coefficient matrix, the closed-form
element mass, symmetry, M V = 0 with ker M of dimension N/9, consistency of
both SIPG forms on exactly representable fields (closed-form boundary
energies), and Corollary 1 (V^T A* V = (alpha/3) sipg_laplacian, with A V
assembled through the two independent forms) are checked in
tests/test_oracle_discretisation3d.py.
"""
import numpy as np
import scipy.sparse as sp

from .discretisation import GAUSS_POINTS, GAUSS_WEIGHTS, dev_coefficients, deflation_vector

D = 3
N_COMP = D * D
NB = 8                      # Q1 basis functions per hexahedron
DEFAULT_PENALTY = 40.0


# --------------------------------------------------------------------------
# reference Q1 basis on [0,1]^3, corner j = ix + 2 iy + 4 iz
# --------------------------------------------------------------------------
def _b(i, t):
    return t if i == 1 else 1.0 - t


def _db(i):
    return 1.0 if i == 1 else -1.0


def corner(j):
    return j % 2, (j // 2) % 2, j // 4


def q1_value(j, p):
    ix, iy, iz = corner(j)
    return _b(ix, p[0]) * _b(iy, p[1]) * _b(iz, p[2])


def q1_grad(j, p, h):
    """Physical gradient of phi_j at reference point p on a cube of side h."""
    ix, iy, iz = corner(j)
    return np.array([_db(ix) * _b(iy, p[1]) * _b(iz, p[2]),
                     _b(ix, p[0]) * _db(iy) * _b(iz, p[2]),
                     _b(ix, p[0]) * _b(iy, p[1]) * _db(iz)]) / h


def element_index(n, ex, ey, ez):
    return (ez * n + ey) * n + ex


def _volume_points():
    for gz, wz in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        for gy, wy in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            for gx, wx in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
                yield (gx, gy, gz), wx * wy * wz


# --------------------------------------------------------------------------
# element and face matrices by quadrature
# --------------------------------------------------------------------------
def element_mass(h):
    """int_K phi_b phi_a on one cube."""
    out = np.zeros((NB, NB))
    for p, w in _volume_points():
        v = np.array([q1_value(j, p) for j in range(NB)])
        out += w * h ** 3 * np.outer(v, v)
    return out


def element_grad_grad(h):
    """G[i][j][a, b] = int_K d_i phi_b d_j phi_a (volume part of a^h_ij)."""
    out = np.zeros((D, D, NB, NB))
    for p, w in _volume_points():
        g = np.array([q1_grad(j, p, h) for j in range(NB)])      # (8, 3)
        for i in range(D):
            for j in range(D):
                out[i, j] += w * h ** 3 * np.outer(g[:, j], g[:, i])
    return out


def _face_points(axis, side):
    """Reference points and weights of the 2x2 Gauss rule on the face
    {x_axis = side} of the reference cube."""
    others = [a for a in range(D) if a != axis]
    for g0, w0 in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        for g1, w1 in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
            p = [0.0, 0.0, 0.0]
            p[axis] = float(side)
            p[others[0]], p[others[1]] = g0, g1
            yield tuple(p), w0 * w1


def face_matrices(axis, interior, h, gamma):
    """Face contribution to every a^h_ij on one face normal to ``axis``.

    Interior face: sides (element below, at its x_axis = 1 face, normal +e_axis)
    and (element above, at its x_axis = 0 face, normal -e_axis).  Boundary face
    (the x = 1 side of Gamma_out): the single element below, normal +e_axis.
    Rows = test functions, columns = trial functions, each (8 s, 8 s).
      a_ij gets  - {d_i sigma} [[tau]]_j - {d_j tau} [[sigma]]_i
                 + gamma [[sigma]]_i [[tau]]_j
    with {.} the mean of the traces (the single trace on a boundary face) and
    [[v]] = sum_s v_s n_s."""
    sides = [(1, +1.0), (0, -1.0)] if interior else [(1, +1.0)]
    s = len(sides)
    avg = 0.5 if interior else 1.0
    out = np.zeros((D, D, NB * s, NB * s))
    pts = list(zip(_face_points(axis, 1), _face_points(axis, 0)))
    for (pa, wq), (pb, _) in pts:
        traces = []
        for (side, sign), p in zip(sides, (pa, pb)):
            nrm = np.zeros(D)
            nrm[axis] = sign
            traces.append((np.array([q1_value(j, p) for j in range(NB)]),
                           np.array([q1_grad(j, p, h) for j in range(NB)]), nrm))
        wf = wq * h * h
        for st in range(s):
            vt, gt, nt = traces[st]
            for ss in range(s):
                vs, gs, ns = traces[ss]
                for i in range(D):
                    for j in range(D):
                        blk = (-avg * np.outer(vt * nt[j], gs[:, i])
                               - avg * np.outer(gt[:, j], vs * ns[i])
                               + gamma * np.outer(vt * nt[j], vs * ns[i]))
                        out[i, j, NB * st:NB * st + NB, NB * ss:NB * ss + NB] += wf * blk
    return out


def face_list(n):
    """Faces with SIPG terms: (axis, (e_below, e_above)) for interior faces and
    (0, (e,)) for the faces of Gamma_out = {x = 1}."""
    faces = []
    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                e = element_index(n, ex, ey, ez)
                if ex + 1 < n:
                    faces.append((0, (e, element_index(n, ex + 1, ey, ez))))
                if ey + 1 < n:
                    faces.append((1, (e, element_index(n, ex, ey + 1, ez))))
                if ez + 1 < n:
                    faces.append((2, (e, element_index(n, ex, ey, ez + 1))))
                if ex == n - 1:
                    faces.append((0, (e,)))
    return faces


def _scatter(rows, cols, vals, size):
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(size, size))


def scalar_mass(n):
    """M_1: the scalar DG-Q1 mass matrix (block diagonal)."""
    me = element_mass(1.0 / n)
    m = NB * n ** 3
    rows, cols, vals = [], [], []
    for e in range(n ** 3):
        idx = NB * e + np.arange(NB)
        rows.append(np.repeat(idx, NB))
        cols.append(np.tile(idx, NB))
        vals.append(me.ravel())
    return _scatter(rows, cols, vals, m)


def scalar_forms(n, penalty=DEFAULT_PENALTY, gamma=None):
    """B[i][j]: matrix of a^h_ij(sigma, tau), rows = test, columns = trial."""
    h = 1.0 / n
    if gamma is None:
        gamma = penalty / h
    m = NB * n ** 3
    vol = element_grad_grad(h)
    parts = [[([], [], []) for _ in range(D)] for _ in range(D)]
    for e in range(n ** 3):
        idx = NB * e + np.arange(NB)
        for i in range(D):
            for j in range(D):
                r, c, v = parts[i][j]
                r.append(np.repeat(idx, NB))
                c.append(np.tile(idx, NB))
                v.append(vol[i, j].ravel())
    cache = {(axis, interior): face_matrices(axis, interior, h, gamma)
             for axis in range(D) for interior in (True, False)}
    for axis, elems in face_list(n):
        fm = cache[(axis, len(elems) == 2)]
        idx = np.concatenate([NB * e + np.arange(NB) for e in elems])
        k = len(idx)
        for i in range(D):
            for j in range(D):
                r, c, v = parts[i][j]
                r.append(np.repeat(idx, k))
                c.append(np.tile(idx, k))
                v.append(fm[i, j].ravel())
    return [[_scatter(*parts[i][j], m) for j in range(D)] for i in range(D)]


# --------------------------------------------------------------------------
# tensor operators, component-major: sigma_{k+1,i+1} at block 3 k + i
# --------------------------------------------------------------------------
def comp(k, i):
    return D * k + i


def dev_mass(n, nu=1.0):
    return (sp.kron(sp.csr_matrix(dev_coefficients(D)), scalar_mass(n)) / nu).tocsr()


def divdiv(n, penalty=DEFAULT_PENALTY, B=None):
    """A = blockdiag(C_3, C_3, C_3): row block (k, j), column block (k, i)
    holds B[i][j] (test component (k, j), trial component (k, i))."""
    if B is None:
        B = scalar_forms(n, penalty)
    size = B[0][0].shape[0]
    blocks = [[sp.csr_matrix((size, size)) for _ in range(N_COMP)] for _ in range(N_COMP)]
    for k in range(D):
        for i in range(D):
            for j in range(D):
                blocks[comp(k, j)][comp(k, i)] = B[i][j]
    return sp.bmat(blocks, format='csr')


def operator(n, alpha, nu=1.0, penalty=DEFAULT_PENALTY):
    """A* = M + alpha A (eq. (pb_study)); alpha = dt for implicit Euler."""
    return (dev_mass(n, nu) + alpha * divdiv(n, penalty)).tocsr()


def deflation_basis(n):
    """V = (v (x) I)/sqrt(3), v = 1 on the diagonal components (eq. (Vmatrix))."""
    m = NB * n ** 3
    return sp.kron(sp.csr_matrix(deflation_vector(D).reshape(-1, 1)), sp.identity(m)).tocsr()


def divdiv_on_identity(n, penalty=DEFAULT_PENALTY, B=None):
    """A(q I / sqrt(3), tau) assembled directly: row block (k, j) holds
    a_kj(q, tau_kj)/sqrt(3) (Corollary 1, proof)."""
    if B is None:
        B = scalar_forms(n, penalty)
    rows = [None] * N_COMP
    for k in range(D):
        for j in range(D):
            rows[comp(k, j)] = [B[k][j] / np.sqrt(D)]
    return sp.bmat(rows, format='csr')


# --------------------------------------------------------------------------
# independently written scalar SIPG Laplacian (normal-derivative form)
# --------------------------------------------------------------------------
def sipg_laplacian(n, penalty=DEFAULT_PENALTY, gamma=None):
    """L(q, r) = sum_K int grad q . grad r
               - sum_F int ( {dq/dnu} (r_a - r_b) + {dr/dnu} (q_a - q_b) )
               + gamma sum_F int (q_a - q_b)(r_a - r_b),
    nu the unit normal from element a to element b on interior faces; on
    Gamma_out faces r_b = q_b = 0, nu outward and the single trace."""
    h = 1.0 / n
    if gamma is None:
        gamma = penalty / h
    m = NB * n ** 3
    stiff = np.zeros((NB, NB))
    for p, w in _volume_points():
        g = np.array([q1_grad(j, p, h) for j in range(NB)])
        stiff += w * h ** 3 * (g @ g.T)

    def face_block(axis, interior):
        nu = np.zeros(D)
        nu[axis] = 1.0
        blocks = np.zeros((2, 2, NB, NB))
        for (pa, w), (pb, _) in zip(_face_points(axis, 1), _face_points(axis, 0)):
            sides = []
            for sign, p in ((1.0, pa), (-1.0, pb if interior else None)):
                if p is None:
                    sides.append((0.0, np.zeros(NB), np.zeros(NB)))
                    continue
                val = np.array([q1_value(j, p) for j in range(NB)])
                dn = np.array([q1_grad(j, p, h) @ nu for j in range(NB)])
                sides.append((sign, val, dn))
            mean = 0.5 if interior else 1.0
            for t in range(2):
                st, vt, dt_ = sides[t]
                for s in range(2):
                    ss, vs, ds = sides[s]
                    blocks[t, s] += w * h * h * (-mean * np.outer(st * vt, ds)
                                                 - mean * np.outer(dt_, ss * vs)
                                                 + gamma * np.outer(st * vt, ss * vs))
        return blocks

    inner = [face_block(a, True) for a in range(D)]
    outer = face_block(0, False)
    rows, cols, vals = [], [], []

    def put(ia, ib, blk):
        rows.append(np.repeat(ia, len(ib)))
        cols.append(np.tile(ib, len(ia)))
        vals.append(blk.ravel())

    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                ia = NB * element_index(n, ex, ey, ez) + np.arange(NB)
                put(ia, ia, stiff)
                nxt = [(ex + 1, ey, ez), (ex, ey + 1, ez), (ex, ey, ez + 1)]
                for axis, (x, y, z) in enumerate(nxt):
                    if max(x, y, z) >= n:
                        continue
                    ib = NB * element_index(n, x, y, z) + np.arange(NB)
                    for t, it in ((0, ia), (1, ib)):
                        for s, is_ in ((0, ia), (1, ib)):
                            put(it, is_, inner[axis][t, s])
                if ex == n - 1:
                    put(ia, ia, outer[0, 0])
    return _scatter(rows, cols, vals, m)


# --------------------------------------------------------------------------
# nodal interpolation (pins)
# --------------------------------------------------------------------------
def node_coordinates(n):
    h = 1.0 / n
    xyz = np.zeros((NB * n ** 3, D))
    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                e = element_index(n, ex, ey, ez)
                for j in range(NB):
                    ix, iy, iz = corner(j)
                    xyz[NB * e + j] = ((ex + ix) * h, (ey + iy) * h, (ez + iz) * h)
    return xyz


def interpolate(n, fun):
    """DG-Q1 nodal interpolant of fun(x, y, z) (exact for trilinear fun)."""
    return np.array([fun(*p) for p in node_coordinates(n)])
