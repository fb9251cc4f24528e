"""Rows of the outer multigrid's level operators on a large grid, evaluated
square by square on a small one (test-side, oracle only).

On the uniform grid the DG-Q1 forms scale exactly with the side h: the
element mass as h^2, the div-div SIPG form not at all (its volume term pairs
two gradients with the area; its face terms pair a gradient, or the penalty
gamma = penalty / h, with the face length).  So the rows of
A* = M + dt A of an n x n grid at a square equal the rows of an m x m grid's
operator with nu scaled by (n / m)^2 at the square that has the same
distances (capped at 3) from the four sides.  A level of the Galerkin
hierarchy of A* keeps the finest grid's penalty (P^T A P equals the direct
coarse assembly with the fine gamma), i.e. penalty n_J / n_k on its own grid.

Everything the RAS step computes at a square (Section 4.2: the blocks of the
square and of its edge neighbours, their local matrices and weights) lies
within distance 2 of it, and the residual it is applied to within distance
3; both windows map one to one into the m x m grid, so the oracle evaluates
the level operators of a 512 x 512 grid square by square on a 16 x 16 one.
tests/test_oracle_precond.py checks this against the oracle's own hierarchy.
"""
import numpy as np

from oracle import discretisation as d
from oracle import multigrid as mg
from oracle import precond as pc

RADIUS = 3


def axis_map(x, n, m):
    """Coordinate on the m-grid with the same (capped) distances to the sides."""
    if x < RADIUS:
        return x
    if n - 1 - x < RADIUS:
        return m - (n - x)
    return m // 2


class Window:
    """A*_k of an n_k x n_k level of the hierarchy whose finest grid has
    n_fine squares per side, and its RAS step, on an m x m grid."""

    def __init__(self, n_k, n_fine, dt, nu=1.0, penalty=10.0, m=16):
        assert m >= 2 * RADIUS + 3 and n_k >= m
        self.n, self.m = n_k, m
        self.A = d.operator(m, dt, nu=nu * (n_k / m) ** 2, penalty=penalty * n_fine / n_k)
        self.S = mg.RAS(self.A, *pc.ras_blocks(m))

    def _local(self, v, x, y):
        """v (element-major on the n-grid) copied to the m-grid around the
        image of square (x, y), component-major; zero elsewhere."""
        n, m = self.n, self.m
        xm, ym = axis_map(x, n, m), axis_map(y, n, m)
        out = np.zeros(16 * m * m)
        for dy in range(-RADIUS, RADIUS + 1):
            for dx in range(-RADIUS, RADIUS + 1):
                xs, ys = x + dx, y + dy
                if not (0 <= xs < n and 0 <= ys < n):
                    continue
                xt, yt = xm + dx, ym + dy
                assert 0 <= xt < m and 0 <= yt < m
                vals = np.asarray(v[16 * (ys * n + xs):16 * (ys * n + xs) + 16]).reshape(4, 4)
                e = d.element_index(m, xt, yt)
                for c in range(4):
                    out[c * 4 * m * m + 4 * e:c * 4 * m * m + 4 * e + 4] = vals[c]
        return out, d.element_index(m, xm, ym)

    def _at(self, w, e):
        """The 16 values of square e of a component-major m-grid vector, in
        the element-major order 4 c + j."""
        mm = 4 * self.m * self.m
        return np.concatenate([w[c * mm + 4 * e:c * mm + 4 * e + 4] for c in range(4)])

    def rows(self, z, x, y):
        """(A*_k z) on square (x, y)."""
        zl, e = self._local(z, x, y)
        return self._at(self.A @ zl, e)

    def ras(self, f, x, y, z=None):
        """(S_k f) on square (x, y), or (z + S_k (f - A*_k z)) with a start."""
        fl, e = self._local(f, x, y)
        if z is None:
            return self._at(self.S.apply(fl), e)
        zl, _ = self._local(z, x, y)
        return self._at(zl + self.S.apply(fl - self.A @ zl), e)


def sample_squares(n, count=48, seed=0):
    """Corners, every distance class near each side, and random interior squares."""
    edge = [0, 1, 2, 3, n - 4, n - 3, n - 2, n - 1]
    rng = np.random.default_rng(seed)
    sq = {(x, y) for x in (0, n - 1) for y in (0, n - 1)}
    for a in edge:
        sq.add((a, int(rng.integers(n))))
        sq.add((int(rng.integers(n)), a))
    while len(sq) < count:
        sq.add((int(rng.integers(n)), int(rng.integers(n))))
    return sorted(sq)
