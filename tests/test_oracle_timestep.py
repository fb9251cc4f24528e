"""Pin of the oracle's BDF2 right-hand side (no GPU)."""
import numpy as np

from oracle import timestep as ts


def test_bdf2_matches_scalar_difference_equation():
    # With diagonal M, A every component obeys the BDF2 difference equation
    #   m (3 c_n - 4 c_{n-1} + c_{n-2}) / (2 dt) + a c_n = F,
    # solved here directly for c_n; the oracle's rearranged form must agree.
    m = np.array([1.0, 0.5, 2.0])
    a = np.array([3.0, 10.0, 0.1])
    F = np.array([1.0, -2.0, 0.5])
    dt = 0.01
    alpha = ts.bdf2_alpha(dt)
    M = np.diag(m)
    A = np.diag(a)

    def solve(f, x0):
        return np.linalg.solve(M + alpha * A, f), None

    x, _ = ts.bdf2(M, F, dt, 7, solve)
    c1 = np.zeros(3)
    c2 = np.zeros(3)
    for _ in range(7):
        c = (F + m * (4 * c1 - c2) / (2 * dt)) / (3 * m / (2 * dt) + a)
        c2, c1 = c1, c
    assert np.allclose(x, c1, rtol=1e-13, atol=1e-15)
