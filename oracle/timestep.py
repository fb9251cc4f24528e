"""BDF2 time stepping of the semi-discrete problem (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.3 names BDF schemes and leaves alpha(dt) and the load functional to
the scheme.  For BDF2 applied to M d/dt sigma + A sigma = F:
  (3 s^n - 4 s^{n-1} + s^{n-2}) / (2 dt) M + A s^n = F
which, multiplied by 2 dt / 3, is eq. (weak_IE) with
  alpha = 2 dt / 3,   f*_n = M (4/3 s^{n-1} - 1/3 s^{n-2}) + (2 dt / 3) F.
Reading: s^0 = s^{-1} = 0, the forcing is time independent, and each solve
is warm-started from the extrapolation 2 s^{n-1} - s^{n-2}.

Parity status: pinned.  With a dense direct solve in place of the deflated CG
the recursion is checked against the closed-form solution of the scalar
two-term recurrence on an eigenvector (tests/test_oracle_timestep.py).
"""
import numpy as np


def bdf2_rhs(M, F, s1, s2, dt):
    """f*_n = M (4/3 s^{n-1} - 1/3 s^{n-2}) + (2 dt / 3) F."""
    return M @ (4.0 / 3.0 * s1 - 1.0 / 3.0 * s2) + (2.0 * dt / 3.0) * F


def bdf2_alpha(dt):
    return 2.0 * dt / 3.0


def bdf2(M, F, dt, steps, solve):
    """Runs ``steps`` BDF2 steps from zero history.  ``solve(f, x0)`` returns
    the solution of (M + alpha A) x = f (alpha = 2 dt / 3) and any per-step
    record.  Returns (final state, list of records)."""
    s1 = np.zeros_like(F)
    s2 = np.zeros_like(F)
    records = []
    for _ in range(steps):
        f = bdf2_rhs(M, F, s1, s2, dt)
        x, rec = solve(f, 2.0 * s1 - s2)
        records.append(rec)
        s2, s1 = s1, x
    return s1, records
