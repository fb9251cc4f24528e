"""BDF2 time stepping through the C ABI (Section 2.3; BDF2 reading: alpha =
2 dt / 3, f* = M(4/3 s^{n-1} - 1/3 s^{n-2}) + (2 dt / 3) F, zero history,
warm start 2 s^{n-1} - s^{n-2}).  The operators and the multigrid hierarchy
stay resident across steps; every step is dcg_bdf2_rhs + dcg_solve."""
from ._binding import DCG_OK, DCG_NOT_CONVERGED, DCGError, dcg_bdf2_rhs


class BDF2:
    """Time stepper for n x n squares with step dt and a fixed forcing F
    (device FP64 tensor vector)."""

    def __init__(self, n, dt, nu=1.0, prec="mixed", tol=1e-8, **opts):
        import torch
        from . import Solver
        self.n, self.dt, self.tol = n, dt, tol
        self.alpha = 2.0 * dt / 3.0
        self.solver = Solver(n, self.alpha, nu=nu, prec=prec, x0_given=True, **opts)
        N = 16 * n * n
        self.s1 = torch.zeros(N, dtype=torch.float64, device="cuda")
        self.s2 = torch.zeros_like(self.s1)
        self.f = torch.empty_like(self.s1)
        self.x = torch.empty_like(self.s1)
        self.steps = 0

    def step(self, F, stream=None):
        """Advances one step; returns the dcg_stats of its solve."""
        dcg_bdf2_rhs(self.solver.handle, self.s1, self.s2, F, self.alpha, self.f, self.x, stream)
        status, st = self.solver.solve(self.f, self.x, self.tol, stream)
        if status not in (DCG_OK, DCG_NOT_CONVERGED):
            raise DCGError(status, "BDF2 step %d" % self.steps)
        self.s2, self.s1, self.x = self.s1, self.x, self.s2     # rotate buffers
        self.steps += 1
        return st

    @property
    def state(self):
        return self.s1
