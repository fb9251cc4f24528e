"""MI355X deflated-CG solver for the implicit time step of the pseudo-stress
Stokes problem (A* = M + dt A, deflation onto ker M, W-cycle multigrid with
a Restricted Additive Schwarz smoother for the inner Laplace problem).

The compute path is libdcg.so (HIP kernels for gfx950 behind the C ABI of
include/dcg.h); this package only marshals arguments.  Importing it fails
if the library has not been built.
"""
from ._binding import *          # noqa: F401,F403  (the C entry points)
from ._binding import (DCGError, dcg_defaults, dcg_destroy, dcg_setup, dcg_solve,
                       DCG_FP64, DCG_MIXED, DCG_OUTER_CG, DCG_OUTER_FCG1, LIB_PATH)

__all__ = ["Solver", "DCGError", "LIB_PATH"]


class Solver:
    """A solver handle for one mesh, dt and nu (dcg_setup / dcg_solve).

    >>> s = Solver(n=128, dt=1e-4, prec="mixed")
    >>> status, stats = s.solve(b, x, tol=1e-8)     # b, x: cuda float64 tensors
    """

    def __init__(self, n, dt, nu=1.0, prec="mixed", outer="cg", penalty=10.0, pre=2, post=2,
                 c_F=0.01, max_outer=50000, max_inner=100, x0_given=False, use_graph=True):
        mesh, opt = dcg_defaults()
        mesh.n, mesh.penalty, mesh.pre, mesh.post = n, penalty, pre, post
        opt.prec = {"mixed": DCG_MIXED, "fp64": DCG_FP64}[prec]
        opt.outer = {"cg": DCG_OUTER_CG, "fcg1": DCG_OUTER_FCG1}[outer]
        opt.c_F, opt.max_outer, opt.max_inner = c_F, max_outer, max_inner
        opt.x0_given, opt.use_graph = int(x0_given), int(use_graph)
        self.n, self.dt, self.nu, self.mesh, self.opt = n, dt, nu, mesh, opt
        self.handle = dcg_setup(mesh, dt, nu, opt)

    def solve(self, b, x, tol=1e-8, stream=None):
        return dcg_solve(self.handle, b, x, tol, stream)

    def apply(self, op, inp, out, level=0, in2=None, stream=None):
        from ._binding import dcg_apply
        return dcg_apply(self.handle, op, level, inp, in2, out, stream)

    def close(self):
        if self.handle is not None:
            dcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
