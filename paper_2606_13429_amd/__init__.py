"""MI355X deflated-CG solver for the implicit time step of the pseudo-stress
Stokes problem (A* = M + dt A, deflation onto ker M, W-cycle multigrid with
a Restricted Additive Schwarz smoother for the inner Laplace problem).

The compute path is libdcg.so (HIP kernels for gfx950 behind the C ABI of
include/dcg.h); this package only marshals arguments.  Importing it fails
if the library has not been built.
"""
from ._binding import *          # noqa: F401,F403  (the C entry points)
from ._binding import (DCGError, dcg_defaults, dcg_destroy, dcg_setup, dcg_solve,
                       DCG_FP64, DCG_MIXED, DCG_OUTER_CG, DCG_OUTER_FCG1, DCG_OUTER_FCG,
                       DCG_OUTER_GMRES, DCG_PENDING, LIB_PATH, DCG_INNER_MG, DCG_INNER_EXACT,
                       DCG_INNER_NONE)

_OUTER = {"cg": DCG_OUTER_CG, "fcg1": DCG_OUTER_FCG1, "fcg": DCG_OUTER_FCG, "gmres": DCG_OUTER_GMRES}

__all__ = ["Solver", "Solver3D", "Server", "DCGError", "LIB_PATH"]


class Solver3D:
    """The three-dimensional solver (dcg3d_setup / dcg3d_solve): deflated CG
    for the d = 3 block structure on n^3 cubes, FP64; the inner system solved
    exactly by fast diagonalisation (inner="exact"), by the Multigrid
    iteration of W-cycles with the RAS smoother (inner="mg", ``smooth`` pre-
    and post-smoothing steps, ``levels`` levels, 0 = all) or by block-Jacobi
    CG (inner="cg"), the iterative ones to c_F * tol, or with c_A > 0 to the
    adaptive tolerance of eq. (tol); inner="none" switches the deflation off
    (plain CG on A*).  restarts > 0 reruns Algorithm 2 from the returned x
    while its true residual misses tol (at most that many times).

    >>> s = Solver3D(n=16, dt=1e-3)
    >>> status, stats = s.solve(b, x, tol=1e-8)     # 72 n^3 cuda float64 tensors
    """

    def __init__(self, n, dt, nu=1.0, penalty=40.0, c_F=0.01, max_outer=50000,
                 max_inner=None, inner="exact", c_A=0.0, levels=0, smooth=10, use_graph=True,
                 restarts=0):
        _, opt = dcg_defaults()
        opt.prec, opt.outer, opt.c_A, opt.x0_given = DCG_FP64, DCG_OUTER_CG, c_A, 0
        opt.restarts = restarts
        if max_inner is None:
            max_inner = 100 if inner == "mg" else DCG3D_DEFAULT_MAX_INNER
        opt.c_F, opt.max_outer, opt.max_inner = c_F, max_outer, max_inner
        opt.levels, opt.smooth3d, opt.use_graph = levels, smooth, int(use_graph)
        self.n, self.dt, self.nu, self.penalty, self.opt = n, dt, nu, penalty, opt
        self.inner = inner
        self.handle = dcg3d_setup(n, penalty, dt, nu, opt,
                                  {"exact": DCG3D_INNER_FDM, "cg": DCG3D_INNER_PCG,
                                   "none": DCG3D_INNER_NONE, "mg": DCG3D_INNER_MG}[inner])

    def solve(self, b, x, tol=1e-8):
        return dcg3d_solve(self.handle, b, x, tol)

    def apply(self, op, inp, out, tol=0.0):
        return dcg3d_apply(self.handle, op, inp, out, tol)

    def mg_apply(self, op, level, inp, out, in2=None):
        from ._binding import dcg3d_mg_apply
        return dcg3d_mg_apply(self.handle, op, level, inp, in2, out)

    def mg_levels(self):
        from ._binding import dcg3d_mg_levels
        return dcg3d_mg_levels(self.handle)

    def close(self):
        if self.handle is not None:
            dcg3d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """A solver handle for one mesh, dt and nu (dcg_setup / dcg_solve).

    >>> s = Solver(n=128, dt=1e-4, prec="mixed")
    >>> status, stats = s.solve(b, x, tol=1e-8)     # b, x: cuda float64 tensors
    """

    def __init__(self, n, dt, nu=1.0, prec="mixed", outer="cg", penalty=10.0, pre=2, post=2,
                 c_F=0.01, max_outer=50000, max_inner=100, x0_given=False, use_graph=True,
                 c_A=0.0, m_max=8, inner="mg", levels=0, restarts=0, ras_group=0, outer_mg=0):
        """outer: "cg", "fcg1", "fcg" (truncated FCG with m_max, FCG(inf) for
        m_max = 0) or "gmres"; c_A > 0 selects the adaptive inner tolerance of
        eq. (tol); inner="exact" solves the inner system exactly by fast
        diagonalisation instead of the W-cycle multigrid (uniform grid);
        inner="none" switches the deflation off (plain CG on A*); levels > 0
        keeps the finest ``levels`` levels of the multigrid hierarchy and
        solves its coarsest level exactly by fast diagonalisation; restarts > 0
        reruns Algorithm 2 from the returned x while its true residual misses
        tol (at most that many times); ras_group selects the RAS step kernel
        (0 automatic, 1 / 2 / 4 grouped MFMA tiles, -1 one tile per wavefront
        group); outer_mg = m > 0 (with outer="fcg") preconditions the outer
        iteration with one W-cycle on A* with m smoothing steps."""
        mesh, opt = dcg_defaults()
        mesh.n, mesh.penalty, mesh.pre, mesh.post = n, penalty, pre, post
        opt.prec = {"mixed": DCG_MIXED, "fp64": DCG_FP64}[prec]
        opt.outer = _OUTER[outer]
        opt.c_F, opt.max_outer, opt.max_inner = c_F, max_outer, max_inner
        opt.c_A, opt.m_max = c_A, m_max
        opt.inner = {"mg": DCG_INNER_MG, "exact": DCG_INNER_EXACT, "none": DCG_INNER_NONE}[inner]
        opt.x0_given, opt.use_graph = int(x0_given), int(use_graph)
        opt.levels, opt.restarts, opt.ras_group = levels, restarts, ras_group
        opt.outer_mg = outer_mg
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


class Server:
    """Continuous-batching server (dcg_server_create / dcg_submit / dcg_poll).

    >>> srv = Server(prec="mixed")
    >>> t = srv.submit(n=64, dt=1e-3, b=b, x=x, tol=1e-8)   # returns at once
    >>> status, stats = srv.wait(t)
    """

    def __init__(self, prec="mixed", outer="cg", c_F=0.01, max_outer=50000, max_inner=100,
                 use_graph=True, hbm_budget_bytes=0, max_pending=4096, c_A=0.0):
        from ._binding import dcg_server_create
        _, opt = dcg_defaults()
        opt.prec = {"mixed": DCG_MIXED, "fp64": DCG_FP64}[prec]
        opt.outer = _OUTER[outer]
        opt.c_F, opt.max_outer, opt.max_inner, opt.c_A = c_F, max_outer, max_inner, c_A
        opt.use_graph, opt.hbm_budget_bytes, opt.max_pending = int(use_graph), hbm_budget_bytes, max_pending
        self.opt = opt
        self.handle = dcg_server_create(opt)

    @staticmethod
    def mesh(n, penalty=10.0, pre=2, post=2):
        m, _ = dcg_defaults()
        m.n, m.penalty, m.pre, m.post = n, penalty, pre, post
        return m

    def prepare(self, n, **mesh_kw):
        from ._binding import dcg_server_prepare
        dcg_server_prepare(self.handle, self.mesh(n, **mesh_kw))

    def submit(self, n, dt, b, x, tol=1e-8, nu=1.0, **mesh_kw):
        from ._binding import dcg_submit
        return dcg_submit(self.handle, self.mesh(n, **mesh_kw), dt, nu, b, x, tol)

    def poll(self, ticket):
        from ._binding import dcg_poll
        return dcg_poll(self.handle, ticket)

    def wait(self, ticket, timeout=None, interval=2e-4):
        import time
        t0 = time.perf_counter()
        while True:
            status, st = self.poll(ticket)
            if status != DCG_PENDING:
                return status, st
            if timeout is not None and time.perf_counter() - t0 > timeout:
                raise TimeoutError("request %d still pending" % ticket)
            time.sleep(interval)

    def counters(self):
        from ._binding import dcg_server_counters
        return dcg_server_counters(self.handle)

    def close(self):
        if self.handle is not None:
            from ._binding import dcg_server_destroy
            dcg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
