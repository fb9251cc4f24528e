"""CG, deflated CG and flexible (deflated) CG (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``cg``   plain conjugate gradients on A* x = f with the stopping rule
           ||r_i|| <= tol ||f|| (Section 4.1).
* ``dcg``  Algorithm 2 (FDCG): deflated operator M_D(z) = A*(z - pi(A* z)),
           right-hand side f_D, an outer CG or FCG(m) iteration on the
           deflated system (eq. (defl_sys)) and the reconstruction
           x = (x_hat - pi(A* x_hat)) + pi(f) (eq. (x_defl)).
           pi(z) = V z_hat(V^T z), where z_hat approximates (V^T A* V)^{-1}
           by an exact factorisation or by the Multigrid iteration.

Readings:
* f_D: Algorithm 2 prints f_D = f - pi^T(f), which drops the A* of
  eq. (defl_sys); this oracle uses eq. (defl_sys): f_D = (I - pi_A)^T f =
  f - A* pi(f) (pi is symmetric).
* Outer variants: 'cg' is standard CG on the deflated system (the DCG of
  Tables 2-3, beta = rho_new / rho); 'fcg' is Algorithm 1 with the
  truncation m_i = max{1, mod(i, m_max + 1)}, m_0 = 0 (Remark 5), and
  m_max = None meaning FCG(inf), m_i = i; 'gmres' is unrestarted GMRES
  (Remark 6) with the same inner-tolerance rules, its stopping test on the
  minimal residual norm of the least-squares problem.
* Inner tolerance (a relative tolerance, as the inner stopping rule is
  written): fixed rule tau^c = c_F * tol (eq. (fixed_tol)); adaptive rule
  tau^c = c_A * tol * ||f|| / ||r_i|| (eq. (tol)), used inside the outer loop
  while the prologue and epilogue solves use c_A * tol.
* The outer stopping test is on the recurrence residual of the deflated
  system relative to ||f|| (Section 4.1); the true residual of the
  reconstructed x is reported, never substituted.
* Restarts (not in the paper; ``restarts`` > 0): when the reconstructed x
  misses tol on its true residual, Algorithm 2 is run again from x_0 = x,
  a bounded number of times (the recurrence residual of the inexact
  projections drifts from the true one over a long run).

Parity status: pinned.  CG against the iterates of a library CG; deflated CG
with an exact inner solve against a dense Cholesky solution; the Kahl
identity and the consistency of the deflated system; recurrence residual =
true residual with exact inner solves; FCG(inf) = DCG counts with exact inner
solves; the truncation window of Remark 5 with an inexact two-grid inner
solve (each direction minus r_i spans exactly the kept directions, is
conjugate to the oldest kept one and not to the one before the window, with
coefficients formed from r_i as printed; FCG(m_max) equals FCG(inf) up to
the first wrap); a warm restart closing the gap between the recurrence and
the true residual; the Delta-t trends of Tables 1-2; the adaptive rule of eq. (tol)
reaching the target and the sparse direct solution with FCG(inf), and costing
fewer cycles than the fixed rule (the cost comparison of Table 3) with late inner solves
cheaper than early ones; GMRES iterates equal the minimal-residual points of
the Krylov spaces (dense least squares), GMRES reaches the dense solution in
no more steps than CG, and converges with the adaptive inexact inner solves
at a lower cycle cost than with the fixed rule (tests/test_oracle_krylov.py).
"""
import numpy as np
import scipy.linalg as sla

from .multigrid import multigrid


def cg(A, f, tol=1e-8, max_iter=100000, x0=None):
    """Plain CG.  Returns (x, iterations, residual-norm history)."""
    x = np.zeros_like(f) if x0 is None else x0.copy()
    r = f - A @ x
    fnorm = np.linalg.norm(f)
    p = r.copy()
    rho = r @ r
    hist = [np.sqrt(rho)]
    it = 0
    while it < max_iter and np.sqrt(rho) > tol * fnorm:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        rho_new = r @ r
        p = r + (rho_new / rho) * p
        rho = rho_new
        it += 1
        hist.append(np.sqrt(rho))
    return x, it, hist


def exact_inner(E):
    """z_hat(v) = E^{-1} v by a dense Cholesky factorisation of E = V^T A* V."""
    fac = sla.cho_factor(E.toarray() if hasattr(E, 'toarray') else E, lower=True)

    def solve(v, tol_c):
        return sla.cho_solve(fac, v), 0
    return solve


def mg_inner(H, m1=2, m2=2, n_max=100):
    """z_hat(v) = Multigrid({Z_k}, v, 0, m1, m2, tol_c, n_max) (Algorithm 2)."""
    def solve(v, tol_c):
        return multigrid(H, v, None, m1, m2, tol_c, n_max)
    return solve


class DCGResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _gmres(M_D, r0, x0, eps, max_iter, tol_c):
    """Unrestarted GMRES on the deflated system (Remark 6): the Arnoldi
    process with modified Gram-Schmidt builds an orthonormal basis of the
    Krylov space of r0, Givens rotations keep the least-squares problem
    triangular, and the iteration stops when the minimal residual norm is at
    most eps.  Each product M_D v_j uses the inner tolerance of the current
    residual norm.  Returns (x, iterations, residual norm)."""
    beta = np.linalg.norm(r0)
    if beta <= eps or max_iter == 0:
        return x0, 0, beta
    Vb = [r0 / beta]
    H = []                                    # columns of the Hessenberg matrix
    cs, sn = [], []
    g = [beta]
    rnorm = beta
    j = 0
    while j < max_iter and rnorm > eps:
        w = M_D(Vb[j], tol_c(rnorm))
        h = np.zeros(j + 2)
        for i in range(j + 1):
            h[i] = w @ Vb[i]
            w = w - h[i] * Vb[i]
        hn = np.linalg.norm(w)
        h[j + 1] = hn
        for i in range(j):                    # earlier rotations
            a, b = h[i], h[i + 1]
            h[i], h[i + 1] = cs[i] * a + sn[i] * b, -sn[i] * a + cs[i] * b
        den = np.hypot(h[j], h[j + 1])
        cs.append(h[j] / den)
        sn.append(h[j + 1] / den)
        h[j], h[j + 1] = den, 0.0
        g.append(-sn[j] * g[j])
        g[j] = cs[j] * g[j]
        H.append(h)
        rnorm = abs(g[j + 1])
        Vb.append(w / hn if hn > 0 else w)   # hn = 0: invariant space, rnorm = 0
        j += 1
    R = np.zeros((j, j))
    for c in range(j):
        R[:c + 1, c] = H[c][:c + 1]
    y = sla.solve_triangular(R, np.asarray(g[:j]))
    x = x0 + sum(y[i] * Vb[i] for i in range(j))
    return x, j, rnorm


def dcg(Astar, V, f, inner, tol=1e-8, max_iter=100000, x0=None, outer='cg',
        m_max=None, c_F=0.01, c_A=None, restarts=0, trace=None, precond=None):
    """Deflated (flexible) CG, Algorithm 2.  Returns a DCGResult with x,
    outer iterations, total inner cycles (Tot), the per-solve inner cycle
    counts, and recurrence / true relative residuals.

    ``restarts``: when the reconstructed x misses the tolerance on its true
    residual ||f - A* x|| (the recurrence residual of an inexact inner solve
    drifts from it), Algorithm 2 is run again warm-started from that x, at
    most ``restarts`` times; pi(f) and f_D are those of the first pass (the
    same inner solve of the same vector).  Outer iterations and inner cycles
    are counted over all passes, and max_iter caps their total.

    ``precond``: with outer='fcg', a map B ~ (A*)^{-1} applied to each
    residual; the direction is built from z_i = B(r_i) in place of r_i
    (d_i = z_i - sum_k (z_i, q_k) / (d_k, q_k) d_k over the window, alpha_i =
    (d_i, r_i) / (d_i, q_i)), the flexible preconditioned form of Algorithm 1
    (oracle/precond.py).

    ``trace``: a list that receives, for every iteration i, with FCG the
    residual r_i the direction was built from, the direction d_i and
    q_i = M_D d_i; with CG the norms of r_i and of its component V^T r_i in
    the deflation space, relative to ||f|| (an exact inner solve keeps that
    component zero: V^T M_D = 0 and V^T f_D = 0)."""
    fnorm = np.linalg.norm(f)
    cycles = []
    outer_cycles = []

    def tol_c(rnorm=None):
        if c_A is None:
            return c_F * tol
        if rnorm is None:
            return c_A * tol
        return c_A * tol * fnorm / rnorm

    def pi(z, tc, inside=False):
        y, c = inner(V.T @ z, tc)
        cycles.append(c)
        if inside:
            outer_cycles.append(c)
        return V @ y

    def M_D(z, tc, inside=False):
        return Astar @ (z - pi(Astar @ z, tc, inside))

    def run_cg(x, r, it):
        p = r.copy()
        rho = r @ r
        while it < max_iter and np.sqrt(rho) > tol * fnorm:
            if trace is not None:
                trace.append(dict(rnorm=np.sqrt(rho) / fnorm,
                                  vtr=np.linalg.norm(V.T @ r) / fnorm))
            q = M_D(p, tol_c(np.sqrt(rho)), True)
            alpha = rho / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            rho_new = r @ r
            p = r + (rho_new / rho) * p
            rho = rho_new
            it += 1
        return x, r, it

    def run_fcg(x, r, it):
        # Algorithm 1; the window restarts with every pass of Algorithm 2
        ds, qs, dqs = [], [], []
        i = 0
        while it < max_iter and np.linalg.norm(r) > tol * fnorm:
            if m_max is None:
                m_i = i
            else:
                m_i = 0 if i == 0 else max(1, i % (m_max + 1))
            z = precond(r) if precond is not None else r
            d = z.copy()
            for k in range(i - m_i, i):
                d -= (z @ qs[k]) / dqs[k] * ds[k]
            q = M_D(d, tol_c(np.linalg.norm(r)), True)
            dq = d @ q
            alpha = (d @ r) / dq
            if trace is not None:
                trace.append(dict(r=r.copy(), d=d, q=q))
            x = x + alpha * d
            r = r - alpha * q
            ds.append(d)
            qs.append(q)
            dqs.append(dq)
            if m_max is not None and len(ds) > m_max + 1:
                ds[-m_max - 2] = qs[-m_max - 2] = None      # no longer referenced
            i += 1
            it += 1
        return x, r, it

    def run_gmres(x, r, it):
        x, k, rnorm = _gmres(lambda z, tc: M_D(z, tc, True), r, x, tol * fnorm,
                             max_iter - it, tol_c)
        return x, np.array([rnorm]), it + k     # only the residual norm is reported

    runs = dict(cg=run_cg, fcg=run_fcg, gmres=run_gmres)
    if outer not in runs:
        raise ValueError(outer)
    if precond is not None and outer != 'fcg':
        raise ValueError("a preconditioner needs the flexible outer iteration")
    pf = pi(f, tol_c())                       # pi(f), reused in the epilogue
    f_D = f - Astar @ pf
    x = np.zeros_like(f) if x0 is None else x0.copy()
    r = f_D.copy() if x0 is None else f_D - M_D(x, tol_c())
    it, passes = 0, 0
    while True:
        x, r, it = runs[outer](x, r, it)
        x_out = (x - pi(Astar @ x, tol_c())) + pf
        true = np.linalg.norm(f - Astar @ x_out) / fnorm
        if true <= tol or passes >= restarts or it >= max_iter:
            break
        passes += 1                           # Algorithm 2 again from x_0 = x
        x = x_out
        r = f_D - M_D(x, tol_c())
    rec = np.linalg.norm(r) / fnorm
    return DCGResult(x=x_out, x_hat=x, iterations=it, cycles=cycles,
                     total_cycles=int(sum(cycles)),
                     outer_cycles=outer_cycles, restarts=passes,
                     rel_res_recurrence=rec, rel_res_true=true)
