"""Pins of the oracle's CG / deflated CG / FCG (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import discretisation as d
from oracle import krylov as kr
from oracle import multigrid as mg


def _problem(n, dt, seed=0):
    As = d.operator(n, dt)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = np.random.default_rng(seed).standard_normal(As.shape[0])
    return As, V, E, f


def test_cg_iterates_match_library_cg():
    n, dt = 6, 1e-3
    As, _, _, f = _problem(n, dt)
    its = []
    spla.cg(As, f, rtol=1e-30, atol=0.0, maxiter=25, callback=lambda xk: its.append(xk.copy()))
    for k in (1, 5, 15, 25):
        x, it, _ = kr.cg(As, f, tol=0.0, max_iter=k)
        assert it == k
        assert np.linalg.norm(x - its[k - 1]) <= 1e-10 * np.linalg.norm(its[k - 1])


def test_dcg_exact_inner_reaches_dense_solution():
    n, dt = 16, 1e-2
    As, V, E, f = _problem(n, dt)
    xs = np.linalg.solve(As.toarray(), f)
    r = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-12)
    assert np.linalg.norm(r.x - xs) <= 1e-8 * np.linalg.norm(xs)
    r8 = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8)
    assert r8.rel_res_true <= 1e-8


def test_recurrence_residual_equals_true_residual_with_exact_inner():
    n, dt = 16, 1e-4
    As, V, E, f = _problem(n, dt, seed=3)
    r = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8)
    assert abs(r.rel_res_recurrence - r.rel_res_true) <= 1e-12
    assert r.total_cycles == 0


def _dense_projector(As, V):
    A = As.toarray()
    Vd = V.toarray()
    return A, Vd, Vd @ np.linalg.solve(Vd.T @ A @ Vd, Vd.T @ A)


def test_deflated_matrix_kahl_identity_and_nullity():
    n, dt = 4, 1e-3
    As, V, _, _ = _problem(n, dt)
    A, Vd, pi_A = _dense_projector(As, V)
    I = np.eye(A.shape[0])
    AD = A @ (I - pi_A)
    assert np.abs(AD - (I - pi_A).T @ A @ (I - pi_A)).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(AD - AD.T).max() <= 1e-12 * np.abs(A).max()
    ev = np.linalg.eigvalsh((AD + AD.T) / 2)
    scale = ev.max()
    assert ev.min() > -1e-10 * scale
    assert np.sum(ev < 1e-10 * scale) == Vd.shape[1]        # nullity m = 4 N_e


def test_deflated_system_is_consistent():
    n, dt = 4, 1e-5
    As, V, _, f = _problem(n, dt, seed=7)
    A, Vd, pi_A = _dense_projector(As, V)
    I = np.eye(A.shape[0])
    AD = A @ (I - pi_A)
    fD = (I - pi_A).T @ f
    sol, *_ = np.linalg.lstsq(AD, fD, rcond=None)
    assert np.linalg.norm(AD @ sol - fD) <= 1e-9 * np.linalg.norm(fD)
    # and the decomposition x = (I - pi_A) x_hat + V E^{-1} V^T f solves A x = f
    x = (I - pi_A) @ sol + Vd @ np.linalg.solve(Vd.T @ A @ Vd, Vd.T @ f)
    assert np.linalg.norm(A @ x - f) <= 1e-8 * np.linalg.norm(f)


def test_condition_number_trends_of_table1():
    # kappa(A*) grows like 1/dt for small dt while kappa_eff stays bounded
    n = 8
    M = d.dev_mass(n).toarray()
    A = d.divdiv(n).toarray()
    Vd = d.deflation_basis(n).toarray()
    kap, keff = [], []
    for dt in (1e-6, 1e-7, 1e-8):
        As = M + dt * A
        ev = np.linalg.eigvalsh(As)
        kap.append(ev.max() / ev.min())
        pi_A = Vd @ np.linalg.solve(Vd.T @ As @ Vd, Vd.T @ As)
        AD = As @ (np.eye(len(As)) - pi_A)
        evd = np.linalg.eigvalsh((AD + AD.T) / 2)
        nz = evd[evd > 1e-9 * evd.max()]
        keff.append(nz.max() / nz.min())
    assert 8 < kap[1] / kap[0] < 12 and 8 < kap[2] / kap[1] < 12
    assert max(keff) / min(keff) < 1.5


def test_iteration_trends_of_table2():
    # CG needs more iterations as dt falls; deflated CG needs fewer and plateaus
    n = 16
    counts_cg, counts_dcg = [], []
    for dt in (1e-4, 1e-6, 1e-8):
        As, V, E, f = _problem(n, dt)
        counts_cg.append(kr.cg(As, f, tol=1e-8)[1])
        counts_dcg.append(kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8).iterations)
    assert counts_cg[0] < counts_cg[1] < counts_cg[2]
    assert counts_dcg[0] > counts_dcg[1] >= counts_dcg[2]
    assert counts_dcg[2] < counts_cg[2] / 20


def test_dcg_iterations_within_effective_condition_bound():
    n, dt = 8, 1e-4
    As, V, E, f = _problem(n, dt)
    A = As.toarray()
    Vd = V.toarray()
    pi_A = Vd @ np.linalg.solve(Vd.T @ A @ Vd, Vd.T @ A)
    AD = A @ (np.eye(len(A)) - pi_A)
    ev = np.linalg.eigvalsh((AD + AD.T) / 2)
    nz = ev[ev > 1e-9 * ev.max()]
    keff = nz.max() / nz.min()
    # A-norm bound 2((sqrt k - 1)/(sqrt k + 1))^i, converted to the residual
    # norm with a factor sqrt(kappa_eff)
    bound = int(np.ceil(0.5 * np.sqrt(keff) * np.log(2 * np.sqrt(keff) / 1e-8)))
    assert kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8).iterations <= bound


def test_fcg_matches_dcg_with_exact_inner_solves():
    # with a fixed (exact) inner operator FCG(inf), FCG(1) and CG coincide in
    # exact arithmetic (the c_F rows of Tables 3 and 4 are identical)
    n, dt = 16, 1e-3
    As, V, E, f = _problem(n, dt, seed=5)
    inner = kr.exact_inner(E)
    a = kr.dcg(As, V, f, inner, tol=1e-8)
    b = kr.dcg(As, V, f, inner, tol=1e-8, outer='fcg', m_max=None)
    c = kr.dcg(As, V, f, inner, tol=1e-8, outer='fcg', m_max=1)
    assert abs(a.iterations - b.iterations) <= 1 and abs(a.iterations - c.iterations) <= 2
    assert np.linalg.norm(a.x - b.x) <= 1e-7 * np.linalg.norm(a.x)


def test_dcg_with_multigrid_inner_matches_exact_inner():
    n, dt = 32, 1e-4
    As, V, E, f = _problem(n, dt, seed=1)
    exact = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-8)
    H = mg.Hierarchy(E, n)
    r = kr.dcg(As, V, f, kr.mg_inner(H), tol=1e-8)
    assert abs(r.iterations - exact.iterations) <= 2
    assert np.linalg.norm(r.x - exact.x) <= 1e-8 * np.linalg.norm(exact.x)
    inn = np.mean(r.outer_cycles)
    assert 3 <= inn <= 20 and r.total_cycles == sum(r.cycles)
    assert r.rel_res_true <= 1.1e-8


def test_warm_start_and_not_converged_paths():
    n, dt = 16, 1e-3
    As, V, E, f = _problem(n, dt, seed=2)
    inner = kr.exact_inner(E)
    full = kr.dcg(As, V, f, inner, tol=1e-10)
    warm = kr.dcg(As, V, f, inner, tol=1e-8, x0=full.x)
    assert warm.iterations <= 2
    capped = kr.dcg(As, V, f, inner, tol=1e-8, max_iter=3)
    assert capped.iterations == 3 and capped.rel_res_recurrence > 1e-8


def _spsolve(As, f):
    return spla.spsolve(As.tocsc(), f)


def test_adaptive_inner_tolerance_reaches_the_target_with_fcg():
    # eq. (tol): the inner accuracy is relaxed as the outer residual falls
    # "while still ensuring" the outer iteration reaches the target; with the
    # flexible outer iteration (Algorithm 1) the reconstructed x must reach
    # the tolerance and the sparse direct solution
    n, dt, tol = 32, 1e-3, 1e-8
    As, V, E, f = _problem(n, dt, seed=4)
    xs = _spsolve(As, f)
    H = mg.Hierarchy(E, n)
    r = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, outer='fcg', m_max=None, c_A=0.01,
               max_iter=1000)
    assert r.rel_res_recurrence <= tol
    assert r.rel_res_true <= 10 * tol
    assert np.linalg.norm(r.x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_adaptive_inner_tolerance_costs_fewer_wcycles_than_fixed():
    # Table 3: when both converge, the adaptive rule takes fewer multigrid
    # cycles in total (Tot) than the fixed rule with the same constant, and
    # the inner solves late in the iteration take fewer cycles than early ones
    n, dt, tol = 32, 1e-3, 1e-8
    As, V, E, f = _problem(n, dt, seed=5)
    H = mg.Hierarchy(E, n)
    fixed = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, outer='fcg', m_max=None, c_F=0.01,
                   max_iter=1000)
    adapt = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, outer='fcg', m_max=None, c_A=0.01,
                   max_iter=1000)
    assert fixed.rel_res_recurrence <= tol and adapt.rel_res_recurrence <= tol
    assert adapt.total_cycles < 0.8 * fixed.total_cycles, (adapt.total_cycles, fixed.total_cycles)
    oc = adapt.outer_cycles
    k = len(oc) // 4
    assert np.mean(oc[-k:]) < np.mean(oc[:k])
    assert len(set(fixed.outer_cycles)) <= 3      # the fixed rule: about constant


def test_gmres_iterates_are_the_minimal_residual_points():
    # GMRES's k-th iterate minimises ||f_D - M_D x|| over the k-th Krylov
    # space of f_D (x0 = 0): brute force with a dense least-squares problem
    n, dt = 4, 1e-2
    As, V, E, f = _problem(n, dt, seed=7)
    A, Vd, pi_A = _dense_projector(As, V)
    I = np.eye(A.shape[0])
    MD = A @ (I - pi_A)
    fD = (I - pi_A).T @ f
    for k in (1, 3, 6):
        r = kr.dcg(As, V, f, kr.exact_inner(E), tol=0.0, max_iter=k, outer='gmres')
        K = np.stack([np.linalg.matrix_power(MD, i) @ fD for i in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        c, *_ = np.linalg.lstsq(MD @ Q, fD, rcond=None)
        best = np.linalg.norm(fD - MD @ (Q @ c))
        assert r.iterations == k
        assert abs(r.rel_res_recurrence * np.linalg.norm(f) - best) <= 1e-9 * np.linalg.norm(f)
        assert np.linalg.norm(r.x_hat - Q @ c) <= 1e-8 * np.linalg.norm(Q @ c)


def test_gmres_reaches_the_dense_solution_in_no_more_steps_than_cg():
    # exact inner solves: the minimal-residual property makes GMRES need at
    # most as many steps as CG on the same Krylov spaces
    n, dt = 16, 1e-2
    As, V, E, f = _problem(n, dt, seed=8)
    xs = np.linalg.solve(As.toarray(), f)
    g = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-10, outer='gmres', max_iter=2000)
    c = kr.dcg(As, V, f, kr.exact_inner(E), tol=1e-10, max_iter=2000)
    assert np.linalg.norm(g.x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert g.rel_res_true <= 2e-10
    assert g.iterations <= c.iterations


def test_gmres_with_adaptive_inexact_inner_solves_converges():
    # Remark 6: GMRES with the adaptive inner tolerance converges robustly
    n, dt, tol = 32, 1e-3, 1e-8
    As, V, E, f = _problem(n, dt, seed=9)
    H = mg.Hierarchy(E, n)
    r = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, outer='gmres', c_A=0.01, max_iter=1000)
    assert r.rel_res_recurrence <= tol
    assert r.rel_res_true <= 20 * tol
    # and, as for the CG family (Table 3), the relaxed inner solves cost fewer cycles
    fixed = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, outer='gmres', c_F=0.01, max_iter=1000)
    assert r.total_cycles < 0.8 * fixed.total_cycles, (r.total_cycles, fixed.total_cycles)


# ---------------------------------------------------------------------------
# The truncation window of FCG(m_max) (Algorithm 1 with Remark 5's
# m_0 = 0, m_i = max{1, mod(i, m_max + 1)}), pinned with an inexact
# multigrid inner solve: with a varying (non-symmetric) effective operator
# the kept directions matter, which an exact inner solve (where every
# truncation reduces to CG) cannot show.
# ---------------------------------------------------------------------------
def _inexact_fcg_problem():
    # two-grid inner solve (16 x 16 -> 8 x 8) stopped at a relative residual
    # of 1e-2 (c_F tol = 1e6 * 1e-8): one or two W-cycles per inner solve
    n, dt = 16, 1e-2
    As, V, E, f = _problem(n, dt)
    H = mg.Hierarchy(E, n, coarsest=8)
    return As, V, f, kr.mg_inner(H)


# The windows {i - m_i, ..., i - 1} of Remark 5 for m_max = 3, written out by
# hand: m_i = 0, 1, 2, 3, 1, 1, 2, 3, 1, 1, 2, 3 for i = 0 .. 11.
_WINDOWS_M3 = [[], [0], [0, 1], [0, 1, 2], [3], [4], [4, 5], [4, 5, 6], [7], [8], [8, 9],
               [8, 9, 10]]


def _lstsq_residual(cols, g):
    D = np.stack(cols, axis=1)
    c, *_ = np.linalg.lstsq(D, g, rcond=None)
    return np.linalg.norm(g - D @ c) / np.linalg.norm(g)


def _cos(a, b):
    return abs(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))


def test_fcg_directions_use_exactly_the_kept_window():
    As, V, f, inner = _inexact_fcg_problem()
    tr = []
    kr.dcg(As, V, f, inner, tol=1e-8, max_iter=len(_WINDOWS_M3), outer='fcg', m_max=3,
           c_F=1e6, trace=tr)
    assert len(tr) == len(_WINDOWS_M3)
    for i, (t, w) in enumerate(zip(tr, _WINDOWS_M3)):
        g = t['d'] - t['r']
        if not w:                        # d_0 = r_0
            assert np.array_equal(t['d'], t['r'])
            continue
        # d_i - r_i lies in the span of the kept directions ...
        assert _lstsq_residual([tr[k]['d'] for k in w], g) <= 1e-12, i
        # ... and needs every one of them
        for k in w:
            rest = [tr[kk]['d'] for kk in w if kk != k]
            miss = 1.0 if not rest else _lstsq_residual(rest, g)
            assert miss >= 1e-7, (i, k, miss)


def test_fcg_direction_is_conjugate_to_the_oldest_kept_direction():
    # Within a window the later kept directions were themselves made
    # conjugate to the oldest one, so (d_i, q_s) = 0 for s = i - m_i holds
    # exactly, whatever the symmetry of the varying operator; the direction
    # just before the window is no longer orthogonalised against and keeps a
    # component of the operator's variation.
    As, V, f, inner = _inexact_fcg_problem()
    tr = []
    kr.dcg(As, V, f, inner, tol=1e-8, max_iter=len(_WINDOWS_M3), outer='fcg', m_max=3,
           c_F=1e6, trace=tr)
    for i, w in enumerate(_WINDOWS_M3):
        if not w:
            continue
        s = w[0]
        assert _cos(tr[i]['d'], tr[s]['q']) <= 1e-13, i
        if s > 0:
            assert _cos(tr[i]['d'], tr[s - 1]['q']) >= 1e-6, i
        if len(w) >= 2:
            # Algorithm 1 forms every coefficient from r_i (classical
            # Gram-Schmidt): against the newest kept direction the conjugacy
            # is only as good as the operator's variation allows (a modified
            # Gram-Schmidt loop would make it exact)
            assert _cos(tr[i]['d'], tr[i - 1]['q']) >= 1e-13, i


@pytest.mark.parametrize("m_max", [3, 6])
def test_fcg_truncated_equals_untruncated_until_the_first_wrap(m_max):
    # m_i = i for i <= m_max: FCG(m_max) and FCG(inf) agree iterate for
    # iterate over m_max + 1 iterations; iteration m_max + 1 keeps one
    # direction (m_i = 1) and the iterates part
    As, V, f, inner = _inexact_fcg_problem()
    K = m_max + 1
    a = kr.dcg(As, V, f, inner, tol=1e-8, max_iter=K, outer='fcg', m_max=None, c_F=1e6)
    b = kr.dcg(As, V, f, inner, tol=1e-8, max_iter=K, outer='fcg', m_max=m_max, c_F=1e6)
    assert a.iterations == b.iterations == K
    assert np.array_equal(a.x_hat, b.x_hat)
    a = kr.dcg(As, V, f, inner, tol=1e-8, max_iter=K + 1, outer='fcg', m_max=None, c_F=1e6)
    b = kr.dcg(As, V, f, inner, tol=1e-8, max_iter=K + 1, outer='fcg', m_max=m_max, c_F=1e6)
    assert np.linalg.norm(a.x_hat - b.x_hat) >= 1e-7 * np.linalg.norm(a.x_hat)


def test_restart_brings_the_true_residual_to_tol():
    # An inexact inner solve (two-grid, c_F tol = 1e-8) leaves the
    # reconstructed x of this solve with a true residual above tol although
    # the recurrence residual met it; one warm restart of Algorithm 2 from
    # that x closes the gap.  With exact inner solves the two residuals
    # coincide and no restart is taken.
    n, dt, tol = 16, 1e-3, 1e-8
    As, V, E, f = _problem(n, dt)
    inner = kr.mg_inner(mg.Hierarchy(E, n, coarsest=8))
    plain = kr.dcg(As, V, f, inner, tol=tol, c_F=1.0)
    assert plain.restarts == 0
    assert plain.rel_res_recurrence <= tol < plain.rel_res_true
    again = kr.dcg(As, V, f, inner, tol=tol, c_F=1.0, restarts=2)
    assert again.restarts >= 1 and again.rel_res_true <= tol
    assert again.iterations >= plain.iterations
    # the first pass is the plain solve; the restart starts from its x
    assert again.total_cycles > plain.total_cycles
    exact = kr.dcg(As, V, f, kr.exact_inner(E), tol=tol, restarts=2)
    assert exact.restarts == 0 and exact.rel_res_true <= tol


def test_inexact_projections_leave_a_deflation_space_residual_that_cg_cannot_remove():
    # With exact inner solves V^T M_D = 0 and V^T f_D = 0, so every CG
    # residual has no component in the deflation space.  Inexact inner
    # solves inject one; CG reduces the rest of the residual down to about
    # its size, then the recurrence residual climbs again by orders of
    # magnitude before it converges (the extra outer iterations of the fixed
    # inner tolerance on fine grids).  A tighter inner tolerance keeps that
    # component, and with it the detour, away.
    from dcg_workloads import rhs
    n, dt = 16, 1e-2
    As, V, E, _ = _problem(n, dt)
    f = rhs(n, 0).reshape(n * n, 4, 4).transpose(1, 0, 2).reshape(-1)
    inner = kr.mg_inner(mg.Hierarchy(E, n, coarsest=8))

    def history(c_F, inn=inner):
        tr = []
        r = kr.dcg(As, V, f, inn, tol=1e-8, c_F=c_F, max_iter=3000, trace=tr)
        return r, np.array([t["rnorm"] for t in tr]), np.array([t["vtr"] for t in tr])

    r, rn, vt = history(1.0)                   # inner tolerance 1e-8
    i = int(np.argmin(rn[:len(rn) // 2]))
    assert rn[i] <= 10 * vt[i] and vt[i] > 1e-8
    assert rn[i:].max() >= 100 * rn[i]
    assert r.rel_res_recurrence <= 1e-8
    r, rn, vt = history(0.01)                  # inner tolerance 1e-10
    i = int(np.argmin(rn[:len(rn) // 2]))
    assert rn[i:].max() <= 1.0001 * rn[i] and vt.max() < 1e-8
    _, rn, vt = history(0.01, kr.exact_inner(E))
    assert vt.max() <= 1e-13
