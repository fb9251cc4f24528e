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
