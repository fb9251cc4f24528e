"""The shortened multigrid hierarchy (dcg_options.levels): the finest
``levels`` levels of the Galerkin hierarchy, with the coarsest of them solved
exactly by fast diagonalisation, against the oracle's Algorithms 3 and 4 on a
hierarchy with the same coarsest level (solved there by dense Cholesky).

Bars: the FP64 coarsest solve carries the rounding of four dense products
(relative error ~ eps * kappa(L_1), kappa ~ 1e4 at 32 x 32 squares: 1e-10);
the W-cycle and solve bars are those of the full-hierarchy tests.  At the
headline size (n = 512, four levels, coarsest 64 x 64 squares) the oracle's
dense coarsest solve does not finish in seconds, so the coarsest solve is
checked by its residual against the oracle's Galerkin product P^T ... L ... P
and the W-cycle by its contraction."""
import numpy as np
import pytest

from dcg_workloads import rhs
from layout import comp_to_elem, elem_to_comp
from oracle import discretisation as d
from oracle import krylov as kr
from oracle import multigrid as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2606_13429_amd._binding")
import paper_2606_13429_amd as dcg  # noqa: E402

DT = 1e-3


def _dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


_H = {}


def _hierarchy(n, levels):
    """The oracle's dt-free hierarchy (dt = 2: Z_J = L_J) with ``levels`` levels."""
    key = (n, levels)
    if key not in _H:
        V = d.deflation_basis(n)
        _H[key] = mg.Hierarchy((V.T @ d.operator(n, 2.0) @ V).tocsr(), n, coarsest=n >> (levels - 1))
        assert _H[key].J == levels
    return _H[key]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,levels", [(64, 2), (128, 3), (32, 1)])
def test_coarsest_fast_diagonalisation_solve(n, levels, prec):
    H = _hierarchy(n, levels)
    nc = H.n[1]
    real = torch.float32 if prec == "mixed" else torch.float64
    s = dcg.Solver(n, DT, prec=prec, levels=levels)
    f = np.random.default_rng(41).standard_normal(4 * nc * nc)
    out = torch.empty(4 * nc * nc, dtype=real, device="cuda")
    s.apply(lib.DCG_OP_COARSE, _dev(f, real), out, level=1)
    fr = _host(_dev(f, real))
    ref = np.linalg.solve(H.A[1].toarray(), fr)
    assert _relerr(_host(out), ref) < (1e-6 if prec == "mixed" else 1e-10)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,levels", [(64, 2), (128, 3)])
def test_wcycle_on_shortened_hierarchy(n, levels, prec):
    H = _hierarchy(n, levels)
    real = torch.float32 if prec == "mixed" else torch.float64
    s = dcg.Solver(n, DT, prec=prec, levels=levels)
    for k in range(1, levels + 1):
        nk = H.n[k]
        # FP32 cycle error ~ eps * kappa(L_k) ~ eps * n_k^2, as for the full hierarchy
        bar = 16 * float(np.finfo(np.float32).eps) * nk * nk if prec == "mixed" else 1e-10
        rng = np.random.default_rng(61 + k)
        f = rng.standard_normal(4 * nk * nk)
        z0 = rng.standard_normal(4 * nk * nk) * 1e-3
        out = torch.empty(4 * nk * nk, dtype=real, device="cuda")
        fr, zr = _host(_dev(f, real)), _host(_dev(z0, real))
        s.apply(lib.DCG_OP_WCYCLE, _dev(f, real), out, level=k)
        ref0 = mg.wcycle(H, fr, np.zeros_like(fr), k)
        got = _host(out)
        assert _relerr(got, ref0) < bar, k
        A = H.A[k]
        rho_gpu = np.linalg.norm(fr - A @ got) / np.linalg.norm(fr)
        rho_ref = np.linalg.norm(fr - A @ ref0) / np.linalg.norm(fr)
        assert abs(rho_gpu - rho_ref) <= (1e-3 if prec == "mixed" else 1e-9), (k, rho_gpu, rho_ref)
        s.apply(lib.DCG_OP_WCYCLE, _dev(f, real), out, level=k, in2=_dev(z0, real))
        assert _relerr(_host(out), mg.wcycle(H, fr, zr, k)) < bar, k
    # the shortened hierarchy has no level `levels + 1`
    with pytest.raises(lib.DCGError):
        s.apply(lib.DCG_OP_WCYCLE, _dev(np.zeros(4), real), torch.empty(4, dtype=real, device="cuda"),
                level=levels + 1)
    s.close()


_ORACLE = {}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,levels,dt", [(64, 2, 1e-4), (128, 3, 1e-5), (64, 1, 1e-3)])
def test_solve_on_shortened_hierarchy_matches_oracle(n, levels, dt, prec):
    key = (n, levels, dt)
    if key not in _ORACLE:
        As = d.operator(n, dt)
        V = d.deflation_basis(n)
        E = (V.T @ As @ V).tocsr()
        H = mg.Hierarchy(E, n, coarsest=n >> (levels - 1))
        _ORACLE[key] = kr.dcg(As, V, elem_to_comp(rhs(n, 4), n), kr.mg_inner(H), tol=1e-8)
    ref = _ORACLE[key]
    s = dcg.Solver(n, dt, prec=prec, levels=levels)
    b = torch.from_numpy(rhs(n, 4)).cuda()
    x = torch.empty_like(b)
    status, st = s.solve(b, x, 1e-8)
    torch.cuda.synchronize()
    assert status == lib.DCG_OK
    assert abs(st.outer_iters - ref.iterations) <= 2, (st.outer_iters, ref.iterations)
    xr = comp_to_elem(ref.x, n)
    assert _relerr(x.cpu().numpy(), xr) <= 1e-8
    assert st.rel_res_true <= 2e-8
    assert abs(st.inner_per_outer - np.mean(ref.outer_cycles)) <= 1.0
    if levels == 1:
        # the coarsest level is the finest: one exact cycle per inner solve in
        # FP64; the mixed form rounds the cycle's input and output to FP32, so
        # the FP64 refinement (Algorithm 3) takes a second cycle
        assert st.inner_per_outer == (1.0 if prec == "fp64" else 2.0)
    s.close()


def test_levels_rejected_where_unsupported():
    with pytest.raises(lib.DCGError):
        dcg.Solver(64, DT, levels=4)                  # J = 3 at n = 64
    with pytest.raises(lib.DCGError):
        dcg.Solver(64, DT, levels=-1)
    _, opt = lib.dcg_defaults()
    opt.levels = 2
    with pytest.raises(lib.DCGError):                 # the server runs the full hierarchy
        lib.dcg_server_create(opt)
    s = dcg.Solver(64, DT, levels=2)
    with pytest.raises(lib.DCGError):                 # the batched operators run the full hierarchy
        s.apply(lib.DCG_OP_WCYCLE_BATCH, torch.zeros(16 * 4 * 32 * 32, dtype=torch.float32, device="cuda"),
                torch.empty(16 * 4 * 32 * 32, dtype=torch.float32, device="cuda"), level=1)
    s.close()


def test_full_size_four_levels_coarsest_solve_and_contraction():
    n, levels = 512, 4
    L = d.sipg_laplacian(n).tocsr()
    Lc, nc = L, n
    for _ in range(levels - 1):                      # the oracle's Galerkin products
        P = mg.prolongation(nc // 2)
        Lc = (P.T @ Lc @ P).tocsr()
        nc //= 2
    assert nc == 64
    s = dcg.Solver(n, 1e-4, prec="fp64", levels=levels)
    f = np.random.default_rng(9).standard_normal(4 * nc * nc)
    out = torch.empty(4 * nc * nc, dtype=torch.float64, device="cuda")
    s.apply(lib.DCG_OP_COARSE, _dev(f), out, level=1)
    z = _host(out)
    s.close()
    # FP64 fast diagonalisation: residual ~ eps * kappa(L_1) relative
    assert np.isfinite(z).all()
    assert np.linalg.norm(f - Lc @ z) <= 1e-9 * np.linalg.norm(f)
    s = dcg.Solver(n, 1e-4, prec="mixed", levels=levels)
    m = 4 * n * n
    fJ = torch.from_numpy(np.random.default_rng(7).standard_normal(m)).to("cuda", torch.float32)
    w = torch.empty_like(fJ)
    s.apply(lib.DCG_OP_WCYCLE, fJ, w, level=levels)
    fh, wh = _host(fJ), _host(w)
    s.close()
    rho = np.linalg.norm(fh - L @ wh) / np.linalg.norm(fh)
    assert rho < 0.2, rho


def test_coarsest_solve_on_a_128_grid_by_residual():
    # n = 128 with one level: the fused passes with 2n = 256 (one thread group
    # per column, no partial sums), checked by the residual against the
    # oracle's SIPG Laplacian (the oracle's dense solve of 65,536 unknowns
    # does not finish in seconds)
    n = 128
    L = d.sipg_laplacian(n).tocsr()
    s = dcg.Solver(n, DT, prec="fp64", levels=1)
    f = np.random.default_rng(12).standard_normal(4 * n * n)
    out = torch.empty(4 * n * n, dtype=torch.float64, device="cuda")
    s.apply(lib.DCG_OP_COARSE, _dev(f), out, level=1)
    z = _host(out)
    s.close()
    assert np.isfinite(z).all()
    assert np.linalg.norm(f - L @ z) <= 1e-9 * np.linalg.norm(f)


@pytest.mark.parametrize("outer,c_A", [("fcg1", 0.01), ("cg", 0.01)])
def test_adaptive_tolerance_on_shortened_hierarchy_matches_oracle(outer, c_A):
    # the adaptive inner tolerance of eq. (tol) with a two-level hierarchy
    # (exact 32 x 32 coarsest level) against the oracle with the same depth;
    # the same gate as the full-hierarchy variant tests
    n, dt, tol, levels = 64, 1e-3, 1e-8, 2
    As = d.operator(n, dt)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = elem_to_comp(rhs(n, 6), n)
    kw = dict(outer="fcg", m_max=1) if outer == "fcg1" else dict(outer="cg")
    ref = kr.dcg(As, V, f, kr.mg_inner(mg.Hierarchy(E, n, coarsest=n >> (levels - 1))), tol=tol,
                 c_A=c_A, **kw)
    s = dcg.Solver(n, dt, prec="mixed", outer=outer, c_A=c_A, levels=levels)
    b = torch.from_numpy(rhs(n, 6)).cuda()
    x = torch.empty_like(b)
    status, st = s.solve(b, x, tol)
    torch.cuda.synchronize()
    s.close()
    xr = comp_to_elem(ref.x, n)
    assert status == lib.DCG_OK
    assert abs(st.outer_iters - ref.iterations) <= 2, (st.outer_iters, ref.iterations)
    assert st.rel_res_recurrence <= tol
    assert _relerr(x.cpu().numpy(), xr) <= 1e-8
    assert abs(st.total_wcycles - ref.total_cycles) <= 0.02 * ref.total_cycles + 10
    assert st.rel_res_true <= max(1.5 * ref.rel_res_true, 2 * tol)
