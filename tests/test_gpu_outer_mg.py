"""The outer multigrid preconditioner (dcg_options.outer_mg: one W-cycle on
A* as B in the flexible outer iteration) against the oracle
(oracle/precond.py, krylov.dcg(..., precond=B)).

Level operators: every DCG_OP_OMG_* operator element by element against the
oracle's hierarchy of A* (layout converted element-major <-> component-major),
at n = 16 (two levels, the small-level split kernels) and n = 64 (four
levels; the finest runs the MFMA brick kernels, interior and boundary
bricks).  Bar: max abs difference <= 1e-12 x max |oracle| for the single
operators, 1e-11 for the W-cycle and B (FP64, different summation order).
The MFMA brick kernels on sampled squares of the levels 128 (n = 128) and
512, 256, 128 (n = 512),
against the oracle's rows evaluated square by square on a 16 x 16 window
(tests/window2d.py): A*_k z 1e-12, the RAS step from zero and from a start
1e-11.  Solves: the preconditioned flexible iteration against the oracle's at
n = 16 and 32 (FP64 form: outer counts within +-2, W-cycles within +-2 %, x
within 1e-7; mixed form: counts within +-2); at n = 512, dt = 1e-4 (the
benchmark's size, four inner levels) the solve converges to the true
residual; graph replays of B equal direct launches bit for bit."""
import numpy as np
import pytest
import scipy.linalg as sla

from dcg_workloads import rhs
from layout import comp_to_elem, elem_to_comp, tensor_perm
from window2d import Window, sample_squares
from oracle import discretisation as d
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import precond as pc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2606_13429_amd._binding")
import paper_2606_13429_amd as dcg  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _close(got, ref, rel):
    err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
    assert err <= rel, "max rel error %.3e" % err


def _solver(n, dt, prec="fp64", m=2, **kw):
    return dcg.Solver(n, dt, prec=prec, outer="fcg", m_max=8, outer_mg=m, **kw)


@pytest.mark.parametrize("n,dt,m", [(16, 1e-2, 2), (64, 1e-3, 1)])
def test_level_operators_match_oracle(n, dt, m):
    print("outer mg operators n=%d dt=%g m=%d" % (n, dt, m), flush=True)
    H = pc.Hierarchy(d.operator(n, dt), n)
    s = _solver(n, dt, m=m)
    rng = np.random.default_rng(n)

    def call(op, k, x, x2=None, size=None):
        out = torch.empty(size or x.size, dtype=torch.float64, device="cuda")
        s.apply(op, _dev(x), out, level=k, in2=None if x2 is None else _dev(x2))
        return _host(out)

    for k in range(1, H.J + 1):
        nk = H.n[k]
        pe, pc_ = tensor_perm(nk), np.argsort(tensor_perm(nk))   # comp = elem[pe]; elem = comp[pc_]
        f, z = rng.standard_normal(16 * nk * nk), rng.standard_normal(16 * nk * nk)
        A = H.A[k]
        _close(call(lib.DCG_OP_OMG_LEVEL, k, z), (A @ z[pe])[pc_], 1e-12)
        if k >= 2:
            _close(call(lib.DCG_OP_OMG_RAS, k, f), H.S[k].apply(f[pe])[pc_], 1e-12)
            ref = z[pe] + H.S[k].apply(f[pe] - A @ z[pe])
            _close(call(lib.DCG_OP_OMG_RAS, k, f, z), ref[pc_], 1e-12)
            nc = H.n[k - 1]
            rc = call(lib.DCG_OP_OMG_RESTRICT, k, f, size=16 * nc * nc)
            _close(rc, (H.P[k].T @ f[pe])[np.argsort(tensor_perm(nc))], 1e-12)
            e = rng.standard_normal(16 * nc * nc)
            _close(call(lib.DCG_OP_OMG_PROLONG, k, e, size=16 * nk * nk),
                   (H.P[k] @ e[tensor_perm(nc)])[pc_], 1e-12)
        else:
            _close(call(lib.DCG_OP_OMG_COARSE, 1, f), sla.cho_solve(H.chol, f[pe])[pc_], 1e-11)
        _close(call(lib.DCG_OP_OMG_WCYCLE, k, f), mg.wcycle(H, f[pe], np.zeros(f.size), k, m, m)[pc_], 1e-11)
        _close(call(lib.DCG_OP_OMG_WCYCLE, k, f, z), mg.wcycle(H, f[pe], z[pe], k, m, m)[pc_], 1e-11)
    r = rng.standard_normal(16 * n * n)
    B = pc.preconditioner(H, m)
    got = call(lib.DCG_OP_OMG_APPLY, H.J, r)
    _close(got, B(r[tensor_perm(n)])[np.argsort(tensor_perm(n))], 1e-11)
    s.close()
    # graph replays equal direct launches
    s2 = _solver(n, dt, m=m, use_graph=False)
    out = torch.empty(16 * n * n, dtype=torch.float64, device="cuda")
    s2.apply(lib.DCG_OP_OMG_APPLY, _dev(r), out, level=H.J)
    assert np.array_equal(_host(out), got)
    s2.close()


def _oracle(n, dt, m, tol):
    As = d.operator(n, dt)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = elem_to_comp(rhs(n, 0), n)
    inner = kr.mg_inner(mg.Hierarchy(E, n))
    B = pc.preconditioner(pc.Hierarchy(As, n), m)
    return kr.dcg(As, V, f, inner, tol=tol, outer='fcg', m_max=8, precond=B)


@pytest.mark.parametrize("n,dt", [(16, 1e-2), (32, 1e-3), (32, 1e-1)])
def test_preconditioned_solve_matches_oracle(n, dt):
    tol, m = 1e-8, 2
    print("outer mg solve n=%d dt=%g" % (n, dt), flush=True)
    res = _oracle(n, dt, m, tol)
    b = _dev(rhs(n, 0))
    for prec in ("fp64", "mixed"):
        s = _solver(n, dt, prec=prec, m=m)
        x = torch.empty_like(b)
        status, st = s.solve(b, x, tol)
        s.close()
        print("  %s: Out %d (oracle %d) Tot %d (oracle %d)"
              % (prec, st.outer_iters, res.iterations, st.total_wcycles, res.total_cycles), flush=True)
        assert status == lib.DCG_OK
        assert abs(st.outer_iters - res.iterations) <= 2
        assert st.rel_res_true <= 10 * tol
        if prec == "fp64":
            assert abs(st.total_wcycles - res.total_cycles) <= max(2, 0.02 * res.total_cycles)
            xg = elem_to_comp(_host(x), n)
            assert np.linalg.norm(xg - res.x) <= 1e-7 * np.linalg.norm(res.x)


def test_warm_started_preconditioned_solve_matches_oracle():
    # the time-stepping use: x0 given (here a rough guess), FCG(8) with B,
    # against the oracle's dcg(x0=...) with the same B
    n, dt, tol, m = 32, 1e-2, 1e-8, 2
    print("outer mg warm start n=%d dt=%g" % (n, dt), flush=True)
    As = d.operator(n, dt)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    f = elem_to_comp(rhs(n, 1), n)
    x0 = 0.1 * elem_to_comp(rhs(n, 2), n)
    inner = kr.mg_inner(mg.Hierarchy(E, n))
    B = pc.preconditioner(pc.Hierarchy(As, n), m)
    res = kr.dcg(As, V, f, inner, tol=tol, outer='fcg', m_max=8, precond=B, x0=x0)
    s = _solver(n, dt, m=m, x0_given=True)
    b = _dev(rhs(n, 1))
    x = _dev(comp_to_elem(x0, n))
    status, st = s.solve(b, x, tol)
    s.close()
    print("  Out %d (oracle %d) Tot %d (oracle %d)" % (st.outer_iters, res.iterations,
                                                      st.total_wcycles, res.total_cycles), flush=True)
    assert status == lib.DCG_OK and st.rel_res_true <= 10 * tol
    assert abs(st.outer_iters - res.iterations) <= 2
    assert abs(st.total_wcycles - res.total_cycles) <= max(2, 0.02 * res.total_cycles)
    xg = elem_to_comp(_host(x), n)
    assert np.linalg.norm(xg - res.x) <= 1e-7 * np.linalg.norm(res.x)


@pytest.mark.parametrize("n", [128, 512])
def test_full_size_level_steps_on_sampled_squares(n):
    dt = 1e-4
    print("outer mg large levels n=%d" % n, flush=True)
    s = _solver(n, dt, levels=4)
    rng = np.random.default_rng(n)
    J = 1
    while 8 << (J - 1) < n:
        J += 1
    for k in range(J, 0, -1):
        nk = 8 << (k - 1)
        if nk <= 64:
            break
        f, z = rng.standard_normal(16 * nk * nk), rng.standard_normal(16 * nk * nk)
        got = []
        for op, a, b in ((lib.DCG_OP_OMG_LEVEL, z, None), (lib.DCG_OP_OMG_RAS, f, None),
                         (lib.DCG_OP_OMG_RAS, f, z)):
            out = torch.empty(16 * nk * nk, dtype=torch.float64, device="cuda")
            s.apply(op, _dev(a), out, level=k, in2=None if b is None else _dev(b))
            got.append(_host(out))
        W = Window(nk, n, dt)
        ref = {(x, y): (W.rows(z, x, y), W.ras(f, x, y), W.ras(f, x, y, z))
               for x, y in sample_squares(nk, seed=k)}
        scale = [max(np.abs(r[i]).max() for r in ref.values()) for i in range(3)]
        for (x, y), r in ref.items():
            sl = slice(16 * (y * nk + x), 16 * (y * nk + x) + 16)
            for i, bar in enumerate((1e-12, 1e-11, 1e-11)):
                err = np.abs(got[i][sl] - r[i]).max() / scale[i]
                assert err <= bar, (nk, x, y, i, err)
        print("  level %d (%d squares per side): %d squares checked" % (k, nk, len(ref)), flush=True)
    s.close()


def test_full_size_preconditioned_solve():
    n, dt, tol = 512, 1e-4, 1e-8
    print("outer mg solve n=%d dt=%g" % (n, dt), flush=True)
    s = dcg.Solver(n, dt, prec="mixed", outer="fcg", m_max=8, outer_mg=2, levels=4, max_outer=400)
    b = _dev(rhs(n, 0))
    x = torch.empty_like(b)
    status, st = s.solve(b, x, tol)
    s.close()
    print("  Out %d Tot %d true residual %.3e" % (st.outer_iters, st.total_wcycles, st.rel_res_true),
          flush=True)
    # deflated CG without the preconditioner needs 2092 outer iterations here
    assert status == lib.DCG_OK and st.rel_res_true <= tol
    assert st.outer_iters <= 100


def test_options_are_checked():
    with pytest.raises(lib.DCGError):
        dcg.Solver(16, 1e-3, outer="cg", outer_mg=2)
    with pytest.raises(lib.DCGError):
        dcg.Solver(16, 1e-3, outer="fcg", outer_mg=-1)
    s = dcg.Solver(16, 1e-3, outer="fcg")
    with pytest.raises(lib.DCGError):
        s.apply(lib.DCG_OP_OMG_LEVEL, _dev(np.zeros(16 * 256)),
                torch.empty(16 * 256, dtype=torch.float64, device="cuda"), level=1)
    s.close()
    _, opt = lib.dcg_defaults()
    opt.outer, opt.outer_mg = lib.DCG_OUTER_FCG, 2
    with pytest.raises(lib.DCGError):
        lib.dcg_server_create(opt)
