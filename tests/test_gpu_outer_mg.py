"""The outer multigrid preconditioner (dcg_options.outer_mg: one W-cycle on
A* as B in the flexible outer iteration) against the oracle
(oracle/precond.py, krylov.dcg(..., precond=B)).

Level operators: every DCG_OP_OMG_* operator element by element against the
oracle's hierarchy of A* (layout converted element-major <-> component-major),
at n = 16 (two levels) and n = 64 (four levels; the finest runs the brick
kernels, the others the small-level kernels).  Bar: max abs difference <=
1e-12 x max |oracle| for the single operators, 1e-11 for the W-cycle and B
(FP64, different summation order).  Solves: the preconditioned flexible
iteration against the oracle's at n = 16 and 32 (FP64 form: outer counts
within +-2, W-cycles within +-2 %, x within 1e-7; mixed form: counts within
+-2); graph replays of B equal direct launches bit for bit."""
import numpy as np
import pytest
import scipy.linalg as sla

from dcg_workloads import rhs
from layout import comp_to_elem, elem_to_comp, tensor_perm
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
