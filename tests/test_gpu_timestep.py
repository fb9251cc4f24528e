"""BDF2 time stepping (warm-started deflated CG with resident operators)
against the oracle's BDF2 recursion on the same seeded forcing."""
import os

import numpy as np
import pytest

from dcg_workloads import TIMESTEP, forcing_load, fourier_modes
from layout import comp_to_elem, elem_to_comp
from oracle import discretisation as d
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import timestep as ts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2606_13429_amd._binding")
from paper_2606_13429_amd.timestep import BDF2  # noqa: E402


def test_bdf2_steps_match_oracle():
    n, dt, steps, tol = 32, 1e-3, 5, 1e-8
    F_elem = forcing_load(n, fourier_modes(0))
    alpha = ts.bdf2_alpha(dt)
    As = d.operator(n, alpha)
    V = d.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    H = mg.Hierarchy(E, n)
    M = d.dev_mass(n)

    def solve(f, x0):
        r = kr.dcg(As, V, f, kr.mg_inner(H), tol=tol, x0=x0)
        return r.x, r.iterations

    ref, ref_iters = ts.bdf2(M, elem_to_comp(F_elem, n), dt, steps, solve)

    for prec in ("fp64", "mixed"):
        stepper = BDF2(n, dt, prec=prec, tol=tol)
        F = torch.from_numpy(F_elem).cuda()
        iters = [stepper.step(F).outer_iters for _ in range(steps)]
        torch.cuda.synchronize()
        x = stepper.state.cpu().numpy()
        xr = comp_to_elem(ref, n)
        assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr), prec
        assert all(abs(a - b) <= 2 for a, b in zip(iters, ref_iters)), (iters, ref_iters)
        # warm starts pay off once the history is non-zero
        assert iters[-1] < iters[0]


def test_bdf2_rhs_sampled_at_full_size():
    # the time-stepping workload's size: 1024 x 1024 squares; the right-hand
    # side kernel is checked on sampled squares against the oracle's element
    # blocks (M = (1/nu) C (x) M_1 square by square)
    n, dt, nu = 1024, 1e-5, 1.0
    stepper = BDF2(n, dt, nu=nu, prec="mixed", max_outer=1)
    rng = np.random.default_rng(5)
    N = 16 * n * n
    s1 = torch.from_numpy(rng.standard_normal(N)).cuda()
    s2 = torch.from_numpy(rng.standard_normal(N)).cuda()
    F = torch.from_numpy(rng.standard_normal(N)).cuda()
    f = torch.empty_like(s1)
    x0 = torch.empty_like(s1)
    c = 2.0 * dt / 3.0
    lib.dcg_bdf2_rhs(stepper.solver.handle, s1, s2, F, c, f, x0)
    torch.cuda.synchronize()
    C = d.dev_coefficients(2)
    Me = np.kron(C, d.element_mass(1.0 / n)) / nu
    s1h, s2h, Fh, fh, x0h = (t.cpu().numpy() for t in (s1, s2, F, f, x0))
    for e in list(rng.integers(0, n * n, 64)) + [0, n - 1, n * n - 1]:
        sl = slice(16 * e, 16 * e + 16)
        u = 4.0 / 3.0 * s1h[sl] - 1.0 / 3.0 * s2h[sl]
        ref = Me @ u + c * Fh[sl]
        assert np.allclose(fh[sl], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert np.array_equal(x0h[sl], 2.0 * s1h[sl] - s2h[sl])


GOLDEN_BDF2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "bdf2_n32_dt1e-5_100steps.txt")


def _bdf2_golden():
    rows, samples, final = [], [], None
    with open(GOLDEN_BDF2) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "step":
                rows.append((int(t[2]), int(t[3]), float(t[4])))
            elif t[0] == "final_norm":
                final = float(t[1])
            elif t[0] == "x":
                samples.append((int(t[1]), float(t[2])))
    return rows, final, samples


@pytest.mark.skipif(not os.path.exists(GOLDEN_BDF2), reason="oracle golden file not written")
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bdf2_100_steps_match_stored_oracle(prec):
    # the workload's 100 steps (dt = 1e-5, its forcing) on a 32 x 32 grid
    # against the oracle's run (tests/golden/make_bdf2_golden.py): every
    # step's outer count within +-2 and its state norm, and the final state
    # at 256 sampled entries.  Each solve stops at a relative residual of
    # 1e-8 and the states of both runs carry that error from step to step
    # (BDF2 is stable, so it does not grow); the bars allow 2e-8 of ||s||.
    rows, final, samples = _bdf2_golden()
    n, dt = 32, 1e-5
    print("bdf2 100 steps n=%d %s" % (n, prec), flush=True)
    F = torch.from_numpy(forcing_load(n, fourier_modes(TIMESTEP["seed"], TIMESTEP["modes"]))).cuda()
    stepper = BDF2(n, dt, prec=prec, tol=1e-8)
    worst = 0.0
    for k, (outer, _, nrm) in enumerate(rows):
        st = stepper.step(F)
        assert abs(st.outer_iters - outer) <= 2, (k + 1, st.outer_iters, outer)
        got = torch.linalg.norm(stepper.state).item()
        worst = max(worst, abs(got - nrm) / nrm)
    x = stepper.state.cpu().numpy()
    err = max(abs(x[i] - v) for i, v in samples) / final
    print("  worst step norm difference %.2e, final sampled difference %.2e" % (worst, err), flush=True)
    assert worst <= 2e-8 and err <= 2e-8
