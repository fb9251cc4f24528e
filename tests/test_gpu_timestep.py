"""BDF2 time stepping (warm-started deflated CG with resident operators)
against the oracle's BDF2 recursion on the same seeded forcing."""
import numpy as np
import pytest

from dcg_workloads import forcing_load, fourier_modes
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
