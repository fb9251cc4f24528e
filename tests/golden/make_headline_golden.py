"""Writes the oracle's results for the headline-shaped solves (CPU only).

Calls only the oracle and the seeded input generators.  Two cases, both with
the four-level hierarchy of the paper's experiments (Section 5), Delta t =
1e-4, b = rhs(n, 0), tol 1e-8 and the fixed inner tolerance c_F = 0.01
(eq. (fixed_tol)), plain deflated CG (Algorithm 2 with the CG outer loop):

  n256   the full solve at n = 256 (coarsest level 32 x 32), with at most two
         warm restarts while the true residual misses tol; about two hours.
  n512   the first 30 outer iterations at n = 512 (coarsest level 64 x 64),
         the size of the benchmark, stopped by the iteration cap; about half
         an hour.  A full oracle solve at this size (some 20,000 W-cycles of
         several seconds each) does not fit a working session.

Each file holds the counts, residuals, ||x|| and x at 4096 fixed indices
(element-major layout 16 e + 4 c + j), drawn by default_rng(12345).

Usage:  python tests/golden/make_headline_golden.py n256|n512
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from dcg_workloads import rhs                                   # noqa: E402
from oracle import discretisation, krylov, multigrid            # noqa: E402

CASES = {
    "n256": dict(n=256, coarsest=32, max_iter=100000, restarts=2,
                 out="headline_n256_J4_seed0.txt"),
    "n512": dict(n=512, coarsest=64, max_iter=30, restarts=0,
                 out="headline_n512_J4_seed0_out30.txt"),
}
DT, TOL, SEED, C_F, SAMPLES = 1e-4, 1e-8, 0, 0.01, 4096


def sample_indices(n):
    rng = np.random.default_rng(12345)
    return np.sort(rng.choice(16 * n * n, SAMPLES, replace=False))


def main(name):
    c = CASES[name]
    n = c["n"]
    t0 = time.time()
    As = discretisation.operator(n, DT)
    V = discretisation.deflation_basis(n)
    E = (V.T @ As @ V).tocsr()
    H = multigrid.Hierarchy(E, n, coarsest=c["coarsest"])
    t_setup = time.time() - t0
    print("setup %.0f s, J = %d" % (t_setup, H.J), flush=True)
    b = rhs(n, SEED)
    f = b.reshape(n * n, 4, 4).transpose(1, 0, 2).reshape(-1)    # element -> component
    t0 = time.time()
    r = krylov.dcg(As, V, f, krylov.mg_inner(H), tol=TOL, max_iter=c["max_iter"], c_F=C_F,
                   restarts=c["restarts"])
    t_solve = time.time() - t0
    x = r.x.reshape(4, n * n, 4).transpose(1, 0, 2).reshape(-1)   # component -> element
    idx = sample_indices(n)
    path = os.path.join(HERE, c["out"])
    with open(path, "w") as fh:
        fh.write("# Oracle (CPU, FP64) deflated CG, Algorithm 2 with Algorithms 3-4 as the inner\n")
        fh.write("# solve: n = %d, dt = %g, tol = %g, c_F = %g (eq. (fixed_tol)), four levels\n"
                 % (n, DT, TOL, C_F))
        fh.write("# (coarsest %d x %d, dense Cholesky), m1 = m2 = 2, b = rhs(%d, %d), x0 = 0,\n"
                 % (c["coarsest"], c["coarsest"], n, SEED))
        fh.write("# max outer iterations %d, warm restarts <= %d.\n" % (c["max_iter"], c["restarts"]))
        fh.write("# Written by: python tests/golden/make_headline_golden.py %s\n" % name)
        fh.write("# oracle setup %.0f s, solve %.0f s (CPU, not a benchmark figure)\n"
                 % (t_setup, t_solve))
        fh.write("n %d\ncoarsest %d\ndt %r\ntol %r\nmax_iter %d\nrestarts_max %d\n"
                 % (n, c["coarsest"], DT, TOL, c["max_iter"], c["restarts"]))
        fh.write("outer %d\ntotal_cycles %d\nrestarts %d\n" % (r.iterations, r.total_cycles, r.restarts))
        fh.write("rel_res_recurrence %r\nrel_res_true %r\nx_norm %r\n"
                 % (float(r.rel_res_recurrence), float(r.rel_res_true), float(np.linalg.norm(x))))
        fh.write("# index value\n")
        for i in idx:
            fh.write("%d %r\n" % (i, float(x[i])))
    print("wrote %s: outer %d, Tot %d, restarts %d, true %.3e, %.0f s"
          % (path, r.iterations, r.total_cycles, r.restarts, r.rel_res_true, t_solve), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
