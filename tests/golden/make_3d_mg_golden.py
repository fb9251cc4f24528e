"""Writes the oracle's deflated CG with the three-dimensional multigrid inner
solve (CPU only): the analogue of Table 5 (right) on the hexahedral grid.

Calls only the oracle and the seeded input generators.  n = 8 cubes per side
(the finest of three nested levels 8, 4, 2, as the paper's mesh 3 refines
mesh 1 twice), mu = 0.5, penalty 40, Delta t in {0.5, 0.1, 1e-2, 1e-3, 1e-4},
tol 1e-8, b = rhs3d(8, 0), x0 = 0, W-cycles with m = 10 pre- and
post-smoothing RAS steps; the inner tolerance by eq. (fixed_tol) with
c_F = 0.01 and by eq. (tol) with c_A = 0.02 and 0.005, plain deflated CG
(Algorithm 2 with the CG outer loop).  About half an hour on eight cores.

Each row holds Out, Tot, the number of inner solves, the recurrence and true
residuals and ||x||; for every case x at 128 fixed indices of the
element-major layout 72 e + 8 c + a, drawn by default_rng(12345).

Usage:  python tests/golden/make_3d_mg_golden.py
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N, SEED, TOL, NU, PEN, M, SAMPLES = 8, 0, 1e-8, 0.5, 40.0, 10, 128
DTS = (0.5, 0.1, 1e-2, 1e-3, 1e-4)
RULES = (("F", 0.01), ("A", 0.02), ("A", 0.005))
OUT = "mg3d_table5_n8_seed0.txt"


def sample_indices():
    return np.sort(np.random.default_rng(12345).choice(72 * N ** 3, SAMPLES, replace=False))


def run(case):
    from dcg_workloads import rhs3d
    from oracle import discretisation3d, krylov, multigrid3d
    dt, rule, c = case
    As = discretisation3d.operator(N, dt, nu=NU, penalty=PEN)
    V = discretisation3d.deflation_basis(N)
    E = (V.T @ As @ V).tocsr()
    H = multigrid3d.Hierarchy(E, N)
    b = rhs3d(N, SEED)
    f = b.reshape(N ** 3, 9, 8).transpose(1, 0, 2).reshape(-1)      # element -> component
    t0 = time.time()
    kw = dict(c_F=c) if rule == "F" else dict(c_A=c)
    r = krylov.dcg(As, V, f, krylov.mg_inner(H, M, M), tol=TOL, max_iter=20000, **kw)
    x = r.x.reshape(9, N ** 3, 8).transpose(1, 0, 2).reshape(-1)     # component -> element
    print("dt %g %s %g: Out %d Tot %d true %.2e, %.0f s" % (dt, rule, c, r.iterations, r.total_cycles,
                                                           r.rel_res_true, time.time() - t0), flush=True)
    return (dt, rule, c, r.iterations, r.total_cycles, len(r.cycles), float(r.rel_res_recurrence),
            float(r.rel_res_true), float(np.linalg.norm(x)), x[sample_indices()])


def main():
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    cases = [(dt, rule, c) for dt in DTS for rule, c in RULES]
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=8) as ex:
        rows = list(ex.map(run, cases))
    idx = sample_indices()
    with open(os.path.join(HERE, OUT), "w") as fh:
        fh.write("# Oracle (CPU, FP64) deflated CG, Algorithm 2 with Algorithms 3-4 as the inner\n")
        fh.write("# solve on the three-dimensional hierarchy (levels 8, 4, 2, Galerkin, RAS blocks of\n")
        fh.write("# a cube and its face neighbours, m = %d, exact solve on level 1): n = %d, mu = %g,\n"
                 % (M, N, NU))
        fh.write("# penalty %g, tol %g, b = rhs3d(%d, %d), x0 = 0; the analogue of Table 5 (right).\n"
                 % (PEN, TOL, N, SEED))
        fh.write("# Written by: python tests/golden/make_3d_mg_golden.py (%.0f s on the CPU)\n"
                 % (time.time() - t0))
        fh.write("# row dt rule(F: c_F, A: c_A) c outer total_cycles inner_solves rel_res_recurrence "
                 "rel_res_true x_norm\n")
        for r in rows:
            fh.write("row %r %s %r %d %d %d %r %r %r\n" % r[:9])
        fh.write("# x dt rule c index value (element-major 72 e + 8 c + a)\n")
        for r in rows:
            for i, v in zip(idx, r[9]):
                fh.write("x %r %s %r %d %r\n" % (r[0], r[1], r[2], i, float(v)))


if __name__ == "__main__":
    main()
