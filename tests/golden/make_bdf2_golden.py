"""Writes the oracle's BDF2 time stepping over the workload's 100 steps on a
small grid (CPU only): n = 32 squares per side, dt = 1e-5 (alpha = 2 dt / 3),
the workload's forcing (8 Fourier modes per stress component, seed 0), zero
history, warm start 2 s^{n-1} - s^{n-2}, tol 1e-8, deflated CG with the
W-cycle multigrid inner solve on the full hierarchy (coarsest 16 x 16,
dense Cholesky), c_F = 0.01.

Calls only the oracle and the seeded input generators.  A few minutes on one
core.  Each step's row holds its outer iterations, W-cycles and ||s^n||; the
final state follows at 256 fixed indices of the element-major layout
16 e + 4 c + j, drawn by default_rng(2024), with ||s^100||.

Usage:  python tests/golden/make_bdf2_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N, DT, STEPS, TOL, SAMPLES = 32, 1e-5, 100, 1e-8, 256
OUT = "bdf2_n32_dt1e-5_100steps.txt"


def sample_indices():
    return np.sort(np.random.default_rng(2024).choice(16 * N * N, SAMPLES, replace=False))


def main():
    from dcg_workloads import TIMESTEP, forcing_load, fourier_modes
    from oracle import discretisation as d
    from oracle import krylov as kr
    from oracle import multigrid as mg
    from oracle import timestep as ts

    t0 = time.time()
    F_elem = forcing_load(N, fourier_modes(TIMESTEP["seed"], TIMESTEP["modes"]))
    F = F_elem.reshape(N * N, 4, 4).transpose(1, 0, 2).reshape(-1)   # component-major
    alpha = ts.bdf2_alpha(DT)
    As = d.operator(N, alpha)
    V = d.deflation_basis(N)
    E = (V.T @ As @ V).tocsr()
    H = mg.Hierarchy(E, N)
    M = d.dev_mass(N)

    def solve(f, x0):
        r = kr.dcg(As, V, f, kr.mg_inner(H), tol=TOL, x0=x0)
        return r.x, (r.iterations, r.total_cycles, float(np.linalg.norm(r.x)))

    final, records = ts.bdf2(M, F, DT, STEPS, solve)
    x_elem = final.reshape(4, N * N, 4).transpose(1, 0, 2).reshape(-1)
    idx = sample_indices()
    with open(os.path.join(HERE, OUT), "w") as fh:
        fh.write("# BDF2, n = %d, dt = %g, %d steps, tol %g, workload forcing (seed %d, %d modes)\n"
                 % (N, DT, STEPS, TOL, TIMESTEP["seed"], TIMESTEP["modes"]))
        fh.write("# written by tests/golden/make_bdf2_golden.py (oracle only)\n")
        fh.write("# step outer wcycles norm\n")
        for k, (o, c, nrm) in enumerate(records):
            fh.write("step %d %d %d %.17e\n" % (k + 1, o, c, nrm))
        fh.write("final_norm %.17e\n" % np.linalg.norm(x_elem))
        for i in idx:
            fh.write("x %d %.17e\n" % (i, x_elem[i]))
    print("wrote %s in %.0f s" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
