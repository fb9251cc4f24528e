"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds input generation only: random right-hand sides, the
serving arrival trace and the smooth forcing of the time-stepping run.  It
contains none of the solver's arithmetic, and it is the only code that both
the HIP path's callers and the CPU oracle's callers use.

Vectors are returned in the library's element-major layout
``idx = 16 e + 4 c + j`` (e = ey * n + ex, c in {11, 12, 21, 22} order, local
corner j = ix + 2 iy).  The paper's experiments use meshes and data that are
not available here; these seeded inputs stand in for them.
"""
import numpy as np

# Configurations of the benchmark workloads (sizes and parameters)
SMALL = dict(n=16, dt=1e-2, tol=1e-8)                        # plain + exact inner
SWEEP = dict(n=128, dts=(1e-1, 1e-2, 1e-3, 1e-4, 1e-5), tol=1e-8)
HEADLINE = dict(n=512, dt=1e-4, tol=1e-8)                    # FP64 vs mixed form
SERVING = dict(count=256, rate=50.0, sizes=(32, 64, 128, 256), dt_range=(-6.0, -1.0), tol=1e-8)
TIMESTEP = dict(n=1024, dt=1e-5, steps=100, modes=8, seed=0)
# three-dimensional solver: n^3 cubes, penalty and mu of the 3D test of the paper
THREE_D = dict(n=32, dt=1e-3, tol=1e-8, penalty=40.0, nu=0.5)


def rhs(n, seed):
    """b ~ N(0, 1), length 16 n^2, element-major."""
    return np.random.default_rng(seed).standard_normal(16 * n * n)


def rhs3d(n, seed):
    """b ~ N(0, 1), length 72 n^3, in the 3D element-major layout
    idx = 72 e + 8 c + a."""
    return np.random.default_rng(seed).standard_normal(72 * n ** 3)


def serving_trace(seed=0, count=256, rate=50.0, sizes=(32, 64, 128, 256),
                  dt_range=(-6.0, -1.0)):
    """Poisson arrivals at ``rate`` requests/s; per request n uniform over
    ``sizes``, dt log-uniform over 10**dt_range and an RHS seed.

    Returns a list of dicts {t_arrival, n, dt, seed} sorted by arrival."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    ns = rng.choice(np.asarray(sizes), count)
    dts = 10.0 ** rng.uniform(dt_range[0], dt_range[1], count)
    seeds = rng.integers(2 ** 31, size=count)
    t = np.cumsum(gaps)
    return [dict(t_arrival=float(t[i]), n=int(ns[i]), dt=float(dts[i]), seed=int(seeds[i]))
            for i in range(count)]


def fourier_modes(seed=0, count=8):
    """Per stress component c: F_c(x, y) = sum_m a sin(2 pi (k x + l y) + phi)
    with k, l ~ U{0..4} (not both 0), a ~ N(0, 1)/count, phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 5, size=(4, count))
    l = rng.integers(0, 5, size=(4, count))
    both0 = (k == 0) & (l == 0)
    k[both0] = 1
    a = rng.standard_normal((4, count)) / count
    phi = rng.uniform(0.0, 2.0 * np.pi, (4, count))
    return dict(k=k, l=l, a=a, phi=phi)


def fourier_value(modes, c, x, y):
    """F_c at points (x, y) (arrays of equal shape)."""
    out = np.zeros(np.broadcast(x, y).shape)
    for m in range(modes['a'].shape[1]):
        out = out + modes['a'][c, m] * np.sin(
            2.0 * np.pi * (modes['k'][c, m] * x + modes['l'][c, m] * y) + modes['phi'][c, m])
    return out


def forcing_load(n, modes):
    """Discrete forcing f[16 e + 4 c + j] = int_K F_c phi_j, by the 2 x 2 Gauss
    rule on each square (the same rule the discretisation uses)."""
    h = 1.0 / n
    g = np.array([(1.0 - 1.0 / np.sqrt(3.0)) / 2.0, (1.0 + 1.0 / np.sqrt(3.0)) / 2.0])
    ex, ey = np.meshgrid(np.arange(n), np.arange(n))          # [ey, ex]
    out = np.zeros((n * n, 4, 4))
    for qy in range(2):
        for qx in range(2):
            x = (ex + g[qx]) * h
            y = (ey + g[qy]) * h
            phis = [(1 - g[qx]) * (1 - g[qy]), g[qx] * (1 - g[qy]), (1 - g[qx]) * g[qy], g[qx] * g[qy]]
            for c in range(4):
                val = fourier_value(modes, c, x, y).reshape(-1)
                for j in range(4):
                    out[:, c, j] += 0.25 * h * h * val * phis[j]
    return out.reshape(-1)
