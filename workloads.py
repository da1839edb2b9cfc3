"""Seeded synthetic workloads shared by the oracle tests, the GPU parity tests
and the benchmark.

This module holds only problem parameters and random draws.  It contains none
of the multigrid method's arithmetic: no basis functions, no assembly, no
transfer operators, no smoother.  Each consumer turns these parameters into a
discrete problem with its own code.

Workloads (unit square / cube, homogeneous Dirichlet velocity, manufactured
solution u = curl psi with psi a product of sin^2, pressure a product of
sin(2 pi x_j)):

* ``small2d``   : 2D, k=1, 16x16 elements, 3 grids, nu = sigma = 1.
* ``stokes2d``  : 2D, k=2, 256x256 elements, 6 grids, nu = 1,
                  sigma in {1e-2, 1, 1e2, 1e4}.
* ``stokes3d``  : 3D, k=1, 32^3 elements, 4 grids, nu = 1, eight sigma drawn
                  log-uniformly in [1e-2, 1e4] with seed 3.
* ``oseen2d``   : 2D, k=2, 128x128 elements, 6 grids, sigma = 1,
                  nu in {1, 0.1, 0.01}, rotation advection a = c(-(y-1/2), x-1/2)
                  with |a| h / nu in {0, 0.25, 0.5, 1}, |a| = max |a| = c/sqrt(2).
* ``batch2d``   : 256 independent 2D problems (seed 5): N in {32, 64, 128},
                  k in {1, 2}, sigma log-uniform in [1e-2, 1e4], nu = 1,
                  |a| uniform in [0, 10] (rotation, c = sqrt(2)|a|), coarsest 4x4.
"""
import math
import numpy as np


def small2d():
    return dict(d=2, N=16, k=1, L=3, nu=1.0, sigma=1.0, c=0.0)


def stokes2d(sigma=1.0, N=256, L=6):
    return dict(d=2, N=N, k=2, L=L, nu=1.0, sigma=float(sigma), c=0.0)


STOKES2D_SIGMAS = (1e-2, 1.0, 1e2, 1e4)


def stokes3d_sigmas(n=8, seed=3):
    rng = np.random.default_rng(seed)
    return [float(10.0 ** x) for x in rng.uniform(-2.0, 4.0, n)]


def stokes3d(sigma=1.0, N=32, L=4):
    return dict(d=3, N=N, k=1, L=L, nu=1.0, sigma=float(sigma), c=0.0)


OSEEN2D_NUS = (1.0, 0.1, 0.01)
OSEEN2D_PEH = (0.0, 0.25, 0.5, 1.0)


def rotation_speed(nu, N, peh):
    """c such that max|a| h / nu = peh with h = 1/N and max|a| = c / sqrt(2)."""
    return math.sqrt(2.0) * nu * N * peh


def oseen2d(nu=1.0, peh=0.0, N=128, L=6):
    return dict(d=2, N=N, k=2, L=L, nu=float(nu), sigma=1.0, c=rotation_speed(nu, N, peh))


def batch2d(n=256, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.choice([32, 64, 128]))
        k = int(rng.choice([1, 2]))
        sigma = float(10.0 ** rng.uniform(-2.0, 4.0))
        amag = float(rng.uniform(0.0, 10.0))
        L = int(round(math.log2(N / 4))) + 1
        out.append(dict(d=2, N=N, k=k, L=L, nu=1.0, sigma=sigma, c=math.sqrt(2.0) * amag))
    return out


def random_coefficients(n, seed):
    """Coefficients uniform in (-1, 1): used for random divergence-free initial
    guesses (potential and pressure coefficients) and random vectors."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, int(n))
