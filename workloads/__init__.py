"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the collision method: it only produces the
arrays that both sides read (distribution functions on the velocity grid,
cotangents, and the half-sphere quadrature rules, which the paper takes as
given data from Womersley's design files).

Velocity grid (Section 3.3): c_j = -L + (j + 1/2) dc with 0-based j and
dc = 2L/N, index order (j1, j2, j3) <-> (c1, c2, c3), C-order arrays.

Recipes
-------
* ``maxwellian_mixture``: each item is the sum of two Maxwellians
  n/(pi T)^{3/2} exp(-|c-u|^2/T) (initial-condition formula of Section 3.5)
  with per-item draws, in this order: n1, n2 ~ U[n_lo, n_hi]; T1, T2 ~
  U[T_lo, T_hi]; then u1, u2, each a unit vector from a normalised N(0, I3)
  times |u| = u_max * U^{1/3}; then a multiplicative noise field
  f <- f * (1 + noise * U[0,1)) that keeps f positive and decaying.
* ``bkw``: the Bobylev-Krook-Wu closed form of Section 4.3 at time t.
* ``cotangent``: g = f * N(0,1) (adjoint checks).
"""
import os
import numpy as np

_SPHERE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere")


def velocity_grid(N, L):
    """1-D cell-centred nodes -L + (j+1/2) 2L/N, j = 0..N-1."""
    dc = 2.0 * L / N
    return -L + (np.arange(N) + 0.5) * dc


def grid3(N, L):
    c = velocity_grid(N, L)
    return np.meshgrid(c, c, c, indexing="ij")


def sphere_rule(M):
    """Equal-weight half-sphere rule: (points [M,3], weights [M]), sum w = 2 pi."""
    path = os.path.join(_SPHERE_DIR, f"half_M{M}.txt")
    if not os.path.exists(path):
        raise ValueError(f"no half-sphere rule with M={M} (have 6, 12, 16)")
    a = np.loadtxt(path)
    return np.ascontiguousarray(a[:, :3]), np.ascontiguousarray(a[:, 3])


def maxwellian(N, L, n, u, T):
    c1, c2, c3 = grid3(N, L)
    r2 = (c1 - u[0]) ** 2 + (c2 - u[1]) ** 2 + (c3 - u[2]) ** 2
    return n / (np.pi * T) ** 1.5 * np.exp(-r2 / T)


def maxwellian_mixture(n_items, N, L, seed, n_range=(0.5, 1.5), T_range=(0.5, 2.0),
                       u_max=0.5, noise=0.01):
    """[n_items, N, N, N] float64 mixtures of two Maxwellians (recipe above)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n_items, N, N, N))
    for i in range(n_items):
        n1, n2 = rng.uniform(*n_range, size=2)
        T1, T2 = rng.uniform(*T_range, size=2)
        us = []
        for _ in range(2):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            us.append(d * u_max * rng.uniform() ** (1.0 / 3.0))
        f = maxwellian(N, L, n1, us[0], T1) + maxwellian(N, L, n2, us[1], T2)
        if noise:
            f *= 1.0 + noise * rng.uniform(size=f.shape)
        out[i] = f
    return out


def bkw(N, L, t):
    """BKW solution of Section 4.3 at time t on the N^3 grid (B = 1/(4 pi))."""
    K = 1.0 - np.exp(-t / 6.0)
    c1, c2, c3 = grid3(N, L)
    c2sum = c1 ** 2 + c2 ** 2 + c3 ** 2
    return (np.exp(-c2sum / (2 * K)) / (2 * (2 * np.pi * K) ** 1.5)
            * ((5 * K - 3) / K + (1 - K) / K ** 2 * c2sum))


def cotangent(f, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return f * rng.normal(size=f.shape)


# Workload definitions: the synthetic stand-ins for the paper's physics cases.
WORKLOADS = {
    # space-homogeneous BKW relaxation, Maxwell molecules
    "bkw16": dict(N=16, L=8.0, M=6, N_rho=8, omega=1.0, prefactor=1.0 / (4 * np.pi), items=1),
    # 1D DG batch: 64 elements x 3 Gauss points
    "dg1d_32": dict(N=32, L=6.0, M=12, N_rho=16, omega=0.81, prefactor=None, items=192,
                    svd_tol=1e-8, seed=2),
    # 2D DG batch: 32x32 elements x 2x2 Gauss points
    "dg2d_24": dict(N=24, L=6.0, M=12, N_rho=12, omega=0.74, prefactor=None, items=4096, seed=3),
    # adjoint check
    "adjoint_32": dict(N=32, L=6.0, M=12, N_rho=16, omega=0.81, prefactor=None, items=256, seed=4),
}

# Uneven batch over three velocity grids (shock-like hot/cold states): 2048
# points split 50/35/15 % (rounded half-to-even: 1024/717/307), each grid with
# its own temperature band and maximum drift; M = 12, omega = 0.81, gain table
# truncated by SVD at 1e-6.
UNEVEN = [
    dict(N=24, L=6.0, N_rho=16, items=1024, T_range=(1.0, 1.5), u_max=0.5, seed=5),
    dict(N=32, L=7.0, N_rho=16, items=717, T_range=(1.5, 2.5), u_max=1.2, seed=6),
    dict(N=48, L=9.0, N_rho=24, items=307, T_range=(2.5, 3.5), u_max=2.3, seed=7),
]
UNEVEN_COMMON = dict(M=12, omega=0.81, svd_tol=1e-6)


def uneven_grid(i, items=None):
    g = UNEVEN[i]
    n = g["items"] if items is None else items
    return maxwellian_mixture(n, g["N"], g["L"], g["seed"], T_range=g["T_range"], u_max=g["u_max"])


def mixture_for(name, items=None):
    w = WORKLOADS[name]
    n = w["items"] if items is None else items
    return maxwellian_mixture(n, w["N"], w["L"], w["seed"])
