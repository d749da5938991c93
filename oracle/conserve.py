"""Moments (midpoint rule) and the conservation projection, FP64.

* Moments (Section 3.3, midpoint-rule moments of the rescaled equations):
  n = sum f dc^3,  u = sum f c dc^3 / n,  T = 2/(3n) sum f |c-u|^2 dc^3,
  P = 2 sum f (c-u)(c-u)^T dc^3,  q = sum f (c-u)|c-u|^2 dc^3.
  Output order: n, u1..u3, T, P11, P12, P13, P22, P23, P33, q1..q3 (14 values).
* Conservation projection (not in the paper; the standard constrained
  least-squares correction of the spectral-method literature): with the rows
  of C = [1, c1, c2, c3, |c|^2] evaluated on the grid,
  Q_c = Q - C^T (C C^T)^{-1} C Q, the Euclidean-nearest vector to Q whose
  discrete mass, momentum and energy moments vanish.  The dc^3 factor of the
  moment sums cancels.
"""
import numpy as np
from . import quadrature as qd


def invariants(N, L):
    c1, c2, c3 = qd.grid3(N, L)
    return np.stack([np.ones_like(c1), c1, c2, c3, c1 ** 2 + c2 ** 2 + c3 ** 2]).reshape(5, -1)


def project(Q, N, L):
    """Returns (Q_c, m) with m = C Q the pre-projection invariant sums (no dc^3)."""
    C = invariants(N, L)
    shape = Q.shape
    Qf = Q.reshape(-1, N ** 3)
    m = Qf @ C.T
    lam = np.linalg.solve(C @ C.T, m.T).T
    out = Qf - lam @ C
    return out.reshape(shape), m.reshape(shape[:-3] + (5,))


def moments(f, N, L):
    dc3 = (2.0 * L / N) ** 3
    c = np.stack(qd.grid3(N, L)).reshape(3, -1)
    ff = f.reshape(-1, N ** 3)
    out = np.empty((ff.shape[0], 14))
    for i, g in enumerate(ff):
        n = g.sum() * dc3
        u = (c * g).sum(axis=1) * dc3 / n
        d = c - u[:, None]
        d2 = (d ** 2).sum(axis=0)
        T = 2.0 / (3.0 * n) * (g * d2).sum() * dc3
        P = 2.0 * np.einsum("j,aj,bj->ab", g, d, d) * dc3
        q = (d * (g * d2)).sum(axis=1) * dc3
        out[i] = [n, *u, T, P[0, 0], P[0, 1], P[0, 2], P[1, 1], P[1, 2], P[2, 2], *q]
    return out.reshape(f.shape[:-3] + (14,))


def conservation_residual(Q, N, L):
    """Per-invariant |sum Q phi_i| / sum |Q phi_i| (normwise relative residual)."""
    C = invariants(N, L)
    Qf = Q.reshape(-1, N ** 3)
    num = np.abs(Qf @ C.T)
    den = np.abs(Qf) @ np.abs(C).T
    return (num / np.maximum(den, 1e-300)).reshape(Q.shape[:-3] + (5,))
