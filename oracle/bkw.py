"""Exact collision operator of the BKW solution (Section 4.3), the oracle's pin.

For Maxwell molecules with B = 1/(4 pi), the spatially homogeneous equation
df/dt = Q(f,f) has the closed-form solution
  f = exp(-c^2/(2K)) / (2 (2 pi K)^{3/2}) ((5K-3)/K + (1-K)/K^2 c^2),
  K(t) = 1 - exp(-t/6),
valid for t > 6 ln 2.5, and Q(f,f) = df/dt is
  Q = K' (-3/(2K) + c^2/(2K^2)) f
      + K' exp(-c^2/(2K)) / (2 (2 pi K)^{3/2}) (3/K^2 + (K-2)/K^3 c^2),
  K' = exp(-t/6)/6.
"""
import numpy as np
from . import quadrature as qd


def K(t):
    return 1.0 - np.exp(-t / 6.0)


def f_exact(N, L, t):
    k = K(t)
    c1, c2, c3 = qd.grid3(N, L)
    c2s = c1 ** 2 + c2 ** 2 + c3 ** 2
    return np.exp(-c2s / (2 * k)) / (2 * (2 * np.pi * k) ** 1.5) * ((5 * k - 3) / k + (1 - k) / k ** 2 * c2s)


def Q_exact(N, L, t):
    k = K(t)
    kp = np.exp(-t / 6.0) / 6.0
    c1, c2, c3 = qd.grid3(N, L)
    c2s = c1 ** 2 + c2 ** 2 + c3 ** 2
    f = f_exact(N, L, t)
    g = np.exp(-c2s / (2 * k)) / (2 * (2 * np.pi * k) ** 1.5)
    return kp * (-1.5 / k + c2s / (2 * k ** 2)) * f + g * (3 / k ** 2 + (k - 2) / k ** 3 * c2s) * kp
