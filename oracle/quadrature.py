"""Velocity grid, Fourier frequencies and the radial Gauss-Legendre rule.

* Grid (Section 3.3): N uniform cell-centred points per axis on [-L, L],
  c_j = -L + (j - 1/2) dc for j = 1..N (here 0-based: -L + (j + 1/2) dc),
  dc = 2L/N.
* Frequencies (Appendix, truncated Fourier series): k = -N/2 .. N/2-1.  The
  DFT index n maps to the signed frequency kappa(n) = n for n < N/2 and n - N
  otherwise, so the self-paired index n = N/2 is kappa = -N/2.
* Ball truncation (Appendix): R = 4L/(3 + sqrt 2).
* Radial rule (Appendix, paragraph after the quadrature form): Gauss-Legendre
  with N_rho nodes on [0, R].
"""
import numpy as np


def grid(N, L):
    dc = 2.0 * L / N
    return -L + (np.arange(N) + 0.5) * dc


def grid3(N, L):
    c = grid(N, L)
    return np.meshgrid(c, c, c, indexing="ij")


def kappa(N):
    n = np.arange(N)
    return np.where(n < N // 2, n, n - N).astype(float)


def kappa3(N):
    k = kappa(N)
    return np.meshgrid(k, k, k, indexing="ij")


def ball_radius(L):
    return 4.0 * L / (3.0 + np.sqrt(2.0))


def gauss_legendre(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w
