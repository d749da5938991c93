"""VHS collision kernel and the kernel modes of the fast spectral method.

* Kernel (Section 2, generalised VSS form, and its non-dimensional constant):
  B = b * |g|^{2(1-omega)} (1 + cos chi)^{alpha-1};  here alpha = 1 (VHS), so
  B depends on |g| only.  The non-dimensional constant is
  b = alpha / (2^{2-omega+alpha} Gamma(2.5-omega) pi), i.e. for alpha = 1
  b(omega) = 1 / (2^{3-omega} Gamma(2.5-omega) pi).  The BKW case
  (Section 4.3) fixes B = 1/(4 pi) instead.
* Kernel mode F (Appendix, definition under the real form of G):
  F(k, rho) = 2 rho^2 int_{S^2+} B(rho) cos(pi/L rho (k/2) . c_hat) dc_hat.
  For angle-independent B the half-sphere integral is 2 pi sinc(|a|) with
  a = pi rho k / (2L), giving F = 4 pi b rho^{4-2 omega} sinc(pi rho |k|/(2L)).
  ``F_numeric`` evaluates the defining integral by quadrature (the pin of the
  closed form).
* Gain weights (quadrature form of G): alpha_p(k) = 2 w_p F(k, rho_p), since
  F does not depend on sigma.
* Loss weights (the diagonal mode G(m, m) in the Galerkin projection, which
  in the quadrature form is 2 sum_{p,q} w_p w_q F(2m, rho_p) because
  cos^2 + sin^2 = 1): Lambda(m) = 2 (sum_q w_q) sum_p w_p F(2m, rho_p).
"""
import math
import numpy as np
from . import quadrature as qd


def vhs_prefactor(omega):
    return 1.0 / (2.0 ** (3.0 - omega) * math.gamma(2.5 - omega) * math.pi)


def sinc(z):
    z = np.asarray(z, dtype=float)
    out = np.ones_like(z)
    nz = z != 0
    out[nz] = np.sin(z[nz]) / z[nz]
    return out


def F_closed(kabs, rho, L, omega, b):
    return 4.0 * np.pi * b * rho ** (4.0 - 2.0 * omega) * sinc(np.pi * rho * kabs / (2.0 * L))


def F_numeric(kvec, rho, L, omega, b, n_theta=64, n_phi=128):
    """Defining half-sphere integral of F by a Gauss x trapezoid product rule."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    ct = 0.5 * (x + 1.0)            # cos(theta) in [0, 1]: upper half sphere
    wt = 0.5 * w
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - ct ** 2)
    dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                     np.outer(ct, np.ones_like(ph))], axis=-1)
    wts = np.outer(wt, np.full(n_phi, 2.0 * np.pi / n_phi))
    arg = np.pi / L * rho * 0.5 * (dirs @ np.asarray(kvec, dtype=float))
    B = b * rho ** (2.0 * (1.0 - omega))
    return 2.0 * rho ** 2 * np.sum(wts * B * np.cos(arg))


class KernelTables:
    """Radial rule plus gain and loss weights on the N^3 frequency grid."""

    def __init__(self, N, L, N_rho, sphere_w, omega, prefactor=None):
        self.N, self.L, self.N_rho, self.omega = N, float(L), N_rho, float(omega)
        self.b = vhs_prefactor(omega) if prefactor is None else float(prefactor)
        self.R = qd.ball_radius(L)
        self.rho, self.w_rho = qd.gauss_legendre(N_rho, 0.0, self.R)
        k1, k2, k3 = qd.kappa3(N)
        self.kabs = np.sqrt(k1 ** 2 + k2 ** 2 + k3 ** 2)
        sw = float(np.sum(sphere_w))
        # alpha[p] = 2 w_p F(k, rho_p); Lam = 2 (sum_q w_q) sum_p w_p F(2k, rho_p)
        self.alpha = np.stack([2.0 * wp * F_closed(self.kabs, rp, L, omega, self.b)
                               for rp, wp in zip(self.rho, self.w_rho)])
        self.lam_p = np.stack([2.0 * sw * wp * F_closed(2.0 * self.kabs, rp, L, omega, self.b)
                               for rp, wp in zip(self.rho, self.w_rho)])
        self.lam = self.lam_p.sum(axis=0)

    def dlog_c(self, prefactor_follows_omega=True):
        """d/d omega of ln(b rho_p^{4-2 omega}) for each radial node p."""
        from scipy.special import digamma
        db = (math.log(2.0) + digamma(2.5 - self.omega)) if prefactor_follows_omega else 0.0
        return db - 2.0 * np.log(self.rho)


def truncate_alpha(alpha, svd_tol=None, svd_rank=None):
    """Truncated SVD of the gain-weight table (rows p, columns frequencies).

    Keeps singular values s_i > svd_tol * s_1, or the first svd_rank of them.
    Returns (alpha_truncated, rank).
    """
    A = alpha.reshape(alpha.shape[0], -1)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    if svd_rank is not None and svd_rank > 0:
        r = int(svd_rank)
    elif svd_tol is not None and svd_tol > 0:
        r = int(np.sum(s > svd_tol * s[0]))
    else:
        return alpha.copy(), A.shape[0]
    At = (U[:, :r] * s[:r]) @ Vt[:r]
    return At.reshape(alpha.shape), r
