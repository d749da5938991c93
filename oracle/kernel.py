"""VHS collision kernel and the kernel modes of the fast spectral method.

* Kernel (Section 2, generalised VSS form, and its non-dimensional constant):
  B = b * |g|^{2(1-omega)} (1 + cos chi)^{alpha-1}; for alpha = 1 (VHS) B
  depends on |g| only (VSS, alpha > 1, below).  The non-dimensional constant is
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

VSS kernels (Section 2, alpha in (1, 2]):
* B depends on the deflection angle through (1 + cos chi)^{alpha-1} with
  cos chi = sigma . c_hat_r.  The half-sphere form of G uses the kernel
  symmetrised in cos chi, B_sym = b |g|^{2(1-omega)} A(sigma . c_hat) with
  A(t) = ((1+t)^{alpha-1} + (1-t)^{alpha-1}) / 2 (the Appendix's B_sym).
* F then depends on sigma: F(k, rho, sigma) = 2 rho^2 int_{S^2+} B_sym
  cos(pi/L rho (k/2).c_hat) dc_hat.  The integrand is even in c_hat, so the
  half-sphere integral is half the full one; with the polar axis along sigma
  (t = sigma.c_hat) the azimuthal integral is 2 pi cos(a mu t) J0(a nu
  sqrt(1-t^2)), a = pi rho |k| / (2L), mu = k_hat.sigma, nu = sqrt(1-mu^2), and
  the part of A odd in t drops out.  So
  F = 2 pi b rho^{4-2 omega} int_{-1}^{1} (1-t)^{alpha-1} cos(a mu t)
      J0(a nu sqrt(1-t^2)) dt,
  integrated by Gauss-Jacobi with weight (1-t)^{alpha-1} (``F_vss``);
  ``F_vss_sphere`` evaluates the defining half-sphere integral directly by
  product rules (the pins of the reduction).
* Gain and loss weights keep the quadrature form with the sigma dependence:
  alpha_pq(k) = 2 w_p w_q F(k, rho_p, sigma_q) and
  Lambda(m) = 2 sum_{p,q} w_p w_q F(2m, rho_p, sigma_q).
* Nyquist index: F now depends on the signs of the components of k, not
  only on |k|.  Under the symmetric convention (the one that makes the
  shift factor of the self-paired index the cosine, i.e. the average of the
  factors at +N/2 and -N/2) every multiplier acts on that index as the
  average of its values at the two frequencies the index stands for, per
  axis; so F at an index with Nyquist components is averaged over their
  signs.  The weights are then even under index reflection, the gain and
  loss spectra are Hermitian and Q is real.  The literal convention keeps
  k = -N/2.
* Non-dimensional constant (Section 2): b = alpha / (2^{2-omega+alpha}
  Gamma(2.5-omega) pi).
"""
import math
import numpy as np
from . import quadrature as qd


def vhs_prefactor(omega):
    return 1.0 / (2.0 ** (3.0 - omega) * math.gamma(2.5 - omega) * math.pi)


def vss_prefactor(omega, alpha):
    return alpha / (2.0 ** (2.0 - omega + alpha) * math.gamma(2.5 - omega) * math.pi)


def vss_angular(t, alpha):
    """A(t) = ((1+t)^{alpha-1} + (1-t)^{alpha-1}) / 2."""
    t = np.asarray(t, dtype=float)
    return 0.5 * ((1.0 + t) ** (alpha - 1.0) + (1.0 - t) ** (alpha - 1.0))


def F_vss(kvecs, rho, sigma, L, omega, alpha, b, n_t=None):
    """F(k, rho, sigma) for VSS at every frequency vector of kvecs [..., 3]."""
    from scipy.special import j0, roots_jacobi
    kv = np.asarray(kvecs, dtype=float)
    kabs = np.sqrt(np.sum(kv ** 2, axis=-1))
    a = np.pi * rho * kabs / (2.0 * L)
    safe = np.where(kabs > 0, kabs, 1.0)
    mu = np.where(kabs > 0, (kv @ np.asarray(sigma, dtype=float)) / safe, 1.0)
    mu = np.clip(mu, -1.0, 1.0)
    nu = np.sqrt(1.0 - mu ** 2)
    if n_t is None:
        n_t = int(1.25 * float(np.max(a))) + 48
    t, wt = roots_jacobi(n_t, alpha - 1.0, 0.0)
    s = np.sqrt(1.0 - t ** 2)
    a_ = a[..., None]
    integ = np.cos(a_ * mu[..., None] * t) * j0(a_ * nu[..., None] * s)
    return 2.0 * np.pi * b * rho ** (4.0 - 2.0 * omega) * (integ @ wt)


def F_vss_sphere(kvec, rho, sigma, L, omega, alpha, b, axis="sigma", n_theta=192, n_phi=384):
    """Defining half-sphere integral of F for VSS by a Gauss x trapezoid product
    rule (the pins of the reduction in ``F_vss``).

    axis="z": the half sphere z >= 0 literally (Gauss in cos theta); the
    angular kernel has derivative singularities at +-sigma, so this converges
    slowly.  axis="sigma": the full sphere with the polar angle theta measured
    from sigma (Gauss in theta, where the singularity sits at the poles), halved
    because the integrand is even in c_hat."""
    sigma = np.asarray(sigma, dtype=float)
    kvec = np.asarray(kvec, dtype=float)
    B0 = b * rho ** (2.0 * (1.0 - omega))
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    x, w = np.polynomial.legendre.leggauss(n_theta)
    if axis == "z":
        ct = 0.5 * (x + 1.0)
        wt = 0.5 * w
        st = np.sqrt(1.0 - ct ** 2)
        dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                         np.outer(ct, np.ones_like(ph))], axis=-1)
        wts = np.outer(wt, np.full(n_phi, 2.0 * np.pi / n_phi))
        half = 1.0
    else:
        e1 = np.cross(sigma, [1.0, 0.0, 0.0]) if abs(sigma[0]) < 0.9 else np.cross(sigma, [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(sigma, e1)
        th = 0.5 * np.pi * (x + 1.0)
        wth = 0.5 * np.pi * w * np.sin(th)
        dirs = (np.cos(th)[:, None, None] * sigma
                + np.sin(th)[:, None, None] * (np.cos(ph)[None, :, None] * e1 + np.sin(ph)[None, :, None] * e2))
        wts = np.outer(wth, np.full(n_phi, 2.0 * np.pi / n_phi))
        half = 0.5
    arg = np.pi / L * rho * 0.5 * (dirs @ kvec)
    Bs = B0 * vss_angular(dirs @ sigma, alpha)
    return 2.0 * rho ** 2 * half * np.sum(wts * Bs * np.cos(arg))


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
    """Radial rule plus gain and loss weights on the N^3 frequency grid.

    VHS (vss_alpha = 1): alpha[p] = 2 w_p F(k, rho_p).  VSS (vss_alpha > 1):
    alpha_pq[p, q] = 2 w_p w_q F(k, rho_p, sigma_q) (then ``alpha`` is None)."""

    def __init__(self, N, L, N_rho, sphere_w, omega, prefactor=None, vss_alpha=1.0, sphere_pts=None,
                 nyquist="symmetric"):
        self.N, self.L, self.N_rho, self.omega = N, float(L), N_rho, float(omega)
        self.vss_alpha = float(vss_alpha)
        self.R = qd.ball_radius(L)
        self.rho, self.w_rho = qd.gauss_legendre(N_rho, 0.0, self.R)
        k1, k2, k3 = qd.kappa3(N)
        self.kabs = np.sqrt(k1 ** 2 + k2 ** 2 + k3 ** 2)
        sw = float(np.sum(sphere_w))
        if self.vss_alpha != 1.0:
            self.b = vss_prefactor(omega, self.vss_alpha) if prefactor is None else float(prefactor)
            kv = np.stack([k1, k2, k3], axis=-1)
            M = len(sphere_w)
            nyq = np.abs(kv) == N // 2                 # Nyquist components (k = -N/2)
            sym = np.any(nyq, axis=-1) if nyquist == "symmetric" else np.zeros(kv.shape[:-1], bool)
            ksub = kv[sym]
            nsub = nyq[sym]
            # the 8 sign patterns, applied to the Nyquist components only
            flips = [np.where(nsub, 1.0 - 2.0 * np.array(sg, dtype=float), 1.0) for sg in np.ndindex(2, 2, 2)]

            def F_sym(kvecs, sub, rp, sq):
                # F everywhere, then the sign average of the Nyquist components on the subset
                F = F_vss(kvecs, rp, sq, L, omega, self.vss_alpha, self.b)
                if sub.size:
                    F[sym] = np.mean([F_vss(sub * fl, rp, sq, L, omega, self.vss_alpha, self.b)
                                      for fl in flips], axis=0)
                return F

            self.alpha = None
            self.alpha_pq = np.zeros((N_rho, M) + self.kabs.shape)
            self.lam_p = np.zeros((N_rho,) + self.kabs.shape)
            for p, (rp, wp) in enumerate(zip(self.rho, self.w_rho)):
                for q in range(M):
                    sq = sphere_pts[q]
                    self.alpha_pq[p, q] = 2.0 * wp * sphere_w[q] * F_sym(kv, ksub, rp, sq)
                    self.lam_p[p] += 2.0 * wp * sphere_w[q] * F_sym(2.0 * kv, 2.0 * ksub, rp, sq)
            self.lam = self.lam_p.sum(axis=0)
            return
        self.b = vhs_prefactor(omega) if prefactor is None else float(prefactor)
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
