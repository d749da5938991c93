"""Brute-force quadrature of the collision integral (tiny grids, few points).

Relative-velocity form of the Appendix: with c_r = rho c_hat,
  Q(c) = int_0^R rho^2 int_{S^2} int_{S^2} B(rho)
         [ f(c - rho c_hat/2 + rho sigma/2) f(c - rho c_hat/2 - rho sigma/2)
           - f(c) f(c - rho c_hat) ] dsigma dc_hat drho,
evaluated with an independent product rule for c_hat (Gauss in cos theta x
trapezoid in phi), a given full-sphere rule for sigma, and Gauss-Legendre in
rho.  f is the trigonometric interpolant of the grid values (evaluated by
direct mode summation, Nyquist mode as the cosine of the real interpolant),
periodic on [-L, L]^3.

The loss part uses no Galerkin truncation but its c_hat integral of a single
Fourier mode is the same sinc as the spectral loss weight, so it agrees with
the spectral loss to quadrature precision.  The gain part is the collision
integral of the interpolant itself, so it differs from the spectral gain by
the projection and aliasing error only.
"""
import numpy as np
from . import dft
from . import quadrature as qd


def interpolant(f, L):
    """Returns a callable x [P,3] -> f^N(x) [P] (real)."""
    N = f.shape[0]
    c = dft.fft3(f) / N ** 3
    c0 = -L + L / N            # first grid node
    k = qd.kappa(N)

    def E(xd):
        th = np.pi * np.outer(xd - c0, k) / L
        e = np.exp(1j * th)
        e[:, N // 2] = np.cos(th[:, N // 2])
        return e

    def ev(x, chunk=20000):
        out = np.empty(len(x))
        for i in range(0, len(x), chunk):
            xs = x[i:i + chunk]
            e1, e2, e3 = E(xs[:, 0]), E(xs[:, 1]), E(xs[:, 2])
            t = np.einsum("abc,pc->pab", c, e3)
            t = np.einsum("pab,pb->pa", t, e2)
            out[i:i + chunk] = np.einsum("pa,pa->p", t, e1).real
        return out
    return ev


def sphere_product_rule(n_theta, n_phi):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - x ** 2)
    d = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)), np.outer(x, np.ones(n_phi))], -1)
    ww = np.outer(w, np.full(n_phi, 2 * np.pi / n_phi))
    return d.reshape(-1, 3), ww.reshape(-1)


def collide_points(f, L, points, N_rho, sigma_pts, sigma_w, omega, b, n_theta=12, n_phi=24):
    """(gain, loss) of the collision integral at the given velocity points."""
    fN = interpolant(f, L)
    R = qd.ball_radius(L)
    rho, wr = qd.gauss_legendre(N_rho, 0.0, R)
    ch, wch = sphere_product_rule(n_theta, n_phi)
    gain = np.zeros(len(points))
    loss = np.zeros(len(points))
    for i, c in enumerate(points):
        fc = fN(c[None, :])[0]
        for rp, wp in zip(rho, wr):
            B = b * rp ** (2 * (1 - omega))
            base = c[None, :] - 0.5 * rp * ch                    # [A,3]
            xp = base[:, None, :] + 0.5 * rp * sigma_pts[None]   # [A,S,3]
            xm = base[:, None, :] - 0.5 * rp * sigma_pts[None]
            fp = fN(xp.reshape(-1, 3)).reshape(len(ch), len(sigma_w))
            fm = fN(xm.reshape(-1, 3)).reshape(len(ch), len(sigma_w))
            gain[i] += wp * rp ** 2 * B * np.sum(wch[:, None] * sigma_w[None] * fp * fm)
            fs = fN(c[None, :] - rp * ch)
            loss[i] += wp * rp ** 2 * B * fc * np.sum(wch * fs) * np.sum(sigma_w)
    return gain, loss
