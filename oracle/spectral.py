"""Q(f,f) by the fast Fourier spectral method (Appendix), FP64.

Steps, in the Appendix's order and notation:

1. f on the N^3 grid is periodised on [-L, L]^3 and represented by its
   truncated Fourier series; its coefficients are the DFT X = fft3(f) / N^3
   (the grid phase of the cell-centred nodes cancels in every
   transform-multiply-inverse chain, so plain DFT indices are used).
2. The kernel mode G(l, m) is replaced by its quadrature form: Gauss-Legendre
   in c_r (nodes rho_p, weights w_p) and the half-sphere design (sigma_q, w_q):
   G(l,m) ~ 2 sum_{p,q} w_p w_q F(l+m, rho_p)
            [cos x_l cos x_m + sin x_l sin x_m],   x_l = pi/L rho_p (l/2).sigma_q.
3. The gain coefficient is then a sum over (p,q) of convolutions:
   Q+_k = sum_p alpha_p(k) sum_q w_q sum_{l+m=k} [(cos x_l X_l)(cos x_m X_m)
                                              + (sin x_l X_l)(sin x_m X_m)],
   alpha_p = 2 w_p F(., rho_p).  Each convolution is a product in physical
   space: a = ifft3(cos x . X), b = ifft3(sin x . X), and the (p,q) term is
   w_q (a a + b b).  Convolutions are circular (l + m = k mod N), as a
   transform-based evaluation on the N^3 grid gives (no de-aliasing).
4. The loss is the convolution with G(m,m): Q- = f * ifft3(Lambda * fft3(f)).
5. Q = Q+ - Q-.

Nyquist index (the self-paired DFT index N/2, frequency -N/2), where the
paper's index set is silent about the shift: ``nyquist="symmetric"``
(default) uses the shift of the real trigonometric interpolant, whose Nyquist
factor per axis is cos(pi (N/2) s_d / L); then cos x and sin x are the real
and imaginary parts of the per-axis product and Q is real.
``nyquist="literal"`` uses exp(i pi kappa s_d / L) with kappa = -N/2 as
printed; Q is then complex and its real part is returned.

Optional SVD truncation of the gain-weight table alpha_p(k) (rows p) keeps
singular values above svd_tol times the largest (or the first svd_rank).

VSS kernels (vss_alpha > 1, Section 2): F depends on sigma, so the weights
alpha_pq(k) = 2 w_p w_q F(k, rho_p, sigma_q) multiply the transform of every
(p, q) term separately: Q+_k = sum_{p,q} alpha_pq(k) fft3(a a + b b)_k.
"""
import numpy as np
from . import dft
from . import quadrature as qd
from .kernel import KernelTables, truncate_alpha


class Params:
    def __init__(self, N, L, N_rho, sphere_pts, sphere_w, omega, prefactor=None,
                 svd_tol=None, svd_rank=None, nyquist="symmetric", vss_alpha=1.0):
        self.N, self.L = int(N), float(L)
        self.sphere_pts = np.asarray(sphere_pts, dtype=float)
        self.sphere_w = np.asarray(sphere_w, dtype=float)
        self.M = len(self.sphere_w)
        self.nyquist = nyquist
        self.vss = float(vss_alpha) != 1.0
        self.kt = KernelTables(N, L, N_rho, self.sphere_w, omega, prefactor, vss_alpha, self.sphere_pts, nyquist)
        if self.vss:
            if svd_tol or (svd_rank is not None and svd_rank > 0):
                raise ValueError("no SVD truncation of the VSS weights")
            self.alpha, self.rank = None, N_rho
            self.alpha_pq = self.kt.alpha_pq
        else:
            self.alpha, self.rank = truncate_alpha(self.kt.alpha, svd_tol, svd_rank)
        self.lam = self.kt.lam

    @property
    def N_rho(self):
        return self.kt.N_rho


def shift_factors(N, L, s, nyquist="symmetric"):
    """Per-axis shift multipliers b_d(n) for the shift s (3-vector), [3, N] complex."""
    k = qd.kappa(N)
    out = np.empty((3, N), dtype=complex)
    for d in range(3):
        theta = np.pi * k * s[d] / L
        b = np.exp(1j * theta)
        if nyquist == "symmetric":
            b[N // 2] = np.cos(theta[N // 2])
        out[d] = b
    return out


def beta(N, L, s, nyquist="symmetric"):
    """beta_s(n) = prod_d b_d(n_d) on the N^3 index grid."""
    b = shift_factors(N, L, s, nyquist)
    return b[0][:, None, None] * b[1][None, :, None] * b[2][None, None, :]


def gain_terms(f, P):
    """A_p = sum_q w_q (a a + b b) for every radial node p: [N_rho, N, N, N] complex."""
    X = dft.fft3(f)
    A = np.zeros((P.N_rho,) + f.shape, dtype=complex)
    for p, rho in enumerate(P.kt.rho):
        for q in range(P.M):
            s = 0.5 * rho * P.sphere_pts[q]
            bt = beta(P.N, P.L, s, P.nyquist)
            a = dft.ifft3(bt.real * X)
            b = dft.ifft3(bt.imag * X)
            A[p] += P.sphere_w[q] * (a * a + b * b)
    return A


def gain_vss(f, P):
    """VSS gain: every (p, q) term transformed and weighted by alpha_pq."""
    X = dft.fft3(f)
    Qh = np.zeros(f.shape, dtype=complex)
    for p, rho in enumerate(P.kt.rho):
        for q in range(P.M):
            bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
            a = dft.ifft3(bt.real * X)
            b = dft.ifft3(bt.imag * X)
            Qh += P.alpha_pq[p, q] * dft.fft3(a * a + b * b)
    return dft.ifft3(Qh)


def gain(f, P, A=None):
    if P.vss:
        if A is not None:
            raise ValueError("VSS gain has no per-node accumulators")
        return gain_vss(f, P)
    if A is None:
        A = gain_terms(f, P)
    Qh = np.zeros(f.shape, dtype=complex)
    for p in range(P.N_rho):
        Qh += P.alpha[p] * dft.fft3(A[p])
    return dft.ifft3(Qh)


def loss(f, P):
    return f * dft.ifft3(P.lam * dft.fft3(f))


def collide(f, P, return_parts=False):
    """Q(f,f) for one f of shape [N, N, N] (FP64)."""
    f = np.asarray(f, dtype=float)
    gp = gain(f, P)
    lp = loss(f, P)
    Q = gp - lp
    out = Q.real            # symmetric: Q.imag is rounding only; literal: real part
    if return_parts:
        return out, gp, lp, Q.imag
    return out


def collide_batch(fb, P):
    return np.stack([collide(f, P) for f in fb])


def collide_fg(f, g, P):
    """Bilinear Q(f, g) of the Appendix (the operator the paper evaluates for
    the weak form): gain sum_{l+m=k} G(l,m) f^_l g^_m with the quadrature form
    of G, i.e. per (p, q) the product a_f a_g + b_f b_g of the cos- and
    sin-weighted inverse transforms of f and g; loss f * ifft3(Lambda * fft3 g).
    VSS kernels weight every (p, q) product by its own alpha_pq after its
    transform, as in gain_vss."""
    f = np.asarray(f, dtype=float)
    g = np.asarray(g, dtype=float)
    Xf = dft.fft3(f)
    Xg = dft.fft3(g)
    if P.vss:
        Qh = np.zeros(f.shape, dtype=complex)
        for p, rho in enumerate(P.kt.rho):
            for q in range(P.M):
                bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
                af = dft.ifft3(bt.real * Xf)
                bf = dft.ifft3(bt.imag * Xf)
                ag = dft.ifft3(bt.real * Xg)
                bg = dft.ifft3(bt.imag * Xg)
                Qh += P.alpha_pq[p, q] * dft.fft3(af * ag + bf * bg)
        return (dft.ifft3(Qh) - f * dft.ifft3(P.lam * Xg)).real
    A = np.zeros((P.N_rho,) + f.shape, dtype=complex)
    for p, rho in enumerate(P.kt.rho):
        for q in range(P.M):
            bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
            af = dft.ifft3(bt.real * Xf)
            bf = dft.ifft3(bt.imag * Xf)
            ag = dft.ifft3(bt.real * Xg)
            bg = dft.ifft3(bt.imag * Xg)
            A[p] += P.sphere_w[q] * (af * ag + bf * bg)
    gp = gain(f, P, A=A)
    lp = f * dft.ifft3(P.lam * Xg)
    return (gp - lp).real
