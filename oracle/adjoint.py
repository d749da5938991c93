"""Vector-Jacobian products of Q(f,f) with respect to f and omega (FP64).

Not in the paper; derived from the quadrature form used in ``spectral``.
With a = R f, b = I f, R = ifft3 diag(cos x) fft3, I = ifft3 diag(sin x) fft3,
C_p = ifft3 diag(alpha_p) fft3 and Lam~ = ifft3 diag(Lambda) fft3:

  Q = sum_p C_p sum_q w_q (a a + b b) - f Lam~ f.

For the symmetric Nyquist rule cos x is even and sin x is odd in the
frequency, so with the plain (bilinear) transpose R^T = R, I^T = -I,
C_p^T = C_p and Lam~^T = Lam~.  Hence, for a cotangent g,

  J^T g = sum_{p,q} 2 w_q [ R(h_p a) - I(h_p b) ] - g Lam~ f - Lam~ (f g),
  h_p = C_p g.

omega enters through b(omega) rho_p^{4-2 omega} in both alpha_p and the p-th
part Lambda_p of the loss weights, so

  g . dQ/d omega = sum_p dlog_p [ <g, C_p A_p> - <g, f Lam~_p f> ],
  dlog_p = d ln b / d omega - 2 ln rho_p,

where A_p = sum_q w_q (a a + b b) and d ln b / d omega = ln 2 + psi(2.5 -
omega) when b follows the VHS constant (0 when b is fixed).  Defined for the
untruncated gain weights.

VSS kernels (sigma-dependent weights alpha_pq, which carry w_p w_q): with
C_pq = ifft3 diag(alpha_pq) fft3 (alpha_pq is even in the frequency, so
C_pq^T = C_pq) the gain is sum_{p,q} C_pq (a a + b b), and

  J^T g = sum_{p,q} 2 [ R(h_pq a) - I(h_pq b) ] - g Lam~ f - Lam~ (f g),
  h_pq = C_pq g;
  g . dQ/d omega = sum_p dlog_p [ sum_q <h_pq, a a + b b> - <g, f Lam~_p f> ],

omega entering only through b(omega) rho_p^{4-2 omega} again (the VSS
constant has the same d ln b / d omega as the VHS one).
"""
import numpy as np
from . import dft
from .spectral import beta, gain_terms


def vjp_f(f, g, P):
    assert P.nyquist == "symmetric"
    X = dft.fft3(f)
    out = np.zeros(f.shape, dtype=complex)
    if P.vss:
        G = dft.fft3(g)
        for p, rho in enumerate(P.kt.rho):
            for q in range(P.M):
                h = dft.ifft3(P.alpha_pq[p, q] * G)
                bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
                a = dft.ifft3(bt.real * X)
                b = dft.ifft3(bt.imag * X)
                out += 2.0 * (dft.ifft3(bt.real * dft.fft3(h * a)) - dft.ifft3(bt.imag * dft.fft3(h * b)))
        lf = dft.ifft3(P.lam * X)
        out -= g * lf + dft.ifft3(P.lam * dft.fft3(f * g))
        return out.real
    for p, rho in enumerate(P.kt.rho):
        h = dft.ifft3(P.alpha[p] * dft.fft3(g))
        for q in range(P.M):
            bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
            a = dft.ifft3(bt.real * X)
            b = dft.ifft3(bt.imag * X)
            out += 2.0 * P.sphere_w[q] * (dft.ifft3(bt.real * dft.fft3(h * a))
                                          - dft.ifft3(bt.imag * dft.fft3(h * b)))
    lf = dft.ifft3(P.lam * X)
    out -= g * lf + dft.ifft3(P.lam * dft.fft3(f * g))
    return out.real


def vjp_omega(f, g, P, prefactor_follows_omega=True):
    if P.rank != P.N_rho:
        raise ValueError("omega gradient is defined for untruncated gain weights")
    dl = P.kt.dlog_c(prefactor_follows_omega)
    X = dft.fft3(f)
    tot = 0.0
    if P.vss:
        G = dft.fft3(g)
        for p, rho in enumerate(P.kt.rho):
            gain_p = 0.0
            for q in range(P.M):
                h = dft.ifft3(P.alpha_pq[p, q] * G).real
                bt = beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
                a = dft.ifft3(bt.real * X)
                b = dft.ifft3(bt.imag * X)
                gain_p += np.sum(h * (a * a + b * b).real)
            loss_p = np.sum(g * f * dft.ifft3(P.kt.lam_p[p] * X).real)
            tot += dl[p] * (gain_p - loss_p)
        return tot
    A = gain_terms(f, P)
    for p in range(P.N_rho):
        gain_p = np.sum(g * dft.ifft3(P.alpha[p] * dft.fft3(A[p])).real)
        loss_p = np.sum(g * f * dft.ifft3(P.kt.lam_p[p] * X).real)
        tot += dl[p] * (gain_p - loss_p)
    return tot
