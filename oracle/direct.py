"""The same discrete operator as an explicit O(N^6) double sum (tiny N only).

Galerkin projection of the Appendix, with the quadrature form of G and the
circular index set of a transform-based evaluation:

  Qhat_k = sum_{l + m = k (mod N)} [ G(l, m) - G(m, m) ] c_l c_m ,
  G(l, m) = sum_p alpha_p(k) sum_q w_q [cos x_l cos x_m + sin x_l sin x_m],
  G(m, m) = Lambda(m),

where c = fft3(f)/N^3 are the DFT coefficients and cos x, sin x are the real
and imaginary parts of the shift factor beta_s (see ``spectral``), so that
cos x_l cos x_m + sin x_l sin x_m = Re(beta(l) conj(beta(m))).  Then
Q_j = sum_k Qhat_k exp(2 pi i k.j / N).

Nothing here reuses the transform route of ``spectral`` beyond the forward
DFT of f: the k-sum is a scatter over explicit index pairs.  For VSS kernels
the weight alpha_pq(k) of each (p, q) multiplies its own scatter.
"""
import numpy as np
from . import dft
from .spectral import beta


def collide_direct(f, P, g=None):
    """Q(f, f), or the bilinear Q(f, g) when g is given (l indexes f, m indexes g)."""
    N = P.N
    n3 = N ** 3
    c = (dft.fft3(f) / n3).reshape(-1)
    cg = c if g is None else (dft.fft3(g) / n3).reshape(-1)
    idx = np.indices((N, N, N)).reshape(3, -1)
    # k index of every (l, m) pair
    kk = ((idx[:, :, None] + idx[:, None, :]) % N)
    kflat = (kk[0] * N + kk[1]) * N + kk[2]
    cc = np.outer(c, cg)
    Qh = np.zeros(n3, dtype=complex)
    def scatter(t):
        return (np.bincount(kflat.ravel(), weights=t.real.ravel(), minlength=n3)
                + 1j * np.bincount(kflat.ravel(), weights=t.imag.ravel(), minlength=n3))

    if P.vss:
        # sigma-dependent weights: one scatter per (p, q)
        for p, rho in enumerate(P.kt.rho):
            for q in range(P.M):
                bt = beta(N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist).reshape(-1)
                Qh += P.alpha_pq[p, q].reshape(-1) * scatter(np.real(np.outer(bt, np.conj(bt))) * cc)
    else:
        alpha = P.alpha.reshape(P.N_rho, -1)
        for p, rho in enumerate(P.kt.rho):
            S = np.zeros((n3, n3))
            for q in range(P.M):
                bt = beta(N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist).reshape(-1)
                S += P.sphere_w[q] * np.real(np.outer(bt, np.conj(bt)))
            Qh += alpha[p] * scatter(S * cc)
    lam = P.lam.reshape(-1)
    Qh -= scatter(cc * lam[None, :])
    Q = dft.ifft3(Qh.reshape(N, N, N)) * n3
    return Q.real
