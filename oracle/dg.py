"""DG weak form of the collision term (Sections 3.2 and 3.3.1), FP64.

* Nodal basis: Lagrange polynomials on the P+1 Gauss-Legendre nodes of the
  reference element [-1, 1] (1-D), tensor products on quadrilaterals (2-D).
* Triple-product tensor H_{m l1 l2} = int phi_m phi_l1 phi_l2 dx (the
  collision tensor of the weak form), integrated exactly by a Gauss rule of
  sufficient degree.  The element Jacobian is a caller-side factor.
* Collision term of mode m: sum_{l1,l2} H_{m l1 l2} Q(F_l1, F_l2) (the double
  sum of the weak form).  The oracle evaluates it literally, with the
  symmetric bilinear form obtained from the quadratic Q(f,f) by polarisation,
  Q_s(f, g) = (Q(f+g, f+g) - Q(f,f) - Q(g,g)) / 2; H is symmetric in (l1, l2),
  so only the symmetric part of the bilinear form contributes.
* Low-rank factorisation per m (the paper's SVD of the K x K matrix H_m):
  for symmetric H_m the SVD's U and V columns coincide up to sign, so the
  eigen-decomposition H_m = sum_r lam_r u_r u_r^T is used, giving
  sum_r lam_r Q(u_r . F, u_r . F).  Stacked over m this is
  C = W Q(T F) with T = [u_{m,r}^T] (R x K) and W[m, (m', r)] = lam_r [m = m'].
"""
import numpy as np

from . import spectral


def gauss_nodes(P):
    x, w = np.polynomial.legendre.leggauss(P + 1)
    return x, w


def lgl_nodes(P):
    """Legendre-Gauss-Lobatto nodes on [-1, 1]: the endpoints and the roots of P_P'."""
    if P == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(P + 1)
    c[P] = 1.0
    inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def lagrange(nodes, x):
    """phi_l(x) for every node l: [len(nodes), len(x)]."""
    x = np.atleast_1d(x)
    out = np.ones((len(nodes), len(x)))
    for l, xl in enumerate(nodes):
        for k, xk in enumerate(nodes):
            if k != l:
                out[l] *= (x - xk) / (xl - xk)
    return out


def triple_tensor_1d(P, basis="gauss"):
    nodes = gauss_nodes(P)[0] if basis == "gauss" else lgl_nodes(P)
    xq, wq = np.polynomial.legendre.leggauss(3 * P + 2)   # exact for degree 3P
    ph = lagrange(nodes, xq)
    return np.einsum("q,mq,aq,bq->mab", wq, ph, ph, ph)


def triple_tensor_2d(P, basis="gauss"):
    H1 = triple_tensor_1d(P, basis)
    K1 = P + 1
    H = np.einsum("mab,ncd->mnacbd", H1, H1).reshape(K1 * K1, K1 * K1, K1 * K1)
    return H


def eigen_factors(H, tol=1e-13):
    """T [R, K], W [K, R], ranks per m of the eigen-form factorisation."""
    K = H.shape[0]
    rows, cols, ranks = [], [], []
    for m in range(K):
        # the eigen form needs H_m symmetric in (l1, l2); a tensor that is not
        # (a mis-ordered index, say) is an error, not something to average away
        if not np.allclose(H[m], H[m].T, rtol=0.0, atol=1e-14 * np.abs(H[m]).max()):
            raise ValueError(f"triple tensor slice {m} is not symmetric in (l1, l2)")
        lam, U = np.linalg.eigh(H[m])
        keep = np.abs(lam) > tol * np.abs(lam).max()
        ranks.append(int(keep.sum()))
        for r in np.nonzero(keep)[0]:
            rows.append(U[:, r])
            c = np.zeros(K)
            c[m] = lam[r]
            cols.append(c)
    return np.array(rows), np.array(cols).T, ranks


def q_sym(f, g, P):
    return 0.5 * (spectral.collide(f + g, P) - spectral.collide(f, P) - spectral.collide(g, P))


def collision_term_direct(F, H, P):
    """C_m = sum_{l1, l2} H_{m l1 l2} Q_s(F_l1, F_l2) for F [K, N, N, N]."""
    K = F.shape[0]
    Qd = np.array([spectral.collide(F[l], P) for l in range(K)])
    C = np.zeros_like(F)
    for a in range(K):
        for b in range(K):
            qab = Qd[a] if a == b else q_sym(F[a], F[b], P)
            C += H[:, a, b][:, None, None, None] * qab[None]
    return C


def collision_term_direct_bilinear(F, H, P):
    """C_m = sum_{l1, l2} H_{m l1 l2} Q(F_l1, F_l2) with the bilinear Q(f, g)."""
    K = F.shape[0]
    C = np.zeros_like(F)
    for a in range(K):
        for b in range(K):
            C += H[:, a, b][:, None, None, None] * spectral.collide_fg(F[a], F[b], P)[None]
    return C


def svd_factors(H, tol=1e-13):
    """The paper's SVD variant: H_m = sum_r U_{l1 r} V_{r l2} (singular values in V).
    Returns T1 [R, K] (rows U[:, r]^T), T2 [R, K] (rows V[r, :]), W [K, R]."""
    K = H.shape[0]
    r1, r2, cols = [], [], []
    for m in range(K):
        U, s, Vt = np.linalg.svd(H[m])
        for r in range(K):
            if s[r] > tol * s[0]:
                r1.append(U[:, r])
                r2.append(s[r] * Vt[r])
                c = np.zeros(K)
                c[m] = 1.0
                cols.append(c)
    return np.array(r1), np.array(r2), np.array(cols).T


def collision_term_svd(F, T1, T2, W, P):
    """sum_r W[m][r] Q(T1_r . F, T2_r . F) with the bilinear Q."""
    f = np.einsum("rk,kxyz->rxyz", T1, F)
    g = np.einsum("rk,kxyz->rxyz", T2, F)
    Qr = np.array([spectral.collide_fg(a, b, P) for a, b in zip(f, g)])
    return np.einsum("kr,rxyz->kxyz", W, Qr)


def collision_term_factored(F, T, W, P):
    h = np.einsum("rk,kxyz->rxyz", T, F)
    Qh = np.array([spectral.collide(x, P) for x in h])
    return np.einsum("kr,rxyz->kxyz", W, Qh)
