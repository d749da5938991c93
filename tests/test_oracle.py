"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins; none re-types the oracle's own formula.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, bkw, brute, conserve, dft, direct, kernel, spectral
from oracle import quadrature as qd

HERE = os.path.dirname(os.path.abspath(__file__))


def params(N, L, N_rho, M=6, omega=0.81, **kw):
    pts, w = W.sphere_rule(M)
    return spectral.Params(N, L, N_rho, pts, w, omega, **kw)


# ---------------------------------------------------------------- transforms
def test_dft_matches_library_fft():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 6, 6, 6)) + 1j * rng.normal(size=(2, 6, 6, 6))
    assert np.allclose(dft.fft3(x), np.fft.fftn(x, axes=(-3, -2, -1)), atol=1e-12, rtol=0)
    assert np.allclose(dft.ifft3(dft.fft3(x)), x, atol=1e-14, rtol=0)


def test_dft_parseval():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(8, 8, 8))
    X = dft.fft3(x)
    assert abs(np.sum(np.abs(X) ** 2) / 8 ** 3 - np.sum(x ** 2)) < 1e-10 * np.sum(x ** 2)


# ---------------------------------------------------------------- quadratures
@pytest.mark.parametrize("n", [1, 4, 8, 16])
def test_gauss_legendre_exact_degree(n):
    R = qd.ball_radius(6.0)
    x, w = qd.gauss_legendre(n, 0.0, R)
    for d in range(2 * n):
        assert abs(np.sum(w * x ** d) - R ** (d + 1) / (d + 1)) < 1e-12 * R ** (d + 1)


def test_ball_radius():
    # R = 4L/(3+sqrt 2) of the Appendix's truncation criterion: L = 6 -> 5.43698
    assert abs(qd.ball_radius(6.0) - 5.43698) < 1e-5


def _sphere_monomial(a, b, c):
    """Exact integral of x^a y^b z^c over the unit sphere."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    return 2 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)


@pytest.mark.parametrize("M,deg", [(6, 5), (12, 5), (16, 7)])
def test_half_sphere_design_degree(M, deg):
    pts, w = W.sphere_rule(M)
    assert pts.shape == (M, 3)
    assert abs(w.sum() - 2 * math.pi) < 1e-14
    # one representative per antipodal pair
    assert np.all(pts[:, 2] >= 0)
    assert np.linalg.norm(pts[:, None] + pts[None], axis=-1).min() > 0.1
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-15)
    full = np.concatenate([pts, -pts])
    fw = np.concatenate([w, w])
    worst = 0.0
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                v = np.sum(fw * full[:, 0] ** a * full[:, 1] ** b * full[:, 2] ** c)
                worst = max(worst, abs(v - _sphere_monomial(a, b, c)))
    assert worst < 1e-12
    # and not exact one even degree higher
    d = deg + 1
    errs = [abs(np.sum(fw * full[:, 0] ** a * full[:, 1] ** (d - a)) - _sphere_monomial(a, d - a, 0))
            for a in range(d + 1)]
    assert max(errs) > 1e-6


# ---------------------------------------------------------------- kernel modes
def test_vhs_prefactor_values():
    # b = 1/(2^{3-w} Gamma(2.5-w) pi); omega = 1 gives 1/(2 pi^{3/2})
    assert abs(kernel.vhs_prefactor(1.0) - 1.0 / (2 * math.pi ** 1.5)) < 1e-16
    assert abs(kernel.vhs_prefactor(0.81) - 0.0769292741) < 1e-10
    assert abs(kernel.vhs_prefactor(0.74) - 0.0721250234) < 1e-10


@pytest.mark.parametrize("kvec,rho,omega", [((0, 0, 0), 1.3, 0.81), ((3, -2, 5), 2.1, 0.81),
                                            ((-8, 0, 1), 4.7, 1.0), ((7, 7, -7), 0.4, 0.5)])
def test_kernel_mode_closed_form_vs_integral(kvec, rho, omega):
    L, b = 6.0, kernel.vhs_prefactor(omega)
    kabs = np.sqrt(np.sum(np.square(kvec)))
    closed = kernel.F_closed(np.array(kabs), rho, L, omega, b)
    num = kernel.F_numeric(kvec, rho, L, omega, b)
    assert abs(closed - num) < 1e-13 * max(1.0, abs(closed))


def test_loss_weight_at_zero_frequency():
    # Lambda(0) = 16 pi^2 b sum_p w_p rho_p^{4-2w}; exact GL integral when 4-2w is an integer
    P = params(8, 6.0, 5, omega=1.0)
    R = qd.ball_radius(6.0)
    b = P.kt.b
    assert abs(P.lam[0, 0, 0] - 16 * math.pi ** 2 * b * R ** 3 / 3) < 1e-12 * P.lam[0, 0, 0]


# ---------------------------------------------------------------- the operator
@pytest.mark.parametrize("nyq", ["symmetric", "literal"])
def test_constant_f_has_zero_collisions(nyq):
    P = params(8, 5.0, 6, nyquist=nyq)
    f = np.full((8, 8, 8), 0.37)
    Q, gp, lp, _ = spectral.collide(f, P, return_parts=True)
    assert np.abs(Q).max() < 1e-13 * np.abs(lp).max()


@pytest.mark.parametrize("N,nyq,svd", [(4, "symmetric", None), (8, "symmetric", None),
                                       (8, "literal", None), (8, "symmetric", 1e-3),
                                       (6, "symmetric", None)])
def test_fast_equals_direct_double_sum(N, nyq, svd):
    f = W.maxwellian_mixture(1, N, 4.0, 11, noise=0.2)[0]
    P = params(N, 4.0, 4, nyquist=nyq, svd_tol=svd)
    Qs = spectral.collide(f, P)
    Qd = direct.collide_direct(f, P)
    assert np.abs(Qs - Qd).max() < 1e-13 * np.abs(Qd).max()


def _table1():
    rows = []
    for line in open(os.path.join(HERE, "golden", "bkw_table1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = line.split()
        rows.append((int(v[0]), int(v[1]), [float(x) for x in v[2:]]))
    return rows


@pytest.mark.parametrize("N,N_r,errs", [r for r in _table1() if r[0] <= 32])
def test_bkw_table1(N, N_r, errs):
    """Error of Q against the exact BKW operator matches the paper's Table 1.

    The paper's M = 6 design is the same icosahedral 5-design up to an unknown
    rotation, so agreement is to within a factor 1.5 rather than digit for digit.
    """
    L = 6.62
    P = params(N, L, N_r, M=6, omega=1.0, prefactor=1.0 / (4 * math.pi))
    for t0, ref in zip((5.5, 6.5, 10.0), errs):
        Q = spectral.collide(bkw.f_exact(N, L, t0), P)
        err = np.abs(Q - bkw.Q_exact(N, L, t0)).max()
        assert ref / 1.5 < err < ref * 1.5, (t0, err, ref)


def test_bkw_exact_operator_is_time_derivative():
    # the printed exact Q must equal d f / dt of the printed BKW solution
    N, L, t, h = 12, 6.0, 7.0, 1e-4
    dfdt = (bkw.f_exact(N, L, t + h) - bkw.f_exact(N, L, t - h)) / (2 * h)
    Q = bkw.Q_exact(N, L, t)
    assert np.abs(dfdt - Q).max() < 1e-8 * np.abs(Q).max()


def test_quadratic_scaling_and_translation():
    N, L = 8, 5.0
    f = W.maxwellian_mixture(1, N, L, 3, noise=0.3)[0]
    P = params(N, L, 4)
    Q = spectral.collide(f, P)
    assert np.abs(spectral.collide(2.5 * f, P) - 6.25 * Q).max() < 1e-13 * np.abs(Q).max() * 6.25
    # periodic translation by whole cells commutes with Q (every step is a
    # Fourier multiplier or a pointwise product)
    fr = np.roll(f, (2, -1, 3), axis=(0, 1, 2))
    assert np.abs(spectral.collide(fr, P) - np.roll(Q, (2, -1, 3), axis=(0, 1, 2))).max() < 1e-13 * np.abs(Q).max()


def test_reflection_and_axis_permutation():
    N, L = 8, 5.0
    f = W.maxwellian_mixture(1, N, L, 5, noise=0.3)[0]
    P = params(N, L, 4, M=6)
    Q = spectral.collide(f, P)
    # c -> -c maps node j to N-1-j
    Qr = spectral.collide(f[::-1, ::-1, ::-1].copy(), P)
    assert np.abs(Qr - Q[::-1, ::-1, ::-1]).max() < 1e-13 * np.abs(Q).max()
    # the icosahedral rule is invariant under the cyclic axis permutation
    fp = np.transpose(f, (1, 2, 0)).copy()
    Qp = spectral.collide(fp, P)
    assert np.abs(Qp - np.transpose(Q, (1, 2, 0))).max() < 1e-12 * np.abs(Q).max()


def test_maxwellian_is_near_equilibrium_spectrally():
    rels = []
    for N in (8, 16, 24):
        L = 6.0
        f = W.maxwellian(N, L, 1.0, np.array([0.2, -0.1, 0.3]), 1.0)
        P = params(N, L, N // 2)
        Q, gp, lp, _ = spectral.collide(f, P, return_parts=True)
        rels.append(np.abs(Q).max() / np.abs(gp).max())
    assert rels[0] > 10 * rels[1] > 100 * rels[2]
    assert rels[2] < 1e-4


def test_brute_force_quadrature_of_collision_integral():
    """Loss to quadrature precision, gain to the projection/aliasing level."""
    N, L, Nr = 12, 6.0, 8
    pts, w = W.sphere_rule(6)
    f = W.maxwellian_mixture(1, N, L, 7, T_range=(0.8, 1.2))[0]
    P = spectral.Params(N, L, Nr, pts, w, 0.81)
    Q, gp, lp, _ = spectral.collide(f, P, return_parts=True)
    c = W.velocity_grid(N, L)
    idx = [(6, 6, 6), (5, 6, 7), (3, 8, 6)]
    points = np.array([[c[i], c[j], c[k]] for i, j, k in idx])
    g, l = brute.collide_points(f, L, points, Nr, np.concatenate([pts, -pts]),
                                np.concatenate([w, w]), 0.81, P.kt.b, n_theta=20, n_phi=40)
    lref = np.array([lp.real[x] for x in idx])
    gref = np.array([gp.real[x] for x in idx])
    assert np.abs(l - lref).max() < 1e-8 * np.abs(lp).max()
    assert np.abs(g - gref).max() < 0.06 * np.abs(gp).max()


# ---------------------------------------------------------------- conservation
def test_conservation_projection():
    N, L = 8, 5.0
    f = W.maxwellian_mixture(2, N, L, 9)
    P = params(N, L, 4)
    Q = spectral.collide_batch(f, P)
    Qc, m = conserve.project(Q, N, L)
    assert np.all(conserve.conservation_residual(Qc, N, L) < 1e-13)
    Qcc, _ = conserve.project(Qc, N, L)
    assert np.abs(Qcc - Qc).max() < 1e-15 * np.abs(Qc).max() * 10
    # the correction lies in the span of the invariants and is orthogonal to Q_c
    C = conserve.invariants(N, L)
    d = (Q - Qc).reshape(2, -1)
    coef, *_ = np.linalg.lstsq(C.T, d.T, rcond=None)
    assert np.abs(C.T @ coef - d.T).max() < 1e-14 * np.abs(Q).max()
    assert np.abs(np.sum(d * Qc.reshape(2, -1), axis=1)).max() < 1e-13 * np.sum(Q ** 2)
    # m holds the pre-projection invariant sums
    assert np.allclose(m, (Q.reshape(2, -1) @ C.T), rtol=0, atol=1e-13 * np.abs(Q).sum())


def test_moments_of_maxwellian():
    N, L = 24, 6.0
    u = np.array([0.3, -0.2, 0.1])
    f = W.maxwellian(N, L, 1.3, u, 0.9)
    mo = conserve.moments(f, N, L)
    assert abs(mo[0] - 1.3) < 1e-10
    assert np.allclose(mo[1:4], u, atol=1e-10)
    assert abs(mo[4] - 0.9) < 1e-10
    # P = n T I (rescaled stress), q = 0
    assert np.allclose(mo[5:11], [1.3 * 0.9, 0, 0, 1.3 * 0.9, 0, 1.3 * 0.9], atol=1e-9)
    assert np.allclose(mo[11:], 0, atol=1e-10)


def test_moments_of_two_maxwellian_mixture_closed_form():
    """Moments of a sum of two drifting Maxwellians n_i (pi T_i)^{-3/2}
    exp(-|c - u_i|^2 / T_i), whose values follow in closed form from the
    Gaussian moments (per unit density, v = c - u_i has covariance T_i/2 I):
      n = n1 + n2, u = (n1 u1 + n2 u2) / n, d_i = u_i - u,
      T = 2/(3n) sum_i n_i (3 T_i / 2 + |d_i|^2),
      P = sum_i n_i (T_i I + 2 d_i d_i^T)          (P = 2 int f (c-u)(c-u)^T),
      q = sum_i n_i d_i (5 T_i / 2 + |d_i|^2)       (q = int f (c-u)|c-u|^2).
    The drifts are not along the axes, so P has off-diagonal parts and q is
    non-zero: a wrong factor in either (a dropped 2, a halved q) fails.  The
    midpoint rule on this grid is accurate to far below the tolerance (spacing
    1/4 against widths T_i >= 1; tails beyond |c| = 8 below 1e-14)."""
    N, L = 64, 8.0
    n = np.array([0.7, 1.2])
    T = np.array([1.0, 1.5])
    us = np.array([[0.6, -0.4, 0.3], [-0.2, 0.5, -0.45]])
    f = sum(W.maxwellian(N, L, n[i], us[i], T[i]) for i in range(2))
    mo = conserve.moments(f, N, L)
    nt = n.sum()
    u = (n[:, None] * us).sum(axis=0) / nt
    d = us - u
    d2 = (d ** 2).sum(axis=1)
    Tt = 2.0 / (3.0 * nt) * np.sum(n * (1.5 * T + d2))
    Pt = sum(n[i] * (T[i] * np.eye(3) + 2.0 * np.outer(d[i], d[i])) for i in range(2))
    qt = sum(n[i] * d[i] * (2.5 * T[i] + d2[i]) for i in range(2))
    exp = np.array([nt, *u, Tt, Pt[0, 0], Pt[0, 1], Pt[0, 2], Pt[1, 1], Pt[1, 2], Pt[2, 2], *qt])
    assert abs(Pt[0, 1]) > 0.05 and np.abs(qt).min() > 0.05   # the pin is not degenerate
    assert np.abs(mo - exp).max() < 1e-12


# ---------------------------------------------------------------- adjoint
def test_vjp_f_matches_central_difference():
    N, L = 8, 5.0
    f = W.maxwellian_mixture(1, N, L, 13, noise=0.3)[0]
    g = W.cotangent(f, 14)
    v = W.cotangent(f, 15)
    P = params(N, L, 4)
    jtg = adjoint.vjp_f(f, g, P)
    h = 1e-3
    # Q is quadratic, so the central difference is exact up to rounding
    jv = (spectral.collide(f + h * v, P) - spectral.collide(f - h * v, P)) / (2 * h)
    lhs, rhs = np.sum(g * jv), np.sum(jtg * v)
    assert abs(lhs - rhs) < 1e-11 * (np.abs(g * jv).sum())


def test_vjp_omega_matches_central_difference():
    N, L, om = 8, 5.0, 0.81
    f = W.maxwellian_mixture(1, N, L, 16)[0]
    g = W.cotangent(f, 17)
    pts, w = W.sphere_rule(6)
    P = spectral.Params(N, L, 4, pts, w, om)
    d = adjoint.vjp_omega(f, g, P)
    h = 1e-6
    Qp = spectral.collide(f, spectral.Params(N, L, 4, pts, w, om + h))
    Qm = spectral.collide(f, spectral.Params(N, L, 4, pts, w, om - h))
    fd = np.sum(g * (Qp - Qm)) / (2 * h)
    assert abs(fd - d) < 1e-7 * max(abs(d), 1e-30) + 1e-12
    # fixed prefactor: only the exponent contributes
    b = kernel.vhs_prefactor(om)
    P = spectral.Params(N, L, 4, pts, w, om, prefactor=b)
    d2 = adjoint.vjp_omega(f, g, P, prefactor_follows_omega=False)
    Qp = spectral.collide(f, spectral.Params(N, L, 4, pts, w, om + h, prefactor=b))
    Qm = spectral.collide(f, spectral.Params(N, L, 4, pts, w, om - h, prefactor=b))
    fd2 = np.sum(g * (Qp - Qm)) / (2 * h)
    assert abs(fd2 - d2) < 1e-7 * abs(d2)


@pytest.mark.parametrize("alpha", [1.5, 2.0])
def test_vss_vjp_matches_central_differences(alpha):
    """VSS VJP in f: dot-product test against a central difference of Q (exact
    up to rounding, Q being quadratic); in omega: central difference h = 1e-6;
    at alpha = 2 both equal the VHS route's."""
    N, L, om = 6, 4.0, 0.81
    pts, w = W.sphere_rule(6)
    P = spectral.Params(N, L, 3, pts, w, om, vss_alpha=alpha)
    f = W.maxwellian_mixture(1, N, L, 51, noise=0.3)[0]
    g = W.cotangent(f, 52)
    v = W.cotangent(f, 53)
    jtg = adjoint.vjp_f(f, g, P)
    hf = 1e-3
    jv = (spectral.collide(f + hf * v, P) - spectral.collide(f - hf * v, P)) / (2 * hf)
    assert abs(np.sum(g * jv) - np.sum(jtg * v)) < 1e-11 * np.abs(g * jv).sum()
    d = adjoint.vjp_omega(f, g, P)
    h = 1e-6
    Qp = spectral.collide(f, spectral.Params(N, L, 3, pts, w, om + h, vss_alpha=alpha))
    Qm = spectral.collide(f, spectral.Params(N, L, 3, pts, w, om - h, vss_alpha=alpha))
    fd = np.sum(g * (Qp - Qm)) / (2 * h)
    assert abs(fd - d) < 1e-7 * np.abs(g * (Qp - Qm) / (2 * h)).sum()
    if alpha == 2.0:
        Pv = spectral.Params(N, L, 3, pts, w, om)
        assert np.abs(jtg - adjoint.vjp_f(f, g, Pv)).max() < 1e-12 * np.abs(jtg).max()
        assert abs(d - adjoint.vjp_omega(f, g, Pv)) < 1e-12 * abs(d)


def test_digamma_constant():
    # d ln b / d omega at omega = 0.81 is ln 2 + psi(1.69)
    P = params(8, 5.0, 3, omega=0.81)
    dl = P.kt.dlog_c(True) + 2 * np.log(P.kt.rho)
    assert np.allclose(dl, 0.893732, atol=1e-6)


# ---------------------------------------------------------------- DG weak form
def test_dg_triple_tensor_properties():
    from oracle import dg
    for P in (1, 2, 3):
        H = dg.triple_tensor_1d(P)
        K = P + 1
        assert H.shape == (K, K, K)
        # symmetric in all index pairs and sum_m H_{m a b} = mass matrix (partition of unity)
        assert np.allclose(H, H.transpose(0, 2, 1)) and np.allclose(H, H.transpose(1, 0, 2))
        nodes, w = dg.gauss_nodes(P)
        assert np.allclose(H.sum(axis=0), np.diag(w), atol=1e-14)   # Gauss-node Lagrange basis: M = diag(w)
    H2 = dg.triple_tensor_2d(1)
    assert H2.shape == (4, 4, 4)
    assert abs(H2.sum() - 4.0) < 1e-13   # integral of 1 over [-1,1]^2


@pytest.mark.parametrize("P", [1, 2])
def test_dg_triple_tensor_2d_against_direct_quadrature(P):
    """The 2-D tensor of the quadrilateral basis phi_(i,j)(x, y) = phi_i(x) phi_j(y),
    ordered as (i, j) -> i (P+1) + j, pinned three ways: every entry against a
    direct 2-D Gauss product rule of the three 2-D basis functions evaluated as
    functions of (x, y); symmetry in (l1, l2) and in (m, l1); and sum_m H =
    the mass matrix, diag(w_i w_j) on the Gauss-node basis (partition of unity).
    A permuted Kronecker index order passes the total-sum check but none of these."""
    from oracle import dg
    H = dg.triple_tensor_2d(P)
    K1 = P + 1
    nodes, w = dg.gauss_nodes(P)
    xq, wq = np.polynomial.legendre.leggauss(2 * P + 3)
    X, Y = np.meshgrid(xq, xq, indexing="ij")
    WW = np.outer(wq, wq)

    def phi2(i, j):
        return dg.lagrange(nodes, X.ravel())[i].reshape(X.shape) * dg.lagrange(nodes, Y.ravel())[j].reshape(Y.shape)

    basis = [phi2(i, j) for i in range(K1) for j in range(K1)]
    ref = np.array([[[np.sum(WW * bm * ba * bb) for bb in basis] for ba in basis] for bm in basis])
    assert np.abs(H - ref).max() < 1e-14
    assert np.allclose(H, H.transpose(0, 2, 1), rtol=0, atol=1e-15)
    assert np.allclose(H, H.transpose(1, 0, 2), rtol=0, atol=1e-15)
    assert np.allclose(H.sum(axis=0), np.diag(np.outer(w, w).ravel()), rtol=0, atol=1e-14)
    # the eigen factorisation refuses a tensor that is not symmetric in (l1, l2)
    bad = H.copy()
    bad[0, 0, 1] += 1e-3
    with pytest.raises(ValueError):
        dg.eigen_factors(bad)


def test_dg_eigen_form_equals_direct_double_sum():
    """The low-rank (eigen) form of the paper's SVD variant reproduces the
    direct double sum of the weak form exactly."""
    from oracle import dg
    N, L = 8, 5.0
    P = params(N, L, 4)
    for deg in (1, 2):
        H = dg.triple_tensor_1d(deg)
        K = deg + 1
        F = W.maxwellian_mixture(K, N, L, 500 + deg, noise=0.2)
        T, Wm, ranks = dg.eigen_factors(H)
        assert sum(ranks) <= K * K
        Cd = dg.collision_term_direct(F, H, P)
        Cf = dg.collision_term_factored(F, T, Wm, P)
        assert np.abs(Cd - Cf).max() < 1e-13 * np.abs(Cd).max()


def test_dg_collocation_is_q_at_quadrature_points():
    """With the K-point Gauss rule as quadrature, H_m collapses to w_m e_m e_m^T and
    the collision term is w_m Q(F_m) (the quadrature-point form)."""
    from oracle import dg
    N, L = 8, 5.0
    P = params(N, L, 4)
    nodes, w = dg.gauss_nodes(2)
    ph = dg.lagrange(nodes, nodes)
    Hq = np.einsum("q,mq,aq,bq->mab", w, ph, ph, ph)
    F = W.maxwellian_mixture(3, N, L, 600, noise=0.2)
    C = dg.collision_term_direct(F, Hq, P)
    ref = np.array([w[m] * spectral.collide(F[m], P) for m in range(3)])
    assert np.abs(C - ref).max() < 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------- bilinear Q(f, g)
def test_bilinear_reduces_to_quadratic_and_matches_direct():
    N, L = 8, 4.0
    P = params(N, L, 4)
    f = W.maxwellian_mixture(1, N, L, 31, noise=0.2)[0]
    g = W.maxwellian_mixture(1, N, L, 32, noise=0.2)[0]
    Qff = spectral.collide(f, P)
    assert np.abs(spectral.collide_fg(f, f, P) - Qff).max() < 1e-14 * np.abs(Qff).max()
    Qfg = spectral.collide_fg(f, g, P)
    Qd = direct.collide_direct(f, P, g=g)
    assert np.abs(Qfg - Qd).max() < 1e-13 * np.abs(Qd).max()
    # symmetric part = polarisation of the quadratic form
    from oracle import dg
    Qs = 0.5 * (Qfg + spectral.collide_fg(g, f, P))
    assert np.abs(Qs - dg.q_sym(f, g, P)).max() < 1e-13 * np.abs(Qs).max()
    # bilinear in each argument
    assert np.abs(spectral.collide_fg(2 * f, 3 * g, P) - 6 * Qfg).max() < 1e-13 * 6 * np.abs(Qfg).max()


@pytest.mark.parametrize("alpha", [1.5, 2.0])
def test_vss_bilinear_reduces_to_quadratic_and_matches_direct(alpha):
    """VSS bilinear Q(f, g): equals Q(f, f) at g = f, the O(N^6) double sum with
    the sigma-dependent weights and two spectra, and its symmetric part is the
    polarisation of the quadratic form; at alpha = 2 it equals the VHS route."""
    N, L = 6, 4.0
    pts, w = W.sphere_rule(6)
    P = spectral.Params(N, L, 3, pts, w, 0.81, vss_alpha=alpha)
    f = W.maxwellian_mixture(1, N, L, 41, noise=0.2)[0]
    g = W.maxwellian_mixture(1, N, L, 42, noise=0.2)[0]
    Qff = spectral.collide(f, P)
    assert np.abs(spectral.collide_fg(f, f, P) - Qff).max() < 1e-14 * np.abs(Qff).max()
    Qfg = spectral.collide_fg(f, g, P)
    Qd = direct.collide_direct(f, P, g=g)
    assert np.abs(Qfg - Qd).max() < 1e-13 * np.abs(Qd).max()
    from oracle import dg
    Qs = 0.5 * (Qfg + spectral.collide_fg(g, f, P))
    assert np.abs(Qs - dg.q_sym(f, g, P)).max() < 1e-13 * np.abs(Qs).max()
    if alpha == 2.0:
        Pv = spectral.Params(N, L, 3, pts, w, 0.81, prefactor=P.kt.b)
        Qv = spectral.collide_fg(f, g, Pv)
        assert np.abs(Qfg - Qv).max() < 1e-13 * np.abs(Qv).max()


def test_dg_paper_svd_form_equals_double_sum():
    """The paper's SVD variant sum_r Q(f_r, g_r) with f_r = U F, g_r = V F (general
    U, V from the SVD of each H_m) reproduces sum H_{m l1 l2} Q(F_l1, F_l2)."""
    from oracle import dg
    N, L = 8, 4.0
    P = params(N, L, 4)
    H = dg.triple_tensor_1d(2)
    F = W.maxwellian_mixture(3, N, L, 33, noise=0.2)
    T1, T2, Wm = dg.svd_factors(H)
    Cd = dg.collision_term_direct_bilinear(F, H, P)
    Cs = dg.collision_term_svd(F, T1, T2, Wm, P)
    assert np.abs(Cd - Cs).max() < 1e-13 * np.abs(Cd).max()
    # and the symmetric H makes it equal to the quadratic double sum too
    Cq = dg.collision_term_direct(F, H, P)
    assert np.abs(Cd - Cq).max() < 1e-13 * np.abs(Cd).max()


def test_dg_lgl_basis_ranks():
    """On Lagrange bases at Gauss-Lobatto nodes the slices H_m have full rank K
    (no saving from the SVD), on Gauss nodes rank K - 1 for P = 2: the rank
    depends on the basis, as the paper notes."""
    from oracle import dg
    H = dg.triple_tensor_1d(2, "lgl")
    assert np.allclose(H, H.transpose(0, 2, 1))
    _, _, r_lgl = dg.eigen_factors(H)
    _, _, r_g = dg.eigen_factors(dg.triple_tensor_1d(2, "gauss"))
    assert r_lgl == [3, 3, 3]
    assert r_g == [2, 2, 2]
    # partition of unity: sum_m H_{m a b} = mass matrix int phi_a phi_b
    x, w = np.polynomial.legendre.leggauss(8)
    ph = dg.lagrange(dg.lgl_nodes(2), x)
    M = np.einsum("q,aq,bq->ab", w, ph, ph)
    assert np.allclose(H.sum(axis=0), M, atol=1e-14)


# ---------------------------------------------------------------- VSS kernels (alpha in (1, 2])
@pytest.mark.parametrize("alpha", [1.3, 1.5, 1.8])
def test_vss_kernel_mode_reduction(alpha):
    """F for VSS from the reduced 1-D Gauss-Jacobi integral against direct
    product-rule quadratures of the defining integral with the symmetrised
    angular kernel (independent routes): the full sphere around sigma (tight)
    and the literal half sphere z >= 0 (slowly convergent, loose)."""
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(4):
        k = rng.integers(-8, 8, size=3).astype(float)
        s = rng.normal(size=3)
        s /= np.linalg.norm(s)
        rho = float(rng.uniform(0.3, 4.0))
        b = 0.071
        F1 = kernel.F_vss(k[None], rho, s, 6.0, 0.74, alpha, b)[0]
        F2 = kernel.F_vss_sphere(k, rho, s, 6.0, 0.74, alpha, b, axis="sigma")
        F3 = kernel.F_vss_sphere(k, rho, s, 6.0, 0.74, alpha, b, axis="z", n_theta=400, n_phi=800)
        assert abs(F1 - F2) <= 1e-10 * abs(F2)
        assert abs(F1 - F3) <= 2e-7 * abs(F3)


@pytest.mark.parametrize("alpha", [1.0, 2.0])
def test_vss_kernel_mode_reduces_to_vhs(alpha):
    """At alpha = 1 the angular factor is 1; at alpha = 2 its symmetrised form is
    ((1+t) + (1-t))/2 = 1: both give the VHS closed form with the same b."""
    rng = np.random.Generator(np.random.PCG64(8))
    kv = rng.integers(-10, 10, size=(20, 3)).astype(float)
    s = rng.normal(size=3)
    s /= np.linalg.norm(s)
    F1 = kernel.F_vss(kv, 2.7, s, 6.0, 0.81, alpha, 0.09)
    F2 = kernel.F_closed(np.linalg.norm(kv, axis=1), 2.7, 6.0, 0.81, 0.09)
    assert np.abs(F1 - F2).max() <= 1e-13 * np.abs(F2).max()
    assert kernel.vss_prefactor(0.81, 1.0) == pytest.approx(kernel.vhs_prefactor(0.81), rel=1e-15)


def test_vss_alpha2_operator_equals_vhs():
    """The whole VSS route (one transform and weight per (p, q)) at alpha = 2
    equals the VHS route (weights collapsed over q) with the same b."""
    N = 8
    f = W.maxwellian_mixture(1, N, 4.0, 12, noise=0.2)[0]
    b = kernel.vhs_prefactor(0.81)
    Pv = params(N, 4.0, 4, vss_alpha=2.0, prefactor=b)
    Ph = params(N, 4.0, 4, prefactor=b)
    Qv = spectral.collide(f, Pv)
    Qh = spectral.collide(f, Ph)
    assert np.abs(Qv - Qh).max() < 1e-13 * np.abs(Qh).max()


def test_vss_constant_f_has_zero_collisions():
    P = params(8, 5.0, 6, vss_alpha=1.5)
    f = np.full((8, 8, 8), 0.37)
    Q, gp, lp, _ = spectral.collide(f, P, return_parts=True)
    assert np.abs(Q).max() < 1e-13 * np.abs(lp).max()


@pytest.mark.parametrize("N,alpha", [(4, 1.5), (6, 1.3), (8, 1.7)])
def test_vss_fast_equals_direct_double_sum(N, alpha):
    f = W.maxwellian_mixture(1, N, 4.0, 13, noise=0.2)[0]
    P = params(N, 4.0, 4, vss_alpha=alpha)
    Qs = spectral.collide(f, P)
    Qd = direct.collide_direct(f, P)
    assert np.abs(Qs - Qd).max() < 1e-13 * np.abs(Qd).max()


def test_vss_maxwellian_is_near_equilibrium_spectrally():
    """Q(M) = 0 for every collision kernel: the discrete VSS operator on a
    Maxwellian decays spectrally with N."""
    rels = []
    for N in (8, 16, 24):
        L = 6.0
        f = W.maxwellian(N, L, 1.0, np.array([0.2, -0.1, 0.3]), 1.0)
        P = params(N, L, N // 2, vss_alpha=1.5)
        Q, gp, lp, _ = spectral.collide(f, P, return_parts=True)
        rels.append(np.abs(Q).max() / np.abs(gp).max())
    assert rels[0] > 10 * rels[1] > 100 * rels[2]
    assert rels[2] < 1e-4


def test_vss_scaling_translation_and_reflection():
    N = 8
    P = params(N, 4.0, 4, M=12, vss_alpha=1.4)
    f = W.maxwellian_mixture(1, N, 4.0, 14, noise=0.3)[0]
    Q = spectral.collide(f, P)
    assert np.abs(spectral.collide(2.5 * f, P) - 6.25 * Q).max() < 1e-12 * 6.25 * np.abs(Q).max()
    fr = np.roll(f, (2, -1, 3), axis=(0, 1, 2))
    assert np.abs(spectral.collide(fr, P) - np.roll(Q, (2, -1, 3), axis=(0, 1, 2))).max() < 1e-12 * np.abs(Q).max()
    # c -> -c (index j -> N-1-j on the cell-centred grid): the weights are even in k
    fm = f[::-1, ::-1, ::-1]
    Qm = spectral.collide(fm, P)
    assert np.abs(Qm - Q[::-1, ::-1, ::-1]).max() < 1e-12 * np.abs(Q).max()


def test_vss_symmetric_nyquist_weights_are_even_and_q_real():
    """Reading of the self-paired Nyquist index for sigma-dependent modes: the
    sign average makes the weights even under index reflection (so the gain and
    loss spectra are Hermitian and Q is real); the literal k = -N/2 does not."""
    N = 8
    f = W.maxwellian_mixture(1, N, 4.0, 15, noise=0.2)[0]
    P = params(N, 4.0, 4, M=12, vss_alpha=1.5)
    refl = lambda a: np.roll(a[..., ::-1, ::-1, ::-1], 1, axis=(-3, -2, -1))   # index n -> -n mod N
    assert np.abs(P.alpha_pq - refl(P.alpha_pq)).max() <= 1e-15 * np.abs(P.alpha_pq).max()
    assert np.abs(P.lam - refl(P.lam)).max() <= 1e-15 * np.abs(P.lam).max()
    Q, gp, lp, Qi = spectral.collide(f, P, return_parts=True)
    assert np.abs(Qi).max() <= 1e-14 * np.abs(Q).max()
    Pl = params(N, 4.0, 4, M=12, vss_alpha=1.5, nyquist="literal")
    assert np.abs(Pl.alpha_pq - refl(Pl.alpha_pq)).max() > 1e-6 * np.abs(Pl.alpha_pq).max()


# ---------------------------------------------------------------- 1-D RKDG driver (Section 3)
def _dg1d(I, P, N=4, L=4.0, inv_kn=0.0, left=None, right=None, coll="collocation", faces=None, M=6):
    from oracle import rkdg
    left = left or rkdg.Bc("periodic")
    right = right or rkdg.Bc("periodic")
    faces = np.linspace(0.0, 1.0, I + 1) if faces is None else faces
    return rkdg.Dg1d(faces, P, params(N, L, 2, M=M), inv_kn, left, right, coll=coll)


def test_rkdg_summation_by_parts():
    """S + S^T = phi(1) phi(1)^T - phi(-1) phi(-1)^T (integration by parts on the
    reference element), and the mass matrix is the Gauss weights."""
    for P in (1, 2, 3):
        d = _dg1d(2, P)
        lhs = d.S + d.S.T
        rhs = np.outer(d.phiR, d.phiR) - np.outer(d.phiL, d.phiL)
        assert np.abs(lhs - rhs).max() < 1e-13
        assert abs(d.w.sum() - 2.0) < 1e-14


def test_rkdg_free_streaming_converges():
    """Without collisions and with periodic ends every velocity point advects:
    f(t, x, c) = g(x - c_x t).  The DG error drops at the expected rate."""
    from oracle import rkdg
    errs = []
    for I in (4, 8, 16):
        d = _dg1d(I, 2, N=4, L=2.0)
        x = d.nodes_x()
        cx = d.cv[0]
        g = lambda y: 1.0 + 0.3 * np.sin(2 * np.pi * y)
        F = g(x[:, :, None, None, None] - 0.0 * cx[None, None])
        T, dt = 0.25, 0.2 / I / 2.0
        steps = int(round(T / dt))
        for _ in range(steps):
            F = d.step(F, dt, rk=3)
        exact = g(x[:, :, None, None, None] - cx[None, None] * steps * dt)
        errs.append(np.abs(F - exact).max())
    assert errs[0] > 6 * errs[1] > 36 * errs[2]
    assert errs[2] < 1e-4


def test_rkdg_diffuse_walls_conserve_mass_and_keep_wall_maxwellian():
    from oracle import rkdg
    N, L = 8, 5.0
    wl = rkdg.Bc("wall", u=(0.0, -0.2, 0.0), T=0.9)
    wr = rkdg.Bc("wall", u=(0.0, 0.2, 0.0), T=1.1)
    d = _dg1d(3, 2, N=N, L=L, inv_kn=0.5, left=wl, right=wr,
              faces=np.array([0.0, 0.2, 0.7, 1.0]))
    x = d.nodes_x()
    F = np.stack([[W.maxwellian(N, L, 1.0 + 0.2 * np.sin(3 * xx), np.array([0.1, 0.0, 0.0]), 1.0)
                   for xx in row] for row in x])
    m0 = d.total_mass(F)
    F1 = d.step(F, 0.01, rk=2)
    assert abs(d.total_mass(F1) - m0) <= 1e-13 * m0
    # equal walls at rest with the matching Maxwellian everywhere: no transport
    w0 = rkdg.Bc("wall", T=1.0)
    d0 = _dg1d(3, 2, N=N, L=L, left=w0, right=rkdg.Bc("wall", T=1.0))
    M = W.maxwellian(N, L, 1.0, np.zeros(3), 1.0)
    F = np.broadcast_to(M, (3, 3) + M.shape).copy()
    assert np.abs(d0.transport(F)).max() <= 1e-13 * np.abs(M).max()
    assert abs(d0.wall_density("L", M) * np.pi ** 1.5 - 1.0) < 1e-13


def test_rkdg_exact_and_collocated_collision_forms_agree_on_uniform_state():
    """For a state constant inside each element both collision forms give Q of
    that state at every node (the exact tensor sums to the mass matrix)."""
    N, L = 8, 5.0
    f = W.maxwellian_mixture(2, N, L, 21, noise=0.2)
    F = np.stack([np.broadcast_to(f[i], (3,) + f[i].shape) for i in range(2)])
    de = _dg1d(2, 2, N=N, L=L, inv_kn=1.0, coll="exact")
    dc = _dg1d(2, 2, N=N, L=L, inv_kn=1.0, coll="collocation")
    Ce, Cc = de.collision(F), dc.collision(F)
    assert np.abs(Ce - Cc).max() <= 1e-12 * np.abs(Cc).max()


def test_kernel_table_truncation_closed_form():
    """The SVD truncation of the gain-weight table (a9) on a table built from
    known factors: alpha = sum_i s_i u_i v_i^T with orthonormal u, v and
    s = (10, 4, 1e-3, 1e-9, 0).  The tolerance fixes the rank, and the result is
    the sum of the kept terms; the residual is orthogonal to it (Frobenius), and
    no random rank-r approximation is closer (Eckart-Young)."""
    rng = np.random.default_rng(7)
    m, N = 5, 4
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((N ** 3, m)))
    s = np.array([10.0, 4.0, 1e-3, 1e-9, 0.0])
    A = (U * s) @ V.T
    alpha = A.reshape(m, N, N, N)
    for tol, r in ((1e-6, 3), (1e-2, 2), (0.5, 1)):
        At, rank = kernel.truncate_alpha(alpha, svd_tol=tol)
        assert rank == r
        ref = (U[:, :r] * s[:r]) @ V[:, :r].T
        At = At.reshape(m, -1)
        assert np.abs(At - ref).max() <= 1e-12 * np.abs(A).max()
        R = A - At
        assert abs(np.sum(At * R)) <= 1e-12 * np.sum(A * A)
        assert abs(np.sum(A * A) - np.sum(At * At) - np.sum(R * R)) <= 1e-12 * np.sum(A * A)
        err = np.linalg.norm(R)
        for _ in range(20):
            Q, _ = np.linalg.qr(rng.standard_normal((m, r)))
            assert err <= np.linalg.norm(A - Q @ (Q.T @ A)) + 1e-12
    # a fixed rank, and the full rank reproduces the table
    At, rank = kernel.truncate_alpha(alpha, svd_rank=2)
    assert rank == 2 and np.abs(At.reshape(m, -1) - (U[:, :2] * s[:2]) @ V[:, :2].T).max() <= 1e-12 * 10
    At, rank = kernel.truncate_alpha(alpha, svd_rank=m)
    assert rank == m and np.abs(At - alpha).max() <= 1e-13 * 10


def test_vss_joint_weight_table_is_nearly_full_rank():
    """Why VSS plans keep the full alpha_pq table (no SVD over (p, q)): a rank-r
    factorisation alpha_pq = sum_s U[pq, s] V_s would replace the N_rho*M
    forward transforms per item by r, at the price of mixing the N_rho*M
    products into r sums, r*N_rho*M multiply-adds per point.  The joint table
    of a VSS kernel keeps most of its rank (here 79 of 96 at 1e-8, 66 at 1e-4;
    163 of 192 at the 1D DG batch's grid), and every radial node but the first
    keeps full rank over q, so the mixing (r*N_rho*M ~ 7.6e3 flops per point)
    costs far more than the 17 transforms it saves (5 log2(N^3) = 60 flops per
    point each, ~1.0e3 in all)."""
    N, L, Nr, M = 16, 6.0, 8, 12
    sph = W.sphere_rule(M)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81, vss_alpha=1.5)
    s = np.linalg.svd(P.alpha_pq.reshape(Nr * M, -1), compute_uv=False)
    r8, r4 = int((s > 1e-8 * s[0]).sum()), int((s > 1e-4 * s[0]).sum())
    assert r8 >= 0.8 * Nr * M and r4 >= 0.65 * Nr * M
    for p in range(1, Nr):
        sp = np.linalg.svd(P.alpha_pq[p].reshape(M, -1), compute_uv=False)
        assert int((sp > 1e-8 * s[0]).sum()) == M
    saved = Nr * M - r8
    assert r8 * Nr * M > 5 * saved * 5 * np.log2(N ** 3)
