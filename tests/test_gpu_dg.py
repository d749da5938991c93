"""GPU parity of qcoll_dg_collide (MFMA contractions + batched Q) against the
oracle's literal weak-form double sum."""
import numpy as np
import pytest

import workloads as W
from oracle import conserve as oc
from oracle import dg, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("dim,P,basis", [(1, 1, "gauss"), (1, 2, "gauss"), (2, 1, "gauss"), (2, 2, "gauss"),
                                         (1, 2, "lgl"), (2, 1, "lgl")])
def test_dg_eigen_form_matches_double_sum(dim, P, basis):
    N, L, Nr = 8, 5.0, 4
    print(f"case dg dim={dim} P={P} basis={basis}", flush=True)
    H = dg.triple_tensor_1d(P, basis) if dim == 1 else dg.triple_tensor_2d(P, basis)
    K = H.shape[0]
    T, Wm, ranks = dg.eigen_factors(H)
    E = 3
    F = np.stack([W.maxwellian_mixture(K, N, L, 700 + 10 * e + P, noise=0.2) for e in range(E)])
    Pp = spectral.Params(N, L, Nr, *W.sphere_rule(6), 0.81)
    ref = np.stack([dg.collision_term_direct(F[e], H, Pp) for e in range(E)])
    plan = qc.Plan(N, L, Nr, sphere=None, omega=0.81, precision=qc.QCOLL_FP64)
    C = plan.dg_collide(gpu(F), gpu(T), gpu(Wm)).cpu().numpy()
    err = np.abs(C - ref).max() / np.abs(ref).max()
    print(f"R={T.shape[0]} (ranks {ranks}) rel {err:.3e}", flush=True)
    assert err <= 1e-12


def test_dg_quadrature_form_and_conservation():
    N, L, Nr = 12, 5.0, 6
    nodes, w = dg.gauss_nodes(2)
    K = 3
    T = np.eye(K)
    Wm = np.diag(w)
    E = 4
    F = np.stack([W.maxwellian_mixture(K, N, L, 800 + e) for e in range(E)])
    sph = W.sphere_rule(12)
    Pp = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
    C = plan.dg_collide(gpu(F), gpu(T), gpu(Wm), conserve=True).cpu().numpy()
    ref = np.stack([[w[m] * oc.project(spectral.collide(F[e, m], Pp)[None], N, L)[0][0] for m in range(K)]
                    for e in range(E)])
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(oc.conservation_residual(C.reshape(-1, N, N, N), N, L) <= 1e-12)


def test_dg_fp32_path():
    N, L, Nr = 16, 6.0, 8
    H = dg.triple_tensor_1d(2)
    T, Wm, _ = dg.eigen_factors(H)
    F = np.stack([W.maxwellian_mixture(3, N, L, 900 + e) for e in range(2)])
    sph = W.sphere_rule(12)
    Pp = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    ref = np.stack([dg.collision_term_factored(F[e], T, Wm, Pp) for e in range(2)])
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32)
    C = plan.dg_collide(gpu(F), gpu(T), gpu(Wm)).cpu().numpy()
    # each term carries the FP32 bound of Q; the combination is a small sum
    assert np.abs(C - ref).max() <= 5e-5 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
@pytest.mark.parametrize("conserve", [False, True])
def test_dg_collocated_form_matches_oracle_and_general_form(precision, conserve):
    """Collocated form (T = I, W = diag(J w_m), no contraction, the weights
    folded into the last store): against the oracle's w_m Q(F_m) (projected
    first when conserve) and against the general entry point with those T, W.
    Elements x nodes = 7 x 3 items at 16^3 (the FP32 plan runs the fused
    schedule), with an item count that is not a multiple of the chunk."""
    N, L, Nr = 16, 6.0, 8
    nodes, w = dg.gauss_nodes(2)
    K, E, J = 3, 7, 0.37
    wj = J * w
    F = np.stack([W.maxwellian_mixture(K, N, L, 1000 + e) for e in range(E)])
    sph = W.sphere_rule(12)
    Pp = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    Q = spectral.collide_batch(F.reshape(-1, N, N, N), Pp).reshape(E, K, N, N, N)
    if conserve:
        Q = oc.project(Q.reshape(-1, N, N, N), N, L)[0].reshape(Q.shape)
    ref = wj[None, :, None, None, None] * Q
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=precision)
    plan.set_chunk(8)
    Fg = gpu(F)
    C = plan.dg_collide_collocated(Fg, wj, conserve=conserve)
    Cg = plan.dg_collide(Fg, gpu(np.eye(K)), gpu(np.diag(wj)), conserve=conserve)
    tol = 1e-12 if precision == qc.QCOLL_FP64 else 2e-5
    e_ref = float(np.abs(C.cpu().numpy() - ref).max() / np.abs(ref).max())
    e_gen = float((C - Cg).abs().max() / Cg.abs().max())
    print(f"collocated prec={precision} conserve={conserve}: vs oracle {e_ref:.3e}, vs general {e_gen:.3e}",
          flush=True)
    assert e_ref <= tol
    assert e_gen <= 1e-14
    if conserve:
        assert np.all(oc.conservation_residual(C.cpu().numpy().reshape(-1, N, N, N), N, L) <= 1e-12)
