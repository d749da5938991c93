"""GPU parity of the bilinear operator Q(f, g) and of the paper's SVD form of
the DG collision term (general U, V factors) against the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import dg, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402

TOL = {qc.QCOLL_FP64: 1e-12, qc.QCOLL_FP32: 2e-5}


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
@pytest.mark.parametrize("N,L,N_rho,M,batch", [(8, 4.0, 4, 6, 5), (12, 5.0, 6, 12, 3), (16, 6.0, 8, 12, 2)])
def test_bilinear_matches_oracle(N, L, N_rho, M, batch, precision):
    print(f"case bilinear N={N} prec={precision}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(batch, N, L, 1100 + N)
    g = W.maxwellian_mixture(batch, N, L, 1200 + N, T_range=(0.7, 1.5))
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81)
    plan = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=precision)
    Q = plan.eval_bilinear(gpu(f), gpu(g)).cpu().numpy()
    ref = np.stack([spectral.collide_fg(f[i], g[i], P) for i in range(batch)])
    err = rel(Q, ref)
    print(f"rel {err:.3e}", flush=True)
    assert err <= TOL[precision]
    # Q(f, f) through the bilinear path equals qcoll_eval
    Qff = plan.eval_bilinear(gpu(f), gpu(f)).cpu().numpy()
    Qe = plan.eval(gpu(f)).cpu().numpy()
    assert rel(Qff, Qe) <= (1e-13 if precision == qc.QCOLL_FP64 else 2 * TOL[precision])


def test_dg_svd_form_matches_double_sum():
    N, L, Nr = 8, 4.0, 4
    sph = W.sphere_rule(6)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    for deg in (1, 2):
        H = dg.triple_tensor_1d(deg)
        K = deg + 1
        T1, T2, Wm = dg.svd_factors(H)
        E = 2
        F = np.stack([W.maxwellian_mixture(K, N, L, 1300 + 10 * e + deg, noise=0.2) for e in range(E)])
        ref = np.stack([dg.collision_term_direct_bilinear(F[e], H, P) for e in range(E)])
        plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
        C = plan.dg_collide_svd(gpu(F), gpu(T1), gpu(T2), gpu(Wm)).cpu().numpy()
        err = np.abs(C - ref).max() / np.abs(ref).max()
        print(f"P={deg} R={T1.shape[0]} rel {err:.3e}", flush=True)
        assert err <= 1e-12
