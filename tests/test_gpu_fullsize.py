"""Full-size parity of the HIP path against the FP64 oracle, in the launch
configurations the benchmark times (autotuned schedule and chunk), with the
oracle fanned out over the host's cores.

* 1D DG batch (192 points, 32^3, M = 12, N_rho = 16, omega 0.81, SVD 1e-8):
  every item, both precisions, before and after the conservation projection.
* 2D DG batch (4096 points, 24^3): a fixed seeded subset of 64 items through
  the autotuned group graph launch.
* Plan tables (radial rule, gain and loss weights) against the oracle's.
* A VSS kernel (alpha = 1.5) at 32^3 against the oracle.

Tolerances (rel L-inf per item, normwise, max over items; unchanged from the
other parity tests): FP64 <= 1e-12, FP32 <= 2e-5; conservation residual
<= 1e-12.
"""
import numpy as np
import pytest

import oracle_pool
import workloads as W
from oracle import conserve as oc
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402

TOL = {qc.QCOLL_FP64: 1e-12, qc.QCOLL_FP32: 2e-5}


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel_items(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


@pytest.mark.timeout(900)
def test_dg1d_every_item_both_precisions():
    w = W.WORKLOADS["dg1d_32"]
    N, L, Nr, M = w["N"], w["L"], w["N_rho"], w["M"]
    sph = W.sphere_rule(M)
    f = W.mixture_for("dg1d_32")
    print(f"case dg1d_32: {f.shape[0]} items, oracle on {oracle_pool.workers()} processes", flush=True)
    ref = oracle_pool.collide_many(f, N=N, L=L, N_rho=Nr, M=M, omega=w["omega"], svd_tol=w["svd_tol"])
    ref_c, _ = oc.project(ref, N, L)
    fg = gpu(f)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], w["omega"], svd_tol=w["svd_tol"])
    for prec in (qc.QCOLL_FP64, qc.QCOLL_FP32):
        plan = qc.Plan(N, L, Nr, sphere=sph, omega=w["omega"], svd_rank=0, svd_tol=w["svd_tol"], precision=prec)
        assert plan.info()["rank"] == P.rank
        sch, ck = plan.autotune(fg)
        Q = plan.eval(fg)
        e = rel_items(Q.cpu().numpy(), ref)
        plan.conserve(Q)
        Qc = Q.cpu().numpy()
        ec = rel_items(Qc, ref_c)
        res = oc.conservation_residual(Qc, N, L).max()
        print(f"dg1d_32 prec={prec} schedule={sch} chunk={ck}: max rel {e.max():.3e} (item {e.argmax()}), "
              f"projected {ec.max():.3e}, conservation residual {res:.2e}", flush=True)
        assert e.max() <= TOL[prec] and ec.max() <= TOL[prec]
        assert res <= 1e-12
        plan.close()


@pytest.mark.timeout(900)
def test_dg2d_sampled_items_through_group_graph():
    w = W.WORKLOADS["dg2d_24"]
    N, L, Nr, M = w["N"], w["L"], w["N_rho"], w["M"]
    sph = W.sphere_rule(M)
    f = W.mixture_for("dg2d_24")
    idx = np.sort(np.random.Generator(np.random.PCG64(2024)).choice(f.shape[0], 64, replace=False))
    print(f"case dg2d_24: 64 of {f.shape[0]} items", flush=True)
    ref = oracle_pool.collide_many(f[idx], project=True, N=N, L=L, N_rho=Nr, M=M, omega=w["omega"])
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=w["omega"], precision=qc.QCOLL_FP32)
    fg = gpu(f)
    plan.autotune(fg)
    grp = qc.Group([plan], [f.shape[0]])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Q = grp.eval([fg], conserve=True, use_graph=True, stream=stream)[0]
    torch.cuda.synchronize()
    e = rel_items(Q.cpu().numpy()[idx], ref)
    print(f"dg2d_24: max rel {e.max():.3e}", flush=True)
    assert e.max() <= TOL[qc.QCOLL_FP32]
    grp.close()
    plan.close()


def gauss_legendre_mp(n, a, b, dps=40):
    """Gauss-Legendre nodes and weights on [a, b] in 40-digit arithmetic (Newton
    on the three-term recurrence of P_n), rounded to FP64 at the end: the exact
    rule that both FP64 routines (the plan's and the oracle's) approximate."""
    import mpmath
    with mpmath.workdps(dps):
        xs, ws = [], []
        for i in range(n):
            z = mpmath.cos(mpmath.pi * (i + mpmath.mpf(3) / 4) / (n + mpmath.mpf(1) / 2))
            for _ in range(100):
                p0, p1 = mpmath.mpf(1), z
                for k in range(2, n + 1):
                    p0, p1 = p1, ((2 * k - 1) * z * p1 - (k - 1) * p0) / k
                dp = n * (z * p1 - p0) / (z * z - 1)
                dz = p1 / dp
                z -= dz
                if abs(dz) < mpmath.mpf(10) ** (-dps + 5):
                    break
            xs.append((b - a) / 2 * z + (b + a) / 2)
            ws.append((b - a) / ((1 - z * z) * dp * dp))
        order = sorted(range(n), key=lambda i: xs[i])
        return (np.array([float(xs[i]) for i in order]), np.array([float(ws[i]) for i in order]))


@pytest.mark.parametrize("svd", [False, True])
def test_plan_tables_match_oracle(svd):
    """The device tables of an FP64 plan at the 1D DG batch's grid: the radial
    rule, the gain weights alpha_p (full, or truncated by the SVD at 1e-8) and
    the loss weights Lambda and Lambda_p, against the oracle's.  Both sides are
    FP64 evaluations of the same closed forms by different routines, each a few
    ulps from the exact values: the radial rule of each is checked against a
    40-digit evaluation (<= 2e-15 of the largest value), and the two sides
    against each other to <= 4e-15 (alpha_p and Lambda inherit the weights'
    last-digit differences)."""
    w = W.WORKLOADS["dg1d_32"]
    N, L, Nr, M = w["N"], w["L"], w["N_rho"], w["M"]
    sph = W.sphere_rule(M)
    tol = w["svd_tol"] if svd else None
    P = spectral.Params(N, L, Nr, sph[0], sph[1], w["omega"], svd_tol=tol)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=w["omega"], svd_rank=0 if svd else -1, svd_tol=tol or 0.0,
                   precision=qc.QCOLL_FP64)
    rho, wr = (np.array(x) for x in plan.radial())
    e_rho = np.abs(rho - P.kt.rho).max() / P.kt.rho.max()
    e_w = np.abs(wr - P.kt.w_rho).max() / P.kt.w_rho.max()
    a = plan.table("gain")
    e_a = np.abs(a - P.alpha).max() / np.abs(P.alpha).max()
    lam = plan.table("loss")
    e_l = np.abs(lam - P.lam).max() / np.abs(P.lam).max()
    xm, wm = gauss_legendre_mp(Nr, 0.0, P.kt.R)
    ex_plan = max(np.abs(rho - xm).max() / xm.max(), np.abs(wr - wm).max() / wm.max())
    ex_orac = max(np.abs(P.kt.rho - xm).max() / xm.max(), np.abs(P.kt.w_rho - wm).max() / wm.max())
    print(f"svd={svd}: rho {e_rho:.2e} w {e_w:.2e} alpha {e_a:.2e} Lambda {e_l:.2e}; radial rule vs 40 digits: "
          f"plan {ex_plan:.2e} oracle {ex_orac:.2e}", flush=True)
    assert ex_plan <= 2e-15 and ex_orac <= 2e-15
    assert e_rho <= 4e-15 and e_w <= 4e-15 and e_l <= 4e-15
    # the truncated table comes from two different SVD routines (the plan's
    # one-sided Jacobi, the oracle's LAPACK): equal to the truncation's
    # conditioning, far below the discarded singular values (1e-8 of the largest)
    assert e_a <= (1e-12 if svd else 4e-15)
    if not svd:
        lp = plan.table("loss_nodes")
        e_lp = np.abs(lp - P.kt.lam_p).max() / np.abs(P.kt.lam_p).max()
        assert e_lp <= 4e-15
    else:
        with pytest.raises(qc.QcollError) as e:
            plan.table("loss_nodes")
        assert e.value.code == 2
    plan.close()


@pytest.mark.timeout(600)
def test_vss_32_matches_oracle():
    """VSS kernel (alpha = 1.5) at 32^3 against the oracle (its kernel modes by
    the Gauss-Jacobi reduction, independent of the plan's Funk-Hecke series):
    FP64 and FP32 plans, two items, N_rho = 6, M = 6."""
    N, L, Nr, M, om, al = 32, 6.0, 6, 6, 0.81, 1.5
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(2, N, L, 3232)
    print("case vss 32^3 alpha 1.5", flush=True)
    ref = oracle_pool.collide_many(f, N=N, L=L, N_rho=Nr, M=M, omega=om, vss_alpha=al)
    for prec in (qc.QCOLL_FP64, qc.QCOLL_FP32):
        plan = qc.Plan(N, L, Nr, sphere=sph, omega=om, precision=prec, alpha=al)
        e = rel_items(plan.eval(gpu(f)).cpu().numpy(), ref)
        print(f"vss 32^3 prec={prec}: max rel {e.max():.3e}", flush=True)
        assert e.max() <= TOL[prec]
        plan.close()
