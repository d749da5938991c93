"""GPU parity of qcoll_vjp (df and d omega) against the FP64 oracle and finite differences."""
import numpy as np
import pytest

import oracle_pool
import workloads as W
from oracle import adjoint
from oracle import conserve as oc
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402

# FP32: the adjoint carries the same gain/loss cancellation as Q itself; the
# bound is stated relative to ||df||_inf like the forward's 2e-5.
TOL = {qc.QCOLL_FP64: 1e-11, qc.QCOLL_FP32: 5e-5}


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
@pytest.mark.parametrize("N,L,N_rho,M,batch", [(8, 4.0, 4, 6, 3), (12, 5.0, 6, 12, 2), (16, 6.0, 8, 12, 2)])
def test_vjp_matches_oracle(N, L, N_rho, M, batch, precision):
    print(f"case vjp N={N} prec={precision}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(batch, N, L, 400 + N)
    g = W.cotangent(f, 401 + N)
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81)
    plan = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=precision)
    df, dw = plan.vjp(gpu(f), gpu(g), want_df=True, want_domega=True)
    df = df.cpu().numpy()
    dw = dw.cpu().numpy()
    ref = np.stack([adjoint.vjp_f(f[i], g[i], P) for i in range(batch)])
    refw = np.array([adjoint.vjp_omega(f[i], g[i], P) for i in range(batch)])
    e = rel(df, ref)
    ew = float(np.max(np.abs(dw - refw) / np.abs(refw)))
    print(f"df rel {e:.3e} domega rel {ew:.3e}", flush=True)
    assert e <= TOL[precision]
    assert ew <= (1e-10 if precision == qc.QCOLL_FP64 else 1e-4)


def test_vjp_through_conservation():
    N, L, Nr = 12, 5.0, 6
    sph = W.sphere_rule(12)
    f = W.maxwellian_mixture(2, N, L, 77)
    g = W.cotangent(f, 78)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
    df, _ = plan.vjp(gpu(f), gpu(g), through_conserve=True)
    gp, _ = oc.project(g, N, L)
    ref = np.stack([adjoint.vjp_f(f[i], gp[i], P) for i in range(2)])
    assert rel(df.cpu().numpy(), ref) <= 1e-11


def test_vjp_truncated_plan_df_and_omega_refusal():
    N, L, Nr = 12, 5.0, 8
    sph = W.sphere_rule(12)
    f = W.maxwellian_mixture(2, N, L, 79)
    g = W.cotangent(f, 80)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81, svd_tol=1e-6)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, svd_rank=0, svd_tol=1e-6, precision=qc.QCOLL_FP64)
    assert plan.info()["rank"] == P.rank < Nr
    df, _ = plan.vjp(gpu(f), gpu(g))
    ref = np.stack([adjoint.vjp_f(f[i], g[i], P) for i in range(2)])
    assert rel(df.cpu().numpy(), ref) <= 1e-11
    with pytest.raises(qc.QcollError) as e:
        plan.vjp(gpu(f), gpu(g), want_df=False, want_domega=True)
    assert e.value.code == 2


def test_adjoint_check_full_size():
    """The adjoint-check batch (256 points, 32^3, M = 12, N_rho = 16, omega 0.81):
    dot-product test against central differences of the GPU's own Q in f (exact
    up to rounding: Q is quadratic) and in omega (h = 1e-6, FP64), every item."""
    w = W.WORKLOADS["adjoint_32"]
    N, L, Nr, M, om = w["N"], w["L"], w["N_rho"], w["M"], w["omega"]
    sph = W.sphere_rule(M)
    f = W.mixture_for("adjoint_32")
    g = W.cotangent(f, 4001)
    v = W.cotangent(f, 4002)
    fg, gg, vg = gpu(f), gpu(g), gpu(v)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=om, precision=qc.QCOLL_FP64)
    df, dw = plan.vjp(fg, gg, want_df=True, want_domega=True)
    h = 1e-3
    jv = (plan.eval(fg + h * vg) - plan.eval(fg - h * vg)) / (2 * h)
    lhs = (gg * jv).sum(dim=(1, 2, 3))
    rhs = (df * vg).sum(dim=(1, 2, 3))
    scale = (gg.abs() * jv.abs()).sum(dim=(1, 2, 3))
    err_f = float(((lhs - rhs).abs() / scale).max())
    hw = 1e-6
    plan.set_omega(om + hw)
    Qp = plan.eval(fg)
    plan.set_omega(om - hw)
    Qm = plan.eval(fg)
    dq = (Qp - Qm) / (2 * hw)
    fd = (dq * gg).sum(dim=(1, 2, 3))
    # normwise, like the dot-product test: |fd - dw| / sum |g dQ/domega|
    # (g . dQ/domega itself can nearly cancel for some items)
    err_w = float(((fd - dw).abs() / (dq * gg).abs().sum(dim=(1, 2, 3))).max())
    err_plain = float(((fd - dw).abs() / dw.abs().clamp_min(1e-30)).median())
    print(f"dot-product rel {err_f:.3e}  omega FD normwise {err_w:.3e} (median plain rel {err_plain:.3e})",
          flush=True)
    assert err_f <= 1e-10
    assert err_w <= 1e-6
    # one item against the oracle's FP64 gradient
    P = spectral.Params(N, L, Nr, sph[0], sph[1], om)
    ref = adjoint.vjp_f(f[5], g[5], P)
    assert np.abs(df[5].cpu().numpy() - ref).max() <= 1e-11 * np.abs(ref).max()


def test_autograd_function():
    N, L, Nr = 12, 5.0, 6
    sph = W.sphere_rule(12)
    f = gpu(W.maxwellian_mixture(2, N, L, 90)).requires_grad_(True)
    om = torch.tensor(0.81, dtype=torch.float64, device="cuda", requires_grad=True)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
    g = gpu(W.cotangent(W.maxwellian_mixture(2, N, L, 90), 91))
    Q = qc.collide(f, plan, omega=om, conserve=True)
    (Q * g).sum().backward()
    df, dw = plan.vjp(f.detach(), g, through_conserve=True, want_domega=True)
    assert torch.allclose(f.grad, df, rtol=0, atol=1e-14 * float(df.abs().max()))
    assert abs(float(om.grad) - float(dw.sum())) <= 1e-12 * abs(float(dw.sum()))


@pytest.mark.parametrize("N,L,N_rho,M,batch", [(24, 6.0, 8, 12, 3), (32, 6.0, 8, 12, 2)])
def test_fused_adjoint_matches_two_pass_and_fp64(N, L, N_rho, M, batch):
    """FP32 plans run the gain adjoint on chip (one workgroup per (item, node)
    pair, Hermitian half-spectrum accumulator); the two-pass schedule computes
    the same df and d omega.  Both against the FP64 plan."""
    print(f"case fused adjoint N={N}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(batch, N, L, 500 + N)
    g = W.cotangent(f, 501 + N)
    fg, gg = gpu(f), gpu(g)
    p64 = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
    ref, refw = (x.cpu().numpy() for x in p64.vjp(fg, gg, want_df=True, want_domega=True))
    fused = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32)
    two = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32)
    two.set_schedule(1)
    for name, pl in (("fused", fused), ("two-pass", two)):
        df, dw = (x.cpu().numpy() for x in pl.vjp(fg, gg, want_df=True, want_domega=True))
        e = rel(df, ref)
        ew = float(np.max(np.abs(dw - refw) / np.abs(refw)))
        print(f"{name}: df rel {e:.3e} domega rel {ew:.3e}", flush=True)
        assert e <= TOL[qc.QCOLL_FP32]
        assert ew <= 1e-4
    # the fused adjoint needs no per-term volume: a much smaller workspace
    assert fused.workspace_bytes(batch, 1) < two.workspace_bytes(batch, 1)


def test_fused_adjoint_truncated_plan_matches_oracle():
    N, L, Nr = 12, 5.0, 8
    sph = W.sphere_rule(12)
    f = W.maxwellian_mixture(3, N, L, 81)
    g = W.cotangent(f, 82)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81, svd_tol=1e-6)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, svd_rank=0, svd_tol=1e-6, precision=qc.QCOLL_FP32)
    df, _ = plan.vjp(gpu(f), gpu(g), through_conserve=True)
    gp, _ = oc.project(g, N, L)
    ref = np.stack([adjoint.vjp_f(f[i], gp[i], P) for i in range(3)])
    e = rel(df.cpu().numpy(), ref)
    print(f"truncated FP32 fused adjoint: df rel {e:.3e}", flush=True)
    assert e <= TOL[qc.QCOLL_FP32]


def test_fused_adjoint_full_size_against_fp64():
    """The adjoint-check batch (256 points, 32^3, M = 12, N_rho = 16), FP32 plan
    with the fused adjoint in the launch configuration the benchmark times,
    every item against the FP64 plan (itself pinned to the oracle above)."""
    w = W.WORKLOADS["adjoint_32"]
    N, L, Nr, M, om = w["N"], w["L"], w["N_rho"], w["M"], w["omega"]
    sph = W.sphere_rule(M)
    f = W.mixture_for("adjoint_32")
    g = W.cotangent(f, 4001)
    fg, gg = gpu(f), gpu(g)
    p64 = qc.Plan(N, L, Nr, sphere=sph, omega=om, precision=qc.QCOLL_FP64)
    ref, refw = p64.vjp(fg, gg, want_df=True, want_domega=True)
    p32 = qc.Plan(N, L, Nr, sphere=sph, omega=om, precision=qc.QCOLL_FP32)
    df, dw = p32.vjp(fg, gg, want_df=True, want_domega=True)
    e = float(((df - ref).abs().amax(dim=(1, 2, 3)) / ref.abs().amax(dim=(1, 2, 3))).max())
    # g . dQ/domega can nearly cancel for single items: the median is checked
    ew = float(((dw - refw).abs() / refw.abs().clamp_min(1e-30)).median())
    print(f"full size FP32 fused adjoint: max item df rel {e:.3e}, median domega rel {ew:.3e}", flush=True)
    assert e <= TOL[qc.QCOLL_FP32]
    assert ew <= 1e-4


@pytest.mark.parametrize("N_rho", [32, 40, 64])
def test_many_radial_nodes_eval_and_vjp(N_rho):
    """Up to the maximum N_rho = 64 (the register widths 32, 48 and 64 of the
    low-rank mixing, unpacking and omega-gradient kernels): eval of a full and
    an SVD-truncated plan in both precisions, and the VJP in f and omega,
    against the oracle at N = 8."""
    N, L, M = 8, 4.0, 6
    print(f"case N_rho={N_rho}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(3, N, L, 700 + N_rho)
    g = W.cotangent(f, 701 + N_rho)
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81)
    Pt = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81, svd_tol=1e-3)
    ref = spectral.collide_batch(f, P)
    reft = spectral.collide_batch(f, Pt)
    for prec in (qc.QCOLL_FP64, qc.QCOLL_FP32):
        full = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=prec)
        trunc = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, svd_rank=0, svd_tol=1e-3, precision=prec)
        trunc.set_schedule(1)   # the two-pass low-rank stage: mix to the rank-S basis
        assert trunc.info()["rank"] == Pt.rank
        tol = 1e-12 if prec == qc.QCOLL_FP64 else 2e-5
        e = rel(full.eval(gpu(f)).cpu().numpy(), ref)
        et = rel(trunc.eval(gpu(f)).cpu().numpy(), reft)
        df, dw = full.vjp(gpu(f), gpu(g), want_df=True, want_domega=True)
        rdf = np.stack([adjoint.vjp_f(f[i], g[i], P) for i in range(3)])
        rdw = np.array([adjoint.vjp_omega(f[i], g[i], P) for i in range(3)])
        ed = rel(df.cpu().numpy(), rdf)
        ew = float(np.max(np.abs(dw.cpu().numpy() - rdw) / np.abs(rdw)))
        print(f"prec={prec} rank={Pt.rank}: eval {e:.3e} truncated {et:.3e} df {ed:.3e} domega {ew:.3e}",
              flush=True)
        assert e <= tol and et <= tol
        assert ed <= TOL[prec]
        assert ew <= (1e-10 if prec == qc.QCOLL_FP64 else 1e-4)


@pytest.mark.parametrize("precision,N,L", [(qc.QCOLL_FP64, 16, 6.0), (qc.QCOLL_FP64, 32, 6.0),
                                           (qc.QCOLL_FP32, 48, 9.0)])
def test_two_pass_vjp_independent_of_chunking(precision, N, L):
    """Every item's df and d omega from the two-pass adjoint are the same bit for
    bit whether it is processed alone or inside a batch of several chunks and
    sub-chunks (the accumulation's fixed task halves, the sub-chunk sizing)."""
    batch = {16: 40, 32: 36, 48: 23}[N]
    print(f"case two-pass vjp chunking N={N} prec={precision} batch={batch}", flush=True)
    sph = W.sphere_rule(12)
    f = W.maxwellian_mixture(batch, N, L, 900 + N)
    g = W.cotangent(f, 901 + N)
    plan = qc.Plan(N, L, 16, sphere=sph, omega=0.81, precision=precision)
    df, dw = plan.vjp(gpu(f), gpu(g), through_conserve=True, want_domega=True)
    for lo, hi in ((0, 1), (batch - 3, batch)):
        d1, w1 = plan.vjp(gpu(f[lo:hi]), gpu(g[lo:hi]), through_conserve=True, want_domega=True)
        assert torch.equal(d1, df[lo:hi])
        assert torch.equal(w1, dw[lo:hi])
    plan.close()


@pytest.mark.timeout(900)
def test_uneven_48_vjp_against_oracle_and_fp64():
    """The 48^3 grid of the uneven batch (307 points, L = 9, N_rho = 24, M = 12,
    SVD 1e-6), FP32 two-pass VJP through the projection in the group's launch
    configuration: three items against the oracle's FP64 adjoint, every item
    against the FP64 plan (the same truncated gain table)."""
    com = W.UNEVEN_COMMON
    g48 = W.UNEVEN[2]
    N, L, Nr, M = g48["N"], g48["L"], g48["N_rho"], com["M"]
    sph = W.sphere_rule(M)
    f = W.uneven_grid(2)
    g = W.cotangent(f, 9002)
    fg, gg = gpu(f), gpu(g)
    print(f"case vjp 48^3: {f.shape[0]} items", flush=True)
    p32 = qc.Plan(N, L, Nr, sphere=sph, omega=com["omega"], svd_rank=0, svd_tol=com["svd_tol"],
                  precision=qc.QCOLL_FP32)
    p64 = qc.Plan(N, L, Nr, sphere=sph, omega=com["omega"], svd_rank=0, svd_tol=com["svd_tol"],
                  precision=qc.QCOLL_FP64)
    assert p32.info()["rank"] == p64.info()["rank"]
    df32, _ = p32.vjp(fg, gg, through_conserve=True)
    df64, _ = p64.vjp(fg, gg, through_conserve=True)
    e_all = float(((df32 - df64).abs().amax(dim=(1, 2, 3)) / df64.abs().amax(dim=(1, 2, 3))).max())
    print(f"48^3 FP32 vs FP64 plan, every item: max rel {e_all:.3e}", flush=True)
    idx = [0, 150, 306]
    ref = oracle_pool.vjp_many(f[idx], g[idx], project=True, N=N, L=L, N_rho=Nr, M=M, omega=com["omega"],
                               svd_tol=com["svd_tol"])
    e64 = rel(df64.cpu().numpy()[idx], ref)
    e32 = rel(df32.cpu().numpy()[idx], ref)
    print(f"48^3 vs oracle: FP64 {e64:.3e} FP32 {e32:.3e}", flush=True)
    assert e64 <= TOL[qc.QCOLL_FP64]
    assert e32 <= TOL[qc.QCOLL_FP32]
    assert e_all <= TOL[qc.QCOLL_FP32]


def test_autograd_two_omegas_before_one_backward():
    """Two collide calls at different omegas on one plan, then one backward
    through both: each part's gradient is taken at its own forward's omega
    (equal to separate backwards), and the plan keeps the last omega set."""
    N, L, Nr = 12, 5.0, 6
    sph = W.sphere_rule(12)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64)
    f0 = W.maxwellian_mixture(2, N, L, 95)
    g1 = gpu(W.cotangent(f0, 96))
    g2 = gpu(W.cotangent(f0, 97))
    f = gpu(f0).requires_grad_(True)
    o1 = torch.tensor(0.7, dtype=torch.float64, device="cuda", requires_grad=True)
    o2 = torch.tensor(0.9, dtype=torch.float64, device="cuda", requires_grad=True)
    Q1 = qc.collide(f, plan, omega=o1, conserve=True)
    Q2 = qc.collide(f, plan, omega=o2, conserve=True)
    ((Q1 * g1).sum() + (Q2 * g2).sum()).backward()
    assert plan.info()["omega"] == 0.9
    ref_df = torch.zeros_like(f)
    ref_dw = []
    for om, gq in ((0.7, g1), (0.9, g2)):
        p = qc.Plan(N, L, Nr, sphere=sph, omega=om, precision=qc.QCOLL_FP64)
        df, dw = p.vjp(f.detach(), gq, through_conserve=True, want_domega=True)
        ref_df += df
        ref_dw.append(float(dw.sum()))
        p.close()
    assert torch.allclose(f.grad, ref_df, rtol=0, atol=1e-13 * float(ref_df.abs().max()))
    assert abs(float(o1.grad) - ref_dw[0]) <= 1e-12 * abs(ref_dw[0])
    assert abs(float(o2.grad) - ref_dw[1]) <= 1e-12 * abs(ref_dw[1])
