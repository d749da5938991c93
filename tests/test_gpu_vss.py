"""GPU parity of VSS plans (alpha in (1, 2], sigma-dependent kernel modes)
against the oracle, plus the reductions and the refused operations."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, kernel, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


# (N, L, N_rho, M, items, alpha): several tiles per axis and ragged item counts
CASES = [(8, 4.0, 4, 6, 5, 1.5), (12, 5.0, 6, 12, 3, 1.3), (16, 6.0, 8, 12, 2, 1.8)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("N,L,N_rho,M,items,alpha", CASES)
def test_vss_eval_matches_oracle(N, L, N_rho, M, items, alpha, precision):
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(items, N, L, 40 + N, noise=0.05)
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81, vss_alpha=alpha)
    ref = spectral.collide_batch(f, P)
    plan = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=precision, alpha=alpha)
    Q = plan.eval(gpu(f)).cpu().numpy()
    err = rel(Q, ref)
    tol = 1e-12 if precision == qc.QCOLL_FP64 else 2e-5
    print(f"VSS N={N} alpha={alpha} prec={precision}: rel {err:.3e}", flush=True)
    assert err <= tol


def test_vss_grid24_fp64_matches_oracle():
    N, L, Nr, M = 24, 6.0, 12, 12
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(2, N, L, 77)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.74, vss_alpha=1.6)
    ref = spectral.collide_batch(f, P)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.74, precision=qc.QCOLL_FP64, alpha=1.6)
    err = rel(plan.eval(gpu(f)).cpu().numpy(), ref)
    print(f"VSS N=24 FP64 rel {err:.3e}", flush=True)
    assert err <= 1e-12


def test_vss_alpha2_equals_vhs_plan():
    """At alpha = 2 the symmetrised angular kernel is 1: the VSS path (one
    forward transform and weight per (p, q)) equals the VHS path with the same b."""
    N, L, Nr = 16, 6.0, 8
    sph = W.sphere_rule(12)
    f = gpu(W.maxwellian_mixture(3, N, L, 55))
    b = kernel.vhs_prefactor(0.81)
    for prec in (qc.QCOLL_FP64, qc.QCOLL_FP32):
        pv = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, prefactor=b, precision=prec, alpha=2.0)
        ph = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, prefactor=b, precision=prec)
        Qv = pv.eval(f).cpu().numpy()
        Qh = ph.eval(f).cpu().numpy()
        err = rel(Qv, Qh)
        print(f"alpha=2 vs VHS prec={prec}: rel {err:.3e}", flush=True)
        assert err <= (1e-12 if prec == qc.QCOLL_FP64 else 2e-5)


def test_vss_constant_f_conservation_and_set_omega():
    N, L, Nr = 12, 5.0, 6
    sph = W.sphere_rule(12)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64, alpha=1.4)
    c = torch.full((2, N, N, N), 0.37, dtype=torch.float64, device="cuda")
    Qc = plan.eval(c).cpu().numpy()
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81, vss_alpha=1.4)
    _, _, lp, _ = spectral.collide(np.full((N, N, N), 0.37), P, return_parts=True)
    assert np.abs(Qc).max() <= 1e-12 * np.abs(lp).max()
    # conservation projection on a VSS result
    f = gpu(W.maxwellian_mixture(2, N, L, 61, noise=0.1))
    Q = plan.eval(f)
    mom = torch.empty(2, 5, dtype=torch.float64, device="cuda")
    plan.conserve(Q, moments=mom)
    from oracle import conserve as oc
    assert np.all(oc.conservation_residual(Q.cpu().numpy(), N, L) <= 1e-12)
    # omega change rebuilds the VSS tables: equal to a fresh plan
    plan.set_omega(0.74)
    fresh = qc.Plan(N, L, Nr, sphere=sph, omega=0.74, precision=qc.QCOLL_FP64, alpha=1.4)
    assert torch.equal(plan.eval(f), fresh.eval(f))


def test_vss_fused_schedule_request():
    N, L, Nr = 8, 4.0, 4
    plan = qc.Plan(N, L, Nr, sphere=W.sphere_rule(6), omega=0.81, precision=qc.QCOLL_FP32, alpha=1.5)
    f = gpu(W.maxwellian_mixture(1, N, L, 3))
    # the fused schedule has a VSS mode (FP32, N <= 32): requesting it is valid
    plan.set_schedule(2)
    assert torch.isfinite(plan.eval(f)).all()


# VJP tolerances as for VHS plans: FP64 1e-11, FP32 5e-5 relative to ||df||_inf
# (the adjoint carries the forward's gain/loss cancellation); d omega 1e-10 / 1e-4
VJP_TOL = {qc.QCOLL_FP64: (1e-11, 1e-10), qc.QCOLL_FP32: (5e-5, 1e-4)}


def _vss_vjp_case(N, L, N_rho, M, batch, alpha, precision, seed):
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(batch, N, L, seed)
    g = W.cotangent(f, seed + 1)
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81, vss_alpha=alpha)
    plan = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=precision, alpha=alpha)
    df, dw = plan.vjp(gpu(f), gpu(g), want_df=True, want_domega=True)
    ref = np.stack([adjoint.vjp_f(f[i], g[i], P) for i in range(batch)])
    refw = np.array([adjoint.vjp_omega(f[i], g[i], P) for i in range(batch)])
    e = rel(df.cpu().numpy(), ref)
    ew = float(np.max(np.abs(dw.cpu().numpy() - refw) / np.abs(refw)))
    return plan, f, g, P, e, ew


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
@pytest.mark.parametrize("N,L,N_rho,M,batch,alpha", [(8, 4.0, 4, 6, 3, 1.5), (12, 5.0, 6, 12, 2, 1.3),
                                                     (16, 6.0, 8, 12, 2, 1.8)])
def test_vss_vjp_matches_oracle(N, L, N_rho, M, batch, alpha, precision):
    """VSS VJP (h_pq = C_pq g per sphere point) against the oracle's adjoint:
    df and the omega gradient."""
    print(f"case vss vjp N={N} prec={precision}", flush=True)
    plan, *_, e, ew = _vss_vjp_case(N, L, N_rho, M, batch, alpha, precision, 4500 + N)
    print(f"vss vjp N={N} prec={precision}: df rel {e:.3e} domega rel {ew:.3e}", flush=True)
    assert e <= VJP_TOL[precision][0] and ew <= VJP_TOL[precision][1]
    plan.close()


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
def test_vss_vjp_32(precision):
    """32^3 VSS VJP against the oracle (FP64 at 32^3 transforms each sphere
    point's h volume on its own, FP32 both of a pair's at once), through the
    conservation projection, and the VJP of a 34-item batch (a full chunk and a
    ragged one) bit-identical to per-item calls."""
    N, L, Nr, M, al = 32, 6.0, 6, 6, 1.5
    print(f"case vss vjp 32^3 prec={precision}", flush=True)
    plan, f, g, P, e, ew = _vss_vjp_case(N, L, Nr, M, 2, al, precision, 4600)
    print(f"vss vjp 32^3 prec={precision}: df rel {e:.3e} domega rel {ew:.3e}", flush=True)
    assert e <= VJP_TOL[precision][0] and ew <= VJP_TOL[precision][1]
    from oracle import conserve as oc
    dfp, _ = plan.vjp(gpu(f), gpu(g), through_conserve=True)
    gp, _ = oc.project(g, N, L)
    refp = np.stack([adjoint.vjp_f(f[i], gp[i], P) for i in range(2)])
    ep = rel(dfp.cpu().numpy(), refp)
    print(f"vss vjp 32^3 through the projection: {ep:.3e}", flush=True)
    assert ep <= VJP_TOL[precision][0]
    fb = gpu(W.maxwellian_mixture(34, N, L, 4700))
    gb = gpu(W.cotangent(fb.cpu().numpy(), 4701))
    dfb, dwb = plan.vjp(fb, gb, want_domega=True)
    for i in (0, 17, 33):
        d1, w1 = plan.vjp(fb[i:i + 1].contiguous(), gb[i:i + 1].contiguous(), want_domega=True)
        assert torch.equal(d1[0], dfb[i]) and torch.equal(w1[0], dwb[i]), i
    plan.close()


@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
@pytest.mark.parametrize("N,L,N_rho,M,items,alpha", [(8, 4.0, 4, 6, 3, 1.5), (12, 5.0, 6, 12, 2, 1.8)])
def test_vss_bilinear_matches_oracle(N, L, N_rho, M, items, alpha, precision):
    """VSS bilinear Q(f, g) (each term's product Re(u_f u_g) weighted by its own
    alpha_pq) against the oracle; Q(f, f) through it equals qcoll_eval; the
    paper's U/V DG form with a VSS plan against the literal double sum."""
    print(f"case vss bilinear N={N} prec={precision}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(items, N, L, 2100 + N)
    g = W.maxwellian_mixture(items, N, L, 2200 + N, T_range=(0.8, 1.6))
    P = spectral.Params(N, L, N_rho, sph[0], sph[1], 0.81, vss_alpha=alpha)
    plan = qc.Plan(N, L, N_rho, sphere=sph, omega=0.81, precision=precision, alpha=alpha)
    Q = plan.eval_bilinear(gpu(f), gpu(g)).cpu().numpy()
    ref = np.stack([spectral.collide_fg(f[i], g[i], P) for i in range(items)])
    tol = 1e-12 if precision == qc.QCOLL_FP64 else 2e-5
    e = rel(Q, ref)
    Qff = plan.eval_bilinear(gpu(f), gpu(f)).cpu().numpy()
    e_ff = rel(Qff, plan.eval(gpu(f)).cpu().numpy())
    print(f"vss bilinear rel {e:.3e}; Q(f, f) through it vs eval {e_ff:.3e}", flush=True)
    assert e <= tol
    assert e_ff <= (1e-12 if precision == qc.QCOLL_FP64 else 4e-5)
    if precision == qc.QCOLL_FP64 and N == 8:
        from oracle import dg
        H = dg.triple_tensor_1d(1)
        T1, T2, Wm = dg.svd_factors(H)
        F = np.stack([W.maxwellian_mixture(2, N, L, 2300 + e_, noise=0.2) for e_ in range(2)])
        C = plan.dg_collide_svd(gpu(F), gpu(T1), gpu(T2), gpu(Wm)).cpu().numpy()
        refd = np.stack([dg.collision_term_direct_bilinear(F[e_], H, P) for e_ in range(2)])
        ed = np.abs(C - refd).max() / np.abs(refd).max()
        print(f"vss U/V DG form rel {ed:.3e}", flush=True)
        assert ed <= 1e-12


@pytest.mark.parametrize("N", [24, 32])
def test_vss_fused_schedule_matches_two_pass(N):
    """FP32 VSS plans run the gain loop on chip (fused kernel, VSS mode) by
    default; the two-pass schedule computes the same operator.  Both against
    the FP64 VSS plan on the 1D DG batch's grid."""
    L, Nr, M = 6.0, 8, 12
    sph = W.sphere_rule(M)
    f = gpu(W.maxwellian_mixture(3, N, L, 91))
    p64 = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64, alpha=1.5)
    ref = p64.eval(f).cpu().numpy()
    fused = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32, alpha=1.5)
    two = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32, alpha=1.5)
    two.set_schedule(1)
    e1 = rel(fused.eval(f).cpu().numpy(), ref)
    e2 = rel(two.eval(f).cpu().numpy(), ref)
    print(f"VSS N={N}: fused {e1:.3e} two-pass {e2:.3e}", flush=True)
    assert e1 <= 2e-5 and e2 <= 2e-5


@pytest.mark.timeout(600)
def test_vss_vjp_48_sub_chunks():
    """VSS VJP at 48^3 with the uneven batch's 48^3 node and sphere counts
    (N_rho = 24, M = 12), FP32: 31 items run as one chunk of three 10-item
    sub-chunks (the paired h_pq volumes of each sub-chunk read the spectrum of
    g, whose first volumes hold the accumulation's second half by then) plus a
    ragged chunk of one.  Items of each sub-chunk equal per-item calls bit for
    bit, and three items agree with the FP64 plan within the FP32 VJP bound."""
    N, L, Nr, M, al = 48, 9.0, 24, 12, 1.5
    sph = W.sphere_rule(M)
    print("case vss vjp 48^3, 31 items", flush=True)
    f = W.maxwellian_mixture(31, N, L, 4800, T_range=(2.5, 3.5))
    g = W.cotangent(f, 4801)
    p32 = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP32, alpha=al)
    fb, gb = gpu(f), gpu(g)
    dfb, dwb = p32.vjp(fb, gb, want_domega=True)
    for i in (0, 15, 29, 30):
        d1, w1 = p32.vjp(fb[i:i + 1].contiguous(), gb[i:i + 1].contiguous(), want_domega=True)
        assert torch.equal(d1[0], dfb[i]) and torch.equal(w1[0], dwb[i]), i
    p64 = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=qc.QCOLL_FP64, alpha=al)
    idx = [0, 15, 30]
    d64, w64 = p64.vjp(fb[idx].contiguous(), gb[idx].contiguous(), want_domega=True)
    e = rel(dfb[idx].cpu().numpy(), d64.cpu().numpy())
    ew = float(np.max(np.abs(dwb[idx].cpu().numpy() - w64.cpu().numpy()) / np.abs(w64.cpu().numpy())))
    print(f"vss vjp 48^3 FP32 vs FP64: df {e:.3e} domega {ew:.3e}", flush=True)
    assert e <= VJP_TOL[qc.QCOLL_FP32][0] and ew <= VJP_TOL[qc.QCOLL_FP32][1]
    p32.close()
    p64.close()
