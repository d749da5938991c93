"""Group launch (several grids in one graph launch) and autotuner, on the 2D DG
batch and the uneven three-grid batch, against per-plan calls and the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import conserve as oc
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


def test_dg2d_autotuned_graph_launch():
    """2D DG batch: 4096 points, 24^3, M=12, N_rho=12, omega 0.74, FP32; autotuned
    schedule, one graph launch, replayed with eager work in between."""
    w = W.WORKLOADS["dg2d_24"]
    N, L, Nr, M = w["N"], w["L"], w["N_rho"], w["M"]
    sph = W.sphere_rule(M)
    f = W.mixture_for("dg2d_24")
    fg = gpu(f)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=w["omega"], precision=qc.QCOLL_FP32)
    sch, ck = plan.autotune(fg)
    print(f"autotune: schedule {sch} chunk {ck}", flush=True)
    ref_eager = plan.eval(fg)
    plan.conserve(ref_eager)
    grp = qc.Group([plan], [f.shape[0]])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = []
        for it in range(3):
            Q = grp.eval([fg], conserve=True, use_graph=True, stream=stream)[0]
            stream.synchronize()
            outs.append(Q.clone())
            junk = plan.eval(fg[:7], stream=stream)   # eager work between replays
            stream.synchronize()
            del junk
    torch.cuda.synchronize()
    for Q in outs:
        assert torch.equal(Q, ref_eager)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], w["omega"])
    idx = [0, 1777, 4095]
    ref = np.stack([oc.project(spectral.collide(f[i], P)[None], N, L)[0][0] for i in idx])
    err = rel(outs[0].cpu().numpy()[idx], ref)
    print(f"rel vs oracle {err:.3e}", flush=True)
    assert err <= 2e-5


def test_uneven_three_grid_group_forward_and_vjp():
    """2048 points over 24^3 / 32^3 / 48^3 grids in one group launch (FP32 +
    conservation, SVD 1e-6): equals the per-plan calls; sampled items per grid
    against the oracle; the group VJP equals the per-plan VJPs."""
    com = W.UNEVEN_COMMON
    sph = W.sphere_rule(com["M"])
    plans, fs, fgs = [], [], []
    for i, g in enumerate(W.UNEVEN):
        plans.append(qc.Plan(g["N"], g["L"], g["N_rho"], sphere=sph, omega=com["omega"], svd_rank=0,
                             svd_tol=com["svd_tol"], precision=qc.QCOLL_FP32))
        f = W.uneven_grid(i)
        fs.append(f)
        fgs.append(gpu(f))
    print("ranks", [p.info()["rank"] for p in plans], flush=True)
    grp = qc.Group(plans, [g["items"] for g in W.UNEVEN])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Qg = grp.eval(fgs, conserve=True, use_graph=True, stream=stream)
        Qg2 = grp.eval(fgs, Qs=[torch.empty_like(q) for q in Qg], conserve=True, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    for i, p in enumerate(plans):
        Qe = p.eval(fgs[i])
        p.conserve(Qe)
        assert torch.equal(Qe, Qg[i])
        assert torch.equal(Qe, Qg2[i])
    for i, g in enumerate(W.UNEVEN):
        N, L = g["N"], g["L"]
        P = spectral.Params(N, L, g["N_rho"], sph[0], sph[1], com["omega"], svd_tol=com["svd_tol"])
        assert P.rank == plans[i].info()["rank"]
        k = g["items"] - 1
        ref = oc.project(spectral.collide(fs[i][k], P)[None], N, L)[0][0]
        err = rel(Qg[i].cpu().numpy()[k:k + 1], ref[None])
        print(f"grid {N}: rel vs oracle {err:.3e}", flush=True)
        assert err <= 2e-5
        assert np.all(oc.conservation_residual(Qg[i].cpu().numpy()[:8], N, L) <= 1e-12)
    # VJP through the group (through the projection) against per-plan VJPs
    gs = [gpu(W.cotangent(f, 9000 + i)) for i, f in enumerate(fs)]
    with torch.cuda.stream(stream):
        dfg = grp.vjp(fgs, gs, through_conserve=True, use_graph=False, stream=stream)
    torch.cuda.synchronize()
    for i, p in enumerate(plans):
        df, _ = p.vjp(fgs[i], gs[i], through_conserve=True)
        assert torch.equal(df, dfg[i])
