"""Throughput of the collision operator on the 1D DG batch workload (one GPU).

Workload: 192 spatial points (64 elements x 3 Gauss points) of seeded
two-Maxwellian mixtures with 1% positive noise, N = 32^3 on [-6, 6]^3,
M = 12 half-sphere points, N_rho = 16, VHS omega = 0.81, gain table truncated
by SVD at 1e-8.  One step = qcoll_eval + qcoll_conserve over the whole batch.
The headline value is the FP32 path with the FP64 conservation fix; the FP64
path is timed beside it, and both are stated with their rel L-inf error
against the FP64 oracle on sampled items.  Both plans take their schedule and
items per chunk from the library's autotuner before any timing.  The timed
region records hipEvents around the dominant kernel only (its launch duration
feeds the roofline entry); the per-kernel breakdown comes from a separate
five-step pass with every kernel timed.

Outside the headline, "secondary" times the rows that the step does not cover,
each on its own synthetic workload: the DG weak-form term (MFMA contractions +
batched Q), a VSS kernel (alpha = 1.5) on the same batch, one SSP-RK2 step of
the 1-D RKDG driver on the paper's Fourier heat-transfer setup, the VJP, and
the group launches (2D DG batch; uneven three-grid batch, forward and VJP).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-acc] [--no-extras]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q(f,f) evals/sec at N=32^3,M=12,Nρ=16: FP32+fix vs FP64, at rel L∞ err"
WORKLOAD = "dg1d_32"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 157.3        # TFLOP/s, published (packed FP32)
FP32_VALU_NONPACKED = 78.6    # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
FP64_VALU_PEAK = 78.6         # TFLOP/s, published FP64 vector (one FP64 FMA per lane and clock)
# on-chip gain kernels (ALU bound): every term's transform and products stay in registers and LDS
ONCHIP_GAIN = ("gain fused", "gain c2", "gain q64")


def _oracle_item(args):
    # CPU baseline worker: the oracle as it stands, one item per call
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    i, f, prm = args
    from oracle import spectral
    from oracle import conserve as oc
    import workloads as W
    sph = W.sphere_rule(prm["M"])
    P = spectral.Params(prm["N"], prm["L"], prm["N_rho"], sph[0], sph[1], prm["omega"], svd_tol=prm["svd_tol"])
    Q = spectral.collide(f, P)
    Qc, _ = oc.project(Q[None], prm["N"], prm["L"])
    return i, Qc[0]


_FFT_CTX = {}


def _fft_item(args):
    """Context worker: the Appendix's formula with numpy.fft (pocketfft, FP64),
    two inverse transforms per (rho_p, sigma_q) term as the oracle writes it,
    the oracle's tables, then the conservation projection."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    i, f, prm = args
    from oracle import spectral
    from oracle import conserve as oc
    import workloads as W
    key = tuple(sorted(prm.items()))
    if key not in _FFT_CTX:
        sph = W.sphere_rule(prm["M"])
        _FFT_CTX[key] = spectral.Params(prm["N"], prm["L"], prm["N_rho"], sph[0], sph[1], prm["omega"],
                                        svd_tol=prm["svd_tol"])
    P = _FFT_CTX[key]
    fft, ifft = np.fft.fftn, np.fft.ifftn
    X = fft(f)
    Qh = np.zeros(f.shape, dtype=complex)
    for p, rho in enumerate(P.kt.rho):
        A = np.zeros(f.shape, dtype=complex)
        for q in range(P.M):
            bt = spectral.beta(P.N, P.L, 0.5 * rho * P.sphere_pts[q], P.nyquist)
            a = ifft(bt.real * X)
            b = ifft(bt.imag * X)
            A += P.sphere_w[q] * (a * a + b * b)
        Qh += P.alpha[p] * fft(A)
    Q = (ifft(Qh) - f * ifft(P.lam * X)).real
    Qc, _ = oc.project(Q[None], prm["N"], prm["L"])
    return i, Qc[0]


def cpu_fft_context(f, prm, ref):
    """CPU context figure: the same formula with numpy.fft instead of the
    oracle's DFT matrices, over the items the oracle leg computed, one process
    per core; also its largest deviation from the oracle."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    items = sorted(ref)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(min(cores, len(items))) as pool:
        res = dict(pool.map(_fft_item, [(i, f[i], prm) for i in items]))
    dt = time.perf_counter() - t0
    dev = max(float(np.abs(res[i] - ref[i]).max() / np.abs(ref[i]).max()) for i in items)
    return {"value": len(items) / dt, "unit": "evals/s", "cores": min(cores, len(items)),
            "kind": "numpy.fft FP64, the Appendix's formula (context, not the target)",
            "sample": f"the {len(items)} items of the oracle leg, {dt:.1f} s wall incl. process start and tables",
            "max_rel_vs_oracle": dev}


def cpu_baseline(f, prm, n_items):
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    n = min(n_items, f.shape[0])
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(min(cores, n)) as pool:
        res = pool.map(_oracle_item, [(i, f[i], prm) for i in range(n)])
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "evals/s", "cores": min(cores, n), "kind": "oracle",
            "sample": f"{n} of the {f.shape[0]} items (FP64 naive-DFT oracle incl. conservation projection), "
                      f"{dt:.1f} s wall on {min(cores, n)} processes"}, dict(res)


def model_flops_fft(N):
    """Model flops of one complex 3-D transform of n = N^3 points: 5 n log2 n."""
    n3 = N ** 3
    return 5.0 * n3 * math.log2(n3)


def model_flops_per_term(N):
    """Model flops of one (item, rho_p, sigma_q) term of the hot loop: one complex
    3-D transform plus 23 pointwise flops per point (the shift multiplier, the
    product of the two shifted copies and the weighted accumulation)."""
    return model_flops_fft(N) + 23.0 * N ** 3


def algorithmic_bytes(role, fp32, B, N, Nr, M, npair, nv, half=None):
    """Bytes per step that a pass of the pipeline must move through HBM (item
    data only; the shared plan tables are read from cache): what each kernel
    role reads and writes once, by the layout of the workspace.  None for roles
    without a byte model."""
    es = 4 if fp32 else 8           # working precision of the gain
    c = 2 * es                      # complex in the working precision
    n3, nh = N ** 3, (N // 2 + 1) * N * N
    if half is None:
        half = fp32                 # the fused schedule keeps half spectra
    c64 = 16                        # complex FP64 (spectra, low-rank stage, gain inverse, assembly)
    m = {
        "forward slab": B * n3 * (8 + 16),
        "forward pencil": B * n3 * ((16 + 16 + 8) if fp32 else (16 + 16)),
        # the item spectrum once (each of its Nr*M terms re-reads it from L2),
        # every term's volume written once
        "gain slab": B * n3 * c + B * Nr * M * n3 * c,
        "gain pencil": B * Nr * n3 * (M * c + es),
        "mix": B * n3 * (Nr + nv) * es,
        # two-pass low-rank stage in FP64 for both precisions: A_p pairs in,
        # complex FP64 volumes out; then the pencil sum over the pairs
        "low-rank slab": B * npair * n3 * (2 * es + c64),
        "low-rank pencil": B * n3 * (npair * c64 + c64),
        "gain inverse slab": B * (nh if half else n3) * (c64 + c64),
        "loss slab": B * (nh if half else n3) * (16 + 16),
        # gain and loss spectra in (complex FP64), f in and Q out (FP64)
        "assemble": B * ((nh * (c64 + 16) + n3 * 16) if half else n3 * (c64 + 16 + 16)),
        # Nr FP32 half spectra in, one FP64 half spectrum out
        "sum nodes": B * nh * (8 * Nr + 16),
        "conserve": B * n3 * (8 + 8),
        "gain fused": B * n3 * 8 + B * Nr * nh * 8,
        # FP64 on chip: the item spectrum once (its Nr classes re-read it from L2), A_p written once
        "gain c2": B * n3 * 16 + B * Nr * n3 * 8,
        "gain q64": B * n3 * 16 + B * Nr * n3 * 8,
    }
    return m.get(role)


def hbm_passes(kt, steps, fp32, B, N, Nr, M, npair, nv, half=None):
    """Per kernel role: time per step, algorithmic bytes per step and the rate
    against the HBM peak (the on-chip gain kernel is ALU bound and listed
    with its bytes only)."""
    out = {}
    tot_b = tot_ms = 0.0
    for role, (ms, n) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        b = algorithmic_bytes(role, fp32, B, N, Nr, M, npair, nv, half)
        ms_step = ms / steps
        ent = {"ms_per_step": round(ms_step, 4), "launches_per_step": n / steps}
        if b is not None:
            gbs = b / (ms_step * 1e-3) / 1e9
            ent.update({"algorithmic_MB": round(b / 1e6, 2), "GB_per_s": round(gbs, 1),
                        "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
            if role not in ONCHIP_GAIN:
                tot_b += b
                tot_ms += ms_step
        out[role] = ent
    summary = None
    if tot_ms > 0:
        gbs = tot_b / (tot_ms * 1e-3) / 1e9
        summary = {"roles": "every slab/pencil/reduction pass through HBM", "ms_per_step": round(tot_ms, 4),
                   "algorithmic_MB": round(tot_b / 1e6, 1), "GB_per_s": round(gbs, 1),
                   "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return out, summary


def measured_traffic(kernel, items_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, scaled
    from the items per launch the counters were taken at to this run's (both the
    spectra read and the per-node spectra written grow linearly with it), or None
    if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get(kernel)
    if not ent or ent.get("source_sha256") != source_digest(ent.get("sources", [])):
        return None
    b = ent.get("bytes_per_launch")
    n0 = ent.get("items_per_launch")
    return b if b is None or not n0 else b * items_per_launch / n0


def source_digest(files):
    """sha256 over the named kernel sources (the counters go stale when they change)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1809_10186_amd", "csrc")
    for fn in files:
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fn.encode() + fh.read())
    return h.hexdigest()


def roofline(name, tot_ms, launches, steps, B, N, Nr, M, fp32=True, npair=0, nv=0):
    """Roofline entry of the dominant kernel.  Units per launch are explained in
    DESIGN.md (section "Kernels and their rooflines")."""
    avg_ms = tot_ms / launches
    key = name if fp32 else f"{name} fp64"
    base = {"kernel": name, "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "traffic": measured_traffic(key, B * steps / launches)}
    if name == "gain fused":
        # ALU bound: model flops of every (item, p, q) term of the timed region
        # plus the forward transform of every (item, p) accumulator (the
        # low-rank stage the kernel runs on chip)
        flops = B * Nr * steps * (M * model_flops_per_term(N) + model_flops_fft(N))
        per_launch = flops / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        base.update({"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VALU_PEAK, 4),
                     "flops_per_launch": per_launch,
                     "peak_nonpacked_fp32": FP32_VALU_NONPACKED})
        return base
    if name in ("gain c2", "gain q64"):
        # FP64 gain loop on chip: model flops of every (item, p, q) term (the
        # low-rank stage runs after it as two passes)
        flops = B * Nr * steps * M * model_flops_per_term(N)
        per_launch = flops / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        base.update({"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK, 4),
                     "flops_per_launch": per_launch})
        return base
    b = algorithmic_bytes(name, fp32, B, N, Nr, M, npair, nv)
    total = None if b is None else b * steps
    if total is None:
        base.update({"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None})
        return base
    per_launch = total / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    base.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": per_launch})
    return base


def copy_probe(mib=1024, reps=5):
    """A plain device copy of known size, for calibrating the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": reps}))


def stream_probe(mib=1024, reps=20, copy_sizes=(16, 32, 64, 128, 192, 256, 512)):
    """Achievable HBM rates on this device: a 1 GiB copy (read + write), a
    1 GiB fill (write only) and a 1 GiB sum (read only), timed with events;
    then copies of smaller buffers, whose source and destination fit the
    Infinity Cache (256 MiB) or the L2s (8 x 4 MiB)."""
    import torch

    def rate(fn, nbytes, n_rep):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_rep):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n_rep
        return {"ms": round(ms, 4), "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 8 * n), ("fill", lambda: b.fill_(1.5), 4 * n),
                             ("read", lambda: a.sum(), 4 * n)):
        out[name] = rate(fn, nbytes, reps)
    copies = {}
    for m in copy_sizes:
        k = m * (1 << 20) // 4
        copies[str(m)] = rate(lambda: b[:k].copy_(a[:k]), 8 * k, max(reps, 2048 // m))["GB_per_s"]
    print(json.dumps({"stream_probe_MiB": mib, **out, "copy_GB_per_s_by_MiB": copies}))


def median_call_ms(torch, fn, n):
    """Wall time of one call: the median of n synchronised calls after an
    untimed one (the secondary rows are single calls of 0.3-100 ms, where one
    slow call would move a mean)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(n):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)) * 1e3


def extras(qc, torch, W, reps=7):
    """Secondary measurements of the rows outside the headline step, each on its
    own synthetic workload: the DG weak-form term with the MFMA contractions,
    the VJP, and the group launches.  Wall time per call after one untimed call."""
    out = {}

    def timeit(fn, n=reps):
        return median_call_ms(torch, fn, n)

    # DG weak form on the 1D DG batch: 64 elements, P = 2 on Gauss nodes (K = 3).
    # Collocation form T = I, W = diag(w_q) (192 Q evals) and eigen form of the
    # triple tensor (R = 6 terms per element, 384 Q evals), FP32 + FP64 fix.
    w = W.WORKLOADS["dg1d_32"]
    sph = W.sphere_rule(w["M"])
    plan = qc.Plan(w["N"], w["L"], w["N_rho"], sphere=sph, omega=w["omega"], svd_rank=0, svd_tol=w["svd_tol"],
                   precision=qc.QCOLL_FP32)
    E, K = 64, 3
    F = torch.from_numpy(W.mixture_for("dg1d_32")).to("cuda").reshape(E, K, w["N"], w["N"], w["N"])
    xg, wg = np.polynomial.legendre.leggauss(K)
    forms = {"collocation": (np.eye(K), np.diag(wg))}
    # eigen form of the exact triple tensor of the Lagrange basis on the Gauss nodes
    xq, wq = np.polynomial.legendre.leggauss(3 * K)
    ph = np.ones((K, xq.size))
    for l in range(K):
        for k in range(K):
            if k != l:
                ph[l] *= (xq - xg[k]) / (xg[l] - xg[k])
    H = np.einsum("q,mq,aq,bq->mab", wq, ph, ph, ph)
    rows, cols = [], []
    for m in range(K):
        lam, U = np.linalg.eigh(H[m])
        for r in np.nonzero(np.abs(lam) > 1e-13 * np.abs(lam).max())[0]:
            rows.append(U[:, r])
            c = np.zeros(K)
            c[m] = lam[r]
            cols.append(c)
    forms["eigen"] = (np.array(rows), np.array(cols).T)
    # collocation form through its own entry point: no contraction (T = I), the
    # weights folded into the last store (W = diag(w)); same 192 evaluations as
    # the headline step
    Cout = torch.empty_like(F)
    plan.autotune(F.reshape(-1, w["N"], w["N"], w["N"]))
    ms = timeit(lambda: plan.dg_collide_collocated(F, wg, conserve=True, out=Cout))
    out["dg_collide_collocated"] = {"elements": E, "K": K, "R": K, "ms": round(ms, 3),
                                    "q_evals_per_s": round(E * K / (ms * 1e-3), 1)}
    for name, (T, Wm) in forms.items():
        Tg = torch.from_numpy(np.ascontiguousarray(T)).to("cuda")
        Wg = torch.from_numpy(np.ascontiguousarray(Wm)).to("cuda")
        Cout = torch.empty_like(F)
        ms = timeit(lambda: plan.dg_collide(F, Tg, Wg, conserve=True, out=Cout))
        qc.timing_reset()
        qc.timing_select("dg contract")
        qc.timing_enable(True)
        plan.dg_collide(F, Tg, Wg, conserve=True, out=Cout)
        qc.timing_enable(False)
        tc, nc = qc.timing_read().get("dg contract", (0.0, 0))
        qc.timing_select(None)
        out[f"dg_collide_{name}"] = {"elements": E, "K": K, "R": int(T.shape[0]), "ms": round(ms, 3),
                                     "q_evals_per_s": round(E * T.shape[0] / (ms * 1e-3), 1),
                                     "mfma_contract_ms": round(tc, 4), "mfma_contract_launches": nc}
    plan.close()

    # VSS kernel (alpha = 1.5, sigma-dependent kernel modes) on the 1D DG batch, eval + conserve
    w = W.WORKLOADS["dg1d_32"]
    sph = W.sphere_rule(w["M"])
    f = torch.from_numpy(W.mixture_for("dg1d_32")).to("cuda")
    Qv = torch.empty_like(f)
    for prec, tag in ((qc.QCOLL_FP32, "fp32"), (qc.QCOLL_FP64, "fp64")):
        pl = qc.Plan(w["N"], w["L"], w["N_rho"], sphere=sph, omega=w["omega"], precision=prec, alpha=1.5)
        pl.autotune(f, Qv)

        def vss_step():
            pl.eval(f, Qv)
            pl.conserve(Qv)
        ms = timeit(vss_step)
        out[f"vss_alpha1.5_{tag}"] = {"items": f.shape[0], "ms": round(ms, 3),
                                      "evals_per_s": round(f.shape[0] / (ms * 1e-3), 1)}
        pl.close()
    del f, Qv

    # RKDG driver (Section 3): Fourier heat transfer between walls at 263 K and
    # 283 K (T0 = 273 K), Maxwell molecules, Kn 1.582 (Cercignani), 10 elements
    # of order 2 refined towards the walls, [-5.09, 5.09]^3 with 24^3 points,
    # M = 6: one SSP-RK2 step = 2 x (30 collision evaluations + transport)
    h = 1.23 ** np.arange(5)
    h = 0.5 * h / h.sum()
    left = np.concatenate([[0.0], np.cumsum(h)])
    faces = np.concatenate([left, 1.0 - left[::-1][1:]])
    for prec, tag in ((qc.QCOLL_FP32, "fp32"), (qc.QCOLL_FP64, "fp64")):
        pl = qc.Plan(24, 5.09, 12, sphere=None, omega=1.0, precision=prec)
        dd = qc.Dg1d(pl, faces, 2, (np.pi / 2.0) / 1.582, qc.Bc("wall", T=263.0 / 273.0),
                     qc.Bc("wall", T=283.0 / 273.0))
        M0 = W.maxwellian(24, 5.09, 1.0, np.zeros(3), 1.0)
        Fd = torch.from_numpy(np.broadcast_to(M0, (10, 3) + M0.shape).copy()).to("cuda")
        ms = timeit(lambda: dd.step(Fd, 0.002, rk=2), n=10)
        out[f"dg1d_fourier_rk2_{tag}"] = {"elements": 10, "order": 2, "grid": "24^3", "M": 6,
                                          "ms_per_step": round(ms, 3), "q_evals_per_step": 60}
        dd.close()
        pl.close()

    # VJP (f and omega, through the conservation projection) on 256 items at 32^3
    w = W.WORKLOADS["adjoint_32"]
    sph = W.sphere_rule(w["M"])
    f = torch.from_numpy(W.mixture_for("adjoint_32")).to("cuda")
    g = torch.from_numpy(W.cotangent(W.mixture_for("adjoint_32"), 4)).to("cuda")
    for prec, tag in ((qc.QCOLL_FP32, "fp32"), (qc.QCOLL_FP64, "fp64")):
        pl = qc.Plan(w["N"], w["L"], w["N_rho"], sphere=sph, omega=w["omega"], precision=prec)
        df = torch.empty_like(f)
        dw = torch.empty(f.shape[0], dtype=torch.float64, device="cuda")
        ms = timeit(lambda: pl.vjp(f, g, df=df, domega=dw, through_conserve=True, want_domega=True))
        out[f"vjp_{tag}"] = {"items": f.shape[0], "ms": round(ms, 3),
                             "items_per_s": round(f.shape[0] / (ms * 1e-3), 1)}
        pl.close()
    del f, g

    # group launches: 2D DG batch (4096 points at 24^3, one plan, autotuned, graph)
    # and the uneven three-grid batch (2048 points, forward and VJP), FP32 + fix
    stream = torch.cuda.Stream()
    w = W.WORKLOADS["dg2d_24"]
    sph = W.sphere_rule(w["M"])
    f = torch.from_numpy(W.mixture_for("dg2d_24")).to("cuda")
    pl = qc.Plan(w["N"], w["L"], w["N_rho"], sphere=sph, omega=w["omega"], precision=qc.QCOLL_FP32)
    pl.autotune(f)
    grp = qc.Group([pl], [f.shape[0]])
    Qs = [torch.empty_like(f)]
    with torch.cuda.stream(stream):
        ms = timeit(lambda: grp.eval([f], Qs=Qs, conserve=True, use_graph=True, stream=stream))
    out["group_dg2d_24"] = {"items": f.shape[0], "ms": round(ms, 3), "evals_per_s": round(f.shape[0] / (ms * 1e-3), 1)}
    grp.close()
    pl.close()
    del f, Qs
    out.update(group_uneven(qc, torch, W, reps))
    return out


def group_uneven(qc, torch, W, reps=7):
    """The uneven three-grid batch through the autotuned group graph (eval with
    the projection, and the VJP through it), and each branch alone."""
    def timeit(fn):
        return median_call_ms(torch, fn, reps)

    out = {}
    stream = torch.cuda.Stream()
    com = W.UNEVEN_COMMON
    sph = W.sphere_rule(com["M"])
    plans, fs, gs = [], [], []
    for i, gdef in enumerate(W.UNEVEN):
        plans.append(qc.Plan(gdef["N"], gdef["L"], gdef["N_rho"], sphere=sph, omega=com["omega"], svd_rank=0,
                             svd_tol=com["svd_tol"], precision=qc.QCOLL_FP32))
        fi = W.uneven_grid(i)
        fs.append(torch.from_numpy(fi).to("cuda"))
        gs.append(torch.from_numpy(W.cotangent(fi, 10 + i)).to("cuda"))
    grp = qc.Group(plans, [gdef["items"] for gdef in W.UNEVEN])
    Qs = [torch.empty_like(x) for x in fs]
    dfs = [torch.empty_like(x) for x in fs]
    grp.autotune(fs, Qs)          # every member plan, before the graph is captured
    n = sum(gdef["items"] for gdef in W.UNEVEN)
    with torch.cuda.stream(stream):
        ms = timeit(lambda: grp.eval(fs, Qs=Qs, conserve=True, use_graph=True, stream=stream))
        ms_v = timeit(lambda: grp.vjp(fs, gs, dfs=dfs, through_conserve=True, use_graph=True, stream=stream))
    # each branch alone (eager, the same tuned plan): the group's time against
    # its longest branch shows whether the critical path or the launch
    # structure bounds the group
    branch = {}
    for pl, fi, gi, qi, di, gdef in zip(plans, fs, gs, Qs, dfs, W.UNEVEN):
        e_ms = timeit(lambda: (pl.eval(fi, qi), pl.conserve(qi)))
        v_ms = timeit(lambda: pl.vjp(fi, gi, df=di, through_conserve=True))
        branch[f"{gdef['N']}^3 x {gdef['items']}"] = {"eval_ms": round(e_ms, 3), "vjp_ms": round(v_ms, 3)}
    out["group_uneven"] = {"items": n, "grids": "1024 x 24^3 + 717 x 32^3 + 307 x 48^3",
                           "eval_ms": round(ms, 3), "evals_per_s": round(n / (ms * 1e-3), 1),
                           "vjp_ms": round(ms_v, 3), "vjps_per_s": round(n / (ms_v * 1e-3), 1),
                           "branches_alone": branch,
                           "sum_of_branches_eval_ms": round(sum(b["eval_ms"] for b in branch.values()), 3),
                           "sum_of_branches_vjp_ms": round(sum(b["vjp_ms"] for b in branch.values()), 3)}
    grp.close()
    for pl in plans:
        pl.close()
    return out


def uneven48(qc, torch, W, steps, warmup):
    """The 48^3 grid of the uneven batch alone (the group's critical path):
    autotuned eval + conserve and the VJP through the projection, per-kernel
    breakdown with algorithmic bytes (for profiler runs)."""
    com, g = W.UNEVEN_COMMON, W.UNEVEN[2]
    N, Nr, M = g["N"], g["N_rho"], com["M"]
    sph = W.sphere_rule(M)
    plan = qc.Plan(N, g["L"], Nr, sphere=sph, omega=com["omega"], svd_rank=0, svd_tol=com["svd_tol"],
                   precision=qc.QCOLL_FP32)
    f_np = W.uneven_grid(2)
    f = torch.from_numpy(f_np).to("cuda")
    gq = torch.from_numpy(W.cotangent(f_np, 10 + 2)).to("cuda")
    B = f.shape[0]
    Q, df = torch.empty_like(f), torch.empty_like(f)
    tuned = plan.autotune(f, Q)
    inf = plan.info()
    out = {"workload": f"uneven batch, 48^3 grid: {B} points, L={g['L']}, N_rho={Nr}, M={M}, rank {inf['rank']}",
           "autotuned_schedule_chunk": tuned}
    for name, fn in (("eval_conserve", lambda: (plan.eval(f, Q), plan.conserve(Q))),
                     ("vjp", lambda: plan.vjp(f, gq, df=df, through_conserve=True))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        # wall time without per-launch events, then the per-role breakdown in
        # a second pass with them (several hundred launches per step here)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps * 1e3
        qc.timing_reset()
        qc.timing_select(None)
        qc.timing_enable(True)
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        qc.timing_enable(False)
        kt = qc.timing_read()
        ent = {"ms": round(dt, 3)}
        if name == "eval_conserve":
            passes, summ = hbm_passes(kt, steps, True, B, N, Nr, M, (inf["rank"] + 1) // 2, inf["rank"],
                                      half=False)
            ent.update({"hbm_passes": passes, "hbm_passes_total": summ})
        else:
            ent["kernel_ms"] = {k: round(v[0] / steps, 4) for k, v in kt.items()}
        out[name] = ent
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-acc", action="store_true")
    ap.add_argument("--cpu-items", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary measurements (DG, VJP, groups)")
    ap.add_argument("--schedule", type=int, default=0, help="hot-loop schedule of the FP32 plan (0 auto)")
    ap.add_argument("--copy-probe", action="store_true", help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only time a 1 GiB copy, fill and sum (achievable HBM rates)")
    ap.add_argument("--only", choices=("both", "fp32", "fp64", "uneven48", "group"), default="both",
                    help="time one path only and print its breakdown (for profiler runs); uneven48: the 48^3 "
                         "grid of the uneven batch (307 points, FP32 + fix), eval + conserve and the VJP; "
                         "group: the uneven three-grid batch through the group graph, and each branch alone")
    a = ap.parse_args()
    if a.copy_probe:
        copy_probe()
        return
    if a.stream_probe:
        stream_probe()
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every item is independent and the box has one GPU; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1809_10186_amd as qc
    import workloads as W

    if a.only == "uneven48":
        print(json.dumps(uneven48(qc, torch, W, a.steps, a.warmup)))
        return
    if a.only == "group":
        print(json.dumps(group_uneven(qc, torch, W, reps=a.steps)))
        return

    w = W.WORKLOADS[WORKLOAD]
    N, L, B = w["N"], w["L"], w["items"]
    sph = W.sphere_rule(w["M"])
    f_np = W.mixture_for(WORKLOAD)
    f = torch.from_numpy(f_np).to("cuda")
    Q = torch.empty_like(f)
    plans = {}
    for prec in (qc.QCOLL_FP32, qc.QCOLL_FP64):
        plans[prec] = qc.Plan(N, L, w["N_rho"], sphere=sph, omega=w["omega"], svd_rank=0,
                              svd_tol=w["svd_tol"], precision=prec)
        if prec == qc.QCOLL_FP32 and a.schedule:
            plans[prec].set_schedule(a.schedule)
    # schedule and items per chunk from the library's autotuner (excluded from timing)
    tuned = {}
    for prec in (qc.QCOLL_FP32, qc.QCOLL_FP64):
        if not (prec == qc.QCOLL_FP32 and a.schedule):
            tuned["fp32" if prec == qc.QCOLL_FP32 else "fp64"] = plans[prec].autotune(f, Q)
        plans[prec].workspace(B, 0)

    def step(plan):
        plan.eval(f, Q)
        plan.conserve(Q)

    def run_steps(plan, steps):
        t0 = time.perf_counter()
        for _ in range(steps):
            step(plan)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    p32, p64 = plans[qc.QCOLL_FP32], plans[qc.QCOLL_FP64]
    Nr, M = w["N_rho"], w["M"]

    def measure(plan, fp32):
        """Warm-up, a short untimed pass with every kernel role timed (the
        per-kernel breakdown), then the timed steps with hipEvents around the
        dominant kernel only (on its launch stream)."""
        for _ in range(a.warmup):
            step(plan)
        torch.cuda.synchronize()
        n_brk = min(a.steps, 5)
        qc.timing_reset()
        qc.timing_select(None)
        qc.timing_enable(True)
        run_steps(plan, n_brk)
        qc.timing_enable(False)
        kt_all = qc.timing_read()
        dominant = max(kt_all.items(), key=lambda kv: kv[1][0])[0]
        many = kt_all[dominant][1] > 4 * n_brk
        if many:
            # a dominant kernel launched many times per step (the FP64 two-pass
            # hot loop: 96 launches) would carry an event pair per launch in
            # the timed region: time the steps clean, then the same number of
            # steps again with the events for its launch duration
            dt = run_steps(plan, a.steps)
        qc.timing_reset()
        qc.timing_select(dominant)
        qc.timing_enable(True)
        dt_ev = run_steps(plan, a.steps)
        qc.timing_enable(False)
        tot_ms, launches = qc.timing_read()[dominant]
        qc.timing_select(None)
        if not many:
            dt = dt_ev
        inf = plan.info()
        npair, nv = (inf["rank"] + 1) // 2, inf["rank"]
        roof = roofline(dominant, tot_ms, launches, a.steps, B, N, Nr, M, fp32=fp32, npair=npair, nv=nv)
        passes, summ = hbm_passes(kt_all, n_brk, fp32, B, N, Nr, M, npair, nv)
        return dt / a.steps * 1e3, roof, passes, summ

    ms32 = ms64 = None
    roof = roof64 = passes32 = passes64 = summ32 = summ64 = None
    if a.only in ("both", "fp32"):
        ms32, roof, passes32, summ32 = measure(p32, True)
    if a.only in ("both", "fp64"):
        ms64, roof64, passes64, summ64 = measure(p64, False)
    if a.only != "both":
        print(json.dumps({"only": a.only, "ms_per_step": ms32 or ms64, "roofline": roof or roof64,
                          "hbm_passes": passes32 or passes64, "hbm_passes_total": summ32 or summ64}))
        return

    info = p32.info()

    extra = None if a.no_extras else extras(qc, torch, W)

    acc = None
    cpu = None
    fft_ctx = None
    if not a.no_acc or not a.no_cpu:
        # about 10-20 s of oracle work: 12 items per host core (one item ~1 s), at most the batch
        n_cpu = a.cpu_items or min(12 * min(os.cpu_count() or 1, 16), B)
        prm = dict(N=N, L=L, N_rho=Nr, M=M, omega=w["omega"], svd_tol=w["svd_tol"])
        cpu, ref = cpu_baseline(f_np[:max(n_cpu, 1)], prm, n_cpu) if not a.no_cpu else (None, {})
        fft_ctx = cpu_fft_context(f_np, prm, ref) if ref else None
        if not a.no_acc:
            from oracle import spectral
            from oracle import conserve as oc
            # every item the CPU leg computed, else three sampled items
            sample = sorted(ref) if ref else [0, B // 2, B - 1]
            P = spectral.Params(N, L, Nr, sph[0], sph[1], w["omega"], svd_tol=w["svd_tol"])
            refs = {}
            for i in sample:
                if i in ref:
                    refs[i] = ref[i]
                else:
                    refs[i] = oc.project(spectral.collide(f_np[i], P)[None], N, L)[0][0]
            acc = {}
            for prec, tag in ((qc.QCOLL_FP32, "fp32_fix"), (qc.QCOLL_FP64, "fp64")):
                step(plans[prec])
                Qh = Q.cpu().numpy()
                errs = [np.abs(Qh[i] - refs[i]).max() / np.abs(refs[i]).max() for i in sample]
                acc[tag] = float(max(errs))
                acc[tag + "_conservation_residual"] = float(oc.conservation_residual(Qh, N, L).max())
            acc["items"] = len(sample)

    out = {
        "metric": METRIC,
        "value": round(B / (ms32 * 1e-3), 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (gain transforms and products; f64 spectrum, loss, assembly, conservation)",
        "data": "synthetic",
        "config": {"workload": "1D DG batch: 64 elements x 3 Gauss points = 192 points, N=32^3, L=6, "
                               "M=12, N_rho=16, VHS omega=0.81, SVD rank at 1e-8",
                   "batch": B, "svd_rank": info["rank"], "step": "qcoll_eval + qcoll_conserve",
                   "autotuned_schedule_chunk": tuned},
        "fp64": {"value": round(B / (ms64 * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms64, 4)},
        "rel_linf_err": acc,
        "roofline": roof,
        "hbm_passes": {"fp32": passes32, "fp32_total": summ32, "fp64": passes64, "fp64_total": summ64},
        "roofline_fp64": roof64,
        "secondary": extra,
        "cpu_baseline": cpu,
        "cpu_fft_context": fft_ctx,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
