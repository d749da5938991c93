"""The 64^3 grid: parity against the oracle in both precisions, and the paper's
Table 1 rows at N = 48 and 64 (BKW exact operator, Section 4.3) reproduced by
the FP64 GPU path."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import bkw, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", [qc.QCOLL_FP64, qc.QCOLL_FP32])
def test_grid64_matches_oracle(precision):
    N, L, Nr, M = 64, 9.0, 2, 6
    print(f"case N=64 prec={precision}", flush=True)
    sph = W.sphere_rule(M)
    f = W.maxwellian_mixture(1, N, L, 6400, T_range=(2.5, 3.5), u_max=2.3)
    P = spectral.Params(N, L, Nr, sph[0], sph[1], 0.81)
    plan = qc.Plan(N, L, Nr, sphere=sph, omega=0.81, precision=precision)
    Q = plan.eval(gpu(f)).cpu().numpy()[0]
    ref = spectral.collide(f[0], P)
    err = np.abs(Q - ref).max() / np.abs(ref).max()
    print(f"N=64 prec={precision} rel {err:.3e}", flush=True)
    assert err <= (1e-12 if precision == qc.QCOLL_FP64 else 2e-5)
    with pytest.raises(qc.QcollError) as e:
        plan.vjp(gpu(f), gpu(f))
    assert e.value.code == 2


def _table1():
    rows = []
    for line in open(os.path.join(HERE, "golden", "bkw_table1.txt")):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            rows.append((int(v[0]), int(v[1]), [float(x) for x in v[2:]]))
    return rows


@pytest.mark.parametrize("N,N_r,errs", [r for r in _table1() if r[0] >= 48])
def test_bkw_table1_large_grids(N, N_r, errs):
    """Error of the FP64 GPU Q against the exact BKW operator on [-6.62, 6.62]^3,
    M = 6, B = 1/(4 pi), for the Table 1 rows the CPU oracle is too slow for.
    As in the oracle's pin of the N <= 32 rows, the paper's design is the same
    icosahedral rule up to an unknown rotation: agreement within a factor 1.5."""
    L = 6.62
    plan = qc.Plan(N, L, N_r, sphere=None, omega=1.0, prefactor=1.0 / (4 * math.pi), precision=qc.QCOLL_FP64)
    f = np.stack([W.bkw(N, L, t0) for t0 in (5.5, 6.5, 10.0)])
    Q = plan.eval(gpu(f)).cpu().numpy()
    got = [float(np.abs(Q[i] - bkw.Q_exact(N, L, t0)).max()) for i, t0 in enumerate((5.5, 6.5, 10.0))]
    print(f"Table 1 N={N} N_r={N_r}: {['%.3g' % g for g in got]} (paper {errs})", flush=True)
    for g, ref in zip(got, errs):
        assert ref / 1.5 < g < ref * 1.5
    plan.close()
