"""GPU parity of the 1-D RKDG driver (qcoll_dg1d_*) against the oracle's
plain implementation of the same semi-discrete scheme (Section 3)."""
import numpy as np
import pytest

import workloads as W
from oracle import rkdg, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1809_10186_amd as qc  # noqa: E402

N, L, NR, M = 8, 5.0, 4, 6


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def state(x, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    F = np.empty(x.shape + (N, N, N))
    for i in range(x.shape[0]):
        for m in range(x.shape[1]):
            xx = x[i, m]
            F[i, m] = W.maxwellian(N, L, 1.0 + 0.3 * np.sin(2.0 * xx), np.array([0.2 * np.cos(xx), 0.1, 0.0]),
                                   0.9 + 0.2 * xx) * (1.0 + 0.01 * rng.random((N, N, N)))
    return F


def setups():
    return {
        "walls": (rkdg.Bc("wall", u=(0.0, -0.3, 0.0), T=0.85), rkdg.Bc("wall", u=(0.0, 0.3, 0.1), T=1.15),
                  qc.Bc("wall", u=(0.0, -0.3, 0.0), T=0.85), qc.Bc("wall", u=(0.0, 0.3, 0.1), T=1.15)),
        "inflow": (rkdg.Bc("inflow", n=1.1, u=(0.4, 0.0, 0.0), T=1.2), rkdg.Bc("inflow", n=0.9, u=(-0.2, 0.0, 0.0), T=0.8),
                   qc.Bc("inflow", n=1.1, u=(0.4, 0.0, 0.0), T=1.2), qc.Bc("inflow", n=0.9, u=(-0.2, 0.0, 0.0), T=0.8)),
        "periodic": (rkdg.Bc(), rkdg.Bc(), qc.Bc(), qc.Bc()),
    }


def make(bcs, coll, inv_kn, precision=qc.QCOLL_FP64, P=2, faces=(0.0, 0.15, 0.55, 1.0)):
    ol, orr, gl, gr = bcs
    sph = W.sphere_rule(M)
    prm = spectral.Params(N, L, NR, sph[0], sph[1], 0.81)
    od = rkdg.Dg1d(np.array(faces), P, prm, inv_kn, ol, orr, coll=coll)
    plan = qc.Plan(N, L, NR, sphere=sph, omega=0.81, precision=precision)
    gd = qc.Dg1d(plan, np.array(faces), P, inv_kn, gl, gr, coll_form=1 if coll == "exact" else 0)
    return od, gd, plan


@pytest.mark.parametrize("bc", ["walls", "inflow", "periodic"])
@pytest.mark.parametrize("coll", ["collocation", "exact"])
def test_dg1d_rhs_matches_oracle(bc, coll):
    od, gd, plan = make(setups()[bc], coll, 0.7)
    assert np.allclose(gd.nodes(), od.nodes_x(), rtol=0, atol=1e-15)
    F = state(od.nodes_x(), 1)
    ref = od.rhs(F)
    R = gd.rhs(gpu(F)).cpu().numpy()
    err = np.abs(R - ref).max() / np.abs(ref).max()
    print(f"dg1d rhs {bc} {coll}: rel {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("rk", [1, 2, 3])
def test_dg1d_step_matches_oracle_and_conserves_mass(rk):
    od, gd, plan = make(setups()["walls"], "collocation", 0.5)
    F = state(od.nodes_x(), 2)
    ref = od.step(F, 0.004, rk=rk)
    Fg = gpu(F)
    gd.step(Fg, 0.004, rk=rk)
    G = Fg.cpu().numpy()
    err = np.abs(G - ref).max() / np.abs(ref).max()
    print(f"dg1d step rk{rk}: rel {err:.3e}", flush=True)
    assert err <= 1e-12
    m0 = od.total_mass(F)
    assert abs(od.total_mass(G) - m0) <= 1e-12 * m0


def test_dg1d_fp32_collision():
    od, gd, plan = make(setups()["walls"], "exact", 0.7, precision=qc.QCOLL_FP32)
    F = state(od.nodes_x(), 3)
    ref = od.rhs(F)
    R = gd.rhs(gpu(F)).cpu().numpy()
    err = np.abs(R - ref).max() / np.abs(ref).max()
    print(f"dg1d rhs FP32 collision: rel {err:.3e}", flush=True)
    assert err <= 2e-5


def test_dg1d_free_streaming_and_refusals():
    od, gd, plan = make(setups()["periodic"], "collocation", 0.0, P=3, faces=np.linspace(0, 1, 6))
    F = state(od.nodes_x(), 4)
    Fg = gpu(F)
    ref = F
    for _ in range(3):
        ref = od.step(ref, 0.01, rk=3)
        gd.step(Fg, 0.01, rk=3)
    assert np.abs(Fg.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(qc.QcollError):
        qc.Dg1d(plan, np.array([0.0, 1.0, 0.5]), 2, 1.0)          # faces not increasing
    with pytest.raises(qc.QcollError):
        qc.Dg1d(plan, np.array([0.0, 1.0]), 2, 1.0, qc.Bc("wall"), qc.Bc("periodic"))
    with pytest.raises(qc.QcollError):
        gd.step(Fg, 0.01, rk=4)


def fourier_faces(n_half=5, ratio=1.23):
    """Element faces on [0, 1] refined geometrically towards both walls."""
    h = ratio ** np.arange(n_half)
    h = 0.5 * h / h.sum()
    left = np.concatenate([[0.0], np.cumsum(h)])
    return np.concatenate([left, 1.0 - left[::-1][1:]])


def test_dg1d_fourier_heat_transfer_qualitative():
    """Fourier heat transfer between walls at rest at 263 K and 283 K (T0 = 273 K),
    Maxwell molecules, Kn (Cercignani) 1.582 -> 1/Kn_Bird = (pi/2)/1.582, 10
    elements of order 2 refined towards the walls, [-5.09, 5.09]^3 with 16^3
    points and M = 6 (a coarser velocity grid than the paper's 24^3).  Only
    qualitative checks are possible without the DSMC data: near steady state the
    temperature rises monotonically from the cold to the hot wall with jumps at
    both walls, the density falls, the heat flux is negative and nearly uniform,
    there is no net mass flow, and mass is conserved."""
    Nv, Lv = 16, 5.09
    Tl, Tr = 263.0 / 273.0, 283.0 / 273.0
    faces = fourier_faces()
    plan = qc.Plan(Nv, Lv, 8, sphere=None, omega=1.0, precision=qc.QCOLL_FP32)
    inv_kn = (np.pi / 2.0) / 1.582
    d = qc.Dg1d(plan, faces, 2, inv_kn, qc.Bc("wall", T=Tl), qc.Bc("wall", T=Tr))
    x = d.nodes()
    M0 = W.maxwellian(Nv, Lv, 1.0, np.zeros(3), 1.0)
    F = gpu(np.broadcast_to(M0, x.shape + M0.shape).copy())
    dc3 = (2 * Lv / Nv) ** 3
    J = 0.5 * np.diff(faces)
    wg = np.polynomial.legendre.leggauss(3)[1]
    mass = lambda G: float(np.sum(J[:, None] * wg[None, :] * G.sum(dim=(2, 3, 4)).cpu().numpy() * dc3))
    m0 = mass(F)
    for _ in range(2500):
        d.step(F, 0.002, rk=2)
    mom = plan.moments(F.reshape(-1, Nv, Nv, Nv)).cpu().numpy().reshape(x.shape + (14,))
    n, ux, T, qx = mom[..., 0].ravel(), mom[..., 1].ravel(), mom[..., 4].ravel(), mom[..., 11].ravel()
    print("T", np.round(T, 4), "\nn", np.round(n, 4), "\nqx", np.round(qx, 5), flush=True)
    assert abs(mass(F) - m0) <= 1e-10 * m0
    assert np.all(np.diff(T) > 0) and Tl < T[0] and T[-1] < Tr
    assert np.all(np.diff(n) < 0)
    assert np.all(qx < 0) and (qx.max() - qx.min()) < 0.1 * abs(qx.mean())
    assert np.abs(ux).max() < 1e-3
