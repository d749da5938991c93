"""Fan the FP64 oracle out over host processes (test infrastructure only).

The full-size parity tests compare many items against the oracle; one item at
32^3 takes about a second on one core, at 48^3 several seconds.  Each worker
builds the oracle's kernel tables once per parameter set and evaluates whole
items, with BLAS threads pinned to one per process.  Nothing here computes any
part of the method: it only calls ``oracle``.
"""
import multiprocessing as mp
import os

import numpy as np

_PARAMS = {}


def workers():
    """Processes to use: the host's cores, at most 16 (the GPU machine's CPU share)."""
    return max(1, min(os.cpu_count() or 1, 16))


def _params(key):
    P = _PARAMS.get(key)
    if P is None:
        import workloads as W
        from oracle import spectral
        N, L, N_rho, M, omega, prefactor, svd_tol, nyquist, vss_alpha = key
        pts, w = W.sphere_rule(M)
        P = spectral.Params(N, L, N_rho, pts, w, omega, prefactor=prefactor, svd_tol=svd_tol, nyquist=nyquist,
                            vss_alpha=vss_alpha)
        _PARAMS[key] = P
    return P


def _key(N, L, N_rho, M, omega, prefactor=None, svd_tol=None, nyquist="symmetric", vss_alpha=1.0):
    return (int(N), float(L), int(N_rho), int(M), float(omega), prefactor, svd_tol, nyquist, float(vss_alpha))


def _collide(args):
    key, f, project = args
    from oracle import spectral
    from oracle import conserve as oc
    P = _params(key)
    Q = spectral.collide(f, P)
    if project:
        Q = oc.project(Q[None], P.N, P.L)[0][0]
    return Q


def _vjp(args):
    key, f, g, project = args
    from oracle import adjoint
    from oracle import conserve as oc
    P = _params(key)
    if project:
        g = oc.project(g[None], P.N, P.L)[0][0]
    return adjoint.vjp_f(f, g, P)


def _map(fn, jobs):
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    n = min(workers(), len(jobs))
    if n <= 1:
        return [fn(j) for j in jobs]
    with mp.get_context("spawn").Pool(n) as pool:
        return pool.map(fn, jobs, chunksize=1)


def collide_many(f, project=False, **prm):
    """Oracle Q(f, f) of every item of f [B, N, N, N] (projected onto the
    collision invariants if project): [B, N, N, N]."""
    key = _key(**prm)
    return np.stack(_map(_collide, [(key, np.ascontiguousarray(x), project) for x in f]))


def vjp_many(f, g, project=False, **prm):
    """Oracle J_f^T g of every item (through the projection if project)."""
    key = _key(**prm)
    return np.stack(_map(_vjp, [(key, np.ascontiguousarray(a), np.ascontiguousarray(b), project)
                                for a, b in zip(f, g)]))
