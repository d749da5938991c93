"""Build the equal-weight half-sphere quadrature rules used as method inputs.

The fast spectral method integrates over the half sphere with a spherical
design (Appendix, quadrature form of the kernel modes and the paragraph after
it).  The paper uses Womersley's antipodal designs, whose point files are not
available here, so the rules are rebuilt:

* M = 6: one vertex per antipodal pair of the regular icosahedron (closed form,
  an antipodal 5-design).
* M = 12, 16: antipodal point sets of 2M points on the full sphere found by
  solving sum_i Y_lm(x_i) = 0 for every even l < t by nonlinear least
  squares (odd degrees vanish by antipodal symmetry), so the result is an
  antipodal t-design; among seeded restarts the one with the smallest
  residual at the next even degrees is kept.  M = 12 reaches t = 5 (24
  antipodal points admit no 7-design of this kind in our search), M = 16
  reaches t = 7 like Womersley's 32-point symmetric design.  Seeds are
  fixed, so the output is deterministic.

The half-sphere representative of each antipodal pair is the one with z > 0
(ties: y > 0, then x > 0).  Weights are 2*pi/M each, summing to the area of
the half sphere.

Run:  python workloads/make_sphere_designs.py   (writes workloads/sphere/*.txt)
"""
import os
import numpy as np
from numpy.polynomial import legendre
from scipy.optimize import least_squares
from scipy.special import sph_harm_y

HERE = os.path.dirname(os.path.abspath(__file__))


def icosahedron_half():
    phi = (1.0 + np.sqrt(5.0)) / 2.0
    v = []
    for a in (1.0, -1.0):
        for b in (phi, -phi):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(v)
    v /= np.linalg.norm(v, axis=1)[:, None]
    return canonical_half(v)


def canonical_half(v):
    """Keep one point of each antipodal pair: z > 0, then y > 0, then x > 0."""
    out = []
    for x in v:
        key = None
        for c in (x[2], x[1], x[0]):
            if abs(c) > 1e-12:
                key = c
                break
        if key > 0:
            out.append(x)
    out = np.array(out)
    order = np.lexsort((out[:, 0], out[:, 1], -out[:, 2]))
    return out[order]


def _to_xyz(ang):
    th, ph = ang[0::2], ang[1::2]
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def _residual(ang, degs, M):
    """Real and imaginary parts of sum_i Y_lm(x_i) over the antipodal set, even l in degs."""
    th = ang[0::2]
    ph = ang[1::2]
    r = []
    for l in degs:
        for m in range(0, l + 1):
            y = sph_harm_y(l, m, th, ph)
            s = 2.0 * y.sum()          # +x and -x contribute equally for even l
            r.append(s.real)
            if m > 0:
                r.append(s.imag)
    return np.array(r)


def optimise(M, t, seed, t_soft=None, restarts=60):
    """Antipodal design of 2M points, exact to degree t; if t_soft is given,
    the even degrees in (t, t_soft) are minimised as a soft second stage."""
    rng = np.random.default_rng(seed)
    hard = list(range(2, t, 2))
    soft = list(range(t + 1, t_soft, 2)) if t_soft else []
    best = None
    for _ in range(restarts):
        z = rng.normal(size=(M, 3))
        z /= np.linalg.norm(z, axis=1)[:, None]
        ang = np.empty(2 * M)
        ang[0::2] = np.arccos(np.clip(z[:, 2], -1, 1))
        ang[1::2] = np.arctan2(z[:, 1], z[:, 0])
        if soft:
            res = least_squares(lambda a: _residual(a, hard + soft, M), ang, xtol=1e-15, ftol=1e-15, gtol=1e-15)
            ang = res.x
        res = least_squares(lambda a: _residual(a, hard, M), ang, xtol=1e-15, ftol=1e-15, gtol=1e-15)
        hard_norm = np.linalg.norm(_residual(res.x, hard, M))
        soft_norm = np.linalg.norm(_residual(res.x, soft, M)) if soft else 0.0
        key = (hard_norm > 1e-13, soft_norm, hard_norm)
        if best is None or key < best[0]:
            best = (key, res.x)
    pts = _to_xyz(best[1])
    return canonical_half(np.concatenate([pts, -pts])), best[0]


def design_degree(points, tmax=21):
    """Largest t such that every spherical polynomial of degree <= t is exact."""
    t = 1
    for l in range(2, tmax + 1, 2):
        x = np.concatenate([points, -points])
        g = np.clip(x @ x.T, -1.0, 1.0)
        c = np.zeros(l + 1)
        c[l] = 1.0
        if abs(legendre.legval(g, c).sum()) > 1e-10 * len(x):
            return t
        t = l + 1
    return t


def write(path, pts, M, note):
    w = 2.0 * np.pi / M
    with open(path, "w") as fh:
        fh.write(f"# {note}\n# x y z weight   (M = {M}, weights sum to 2*pi)\n")
        for p in pts:
            fh.write(f"{p[0]:.17e} {p[1]:.17e} {p[2]:.17e} {w:.17e}\n")


def main():
    os.makedirs(os.path.join(HERE, "sphere"), exist_ok=True)
    ico = icosahedron_half()
    write(os.path.join(HERE, "sphere", "half_M6.txt"), ico, 6,
          f"icosahedron, one vertex per antipodal pair; design degree {design_degree(ico)}")
    for M, t, t_soft, seed in ((12, 5, 9, 12), (16, 7, 11, 16)):
        pts, key = optimise(M, t, seed, t_soft)
        deg = design_degree(pts)
        write(os.path.join(HERE, "sphere", f"half_M{M}.txt"), pts, M,
              f"antipodal design, exact to degree {deg}, degree-{t + 1}..{t_soft - 1} residual {key[1]:.3e} (seed {seed})")
        print(M, "degree", deg, "soft residual", key[1], "hard residual", key[2])


if __name__ == "__main__":
    main()
