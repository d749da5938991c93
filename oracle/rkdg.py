"""1-D RKDG transport of the discrete-velocity Boltzmann system, FP64 (test
infrastructure: the slow, plain reference of the GPU driver).

Follows Section 3 in the paper's order:

* Physical space (Section 3.2): elements [x_i, x_{i+1}], Lagrange nodal basis
  on the K = P+1 Gauss-Legendre nodes of the reference element, x = x_c + J xi
  with J = h/2.  Mass matrix M_ml = J w_m delta_ml (the K-point rule is exact
  for degree 2P); stiffness S_ml = int phi_l dphi_m/dx dx = w_l phi_m'(xi_l).
  Weak form per element and velocity point c^j (1-D: only c_x = c_1 moves f):
    J w_m dF_m/dt = c_x sum_l S_ml F_l - [phi_m(1) c_x f*_R - phi_m(-1) c_x f*_L]
                    + (1/Kn) C_m,
  with the upwind flux f* (interior trace when c.n >= 0, exterior otherwise) and
  the collision term C_m = sum_{l1,l2} H_{m l1 l2} Q(F_l1, F_l2).
* Collision term (Section 3.3.1): ``coll="exact"`` uses the exact triple tensor
  H = J H_ref through its eigen factors (oracle.dg); ``coll="collocation"``
  uses H from the K-point rule itself, H_{m l1 l2} = J w_m delta delta, so that
  C_m = J w_m Q(F_m).  Optionally each Q is conservation-projected.
* Velocity space (Section 3.3): the N^3 cell-centred grid; Q from
  oracle.spectral.
* Time (Section 3.4): SSP-RK2 and SSP-RK3 (and forward Euler).
* Boundaries (Section 3.5): periodic; fully diffuse wall at (u_w, T_w), where
  for (c - u_w).n < 0 the exterior state is n_w exp(-|c - u_w|^2 / T_w) with
  n_w from zero net mass flux through the wall (discrete sums over the grid);
  inflow Maxwellian n (pi T)^{-3/2} exp(-|c - u|^2 / T) for c.n < 0.
"""
import numpy as np

from . import conserve as oc
from . import dg, spectral
from . import quadrature as qd


class Bc:
    def __init__(self, kind="periodic", n=1.0, u=(0.0, 0.0, 0.0), T=1.0):
        assert kind in ("periodic", "wall", "inflow")
        self.kind, self.n, self.u, self.T = kind, float(n), np.asarray(u, dtype=float), float(T)


class Dg1d:
    def __init__(self, faces, P, params, inv_kn, left, right, coll="collocation", conserve=True):
        self.faces = np.asarray(faces, dtype=float)
        self.I = len(self.faces) - 1
        self.P, self.K = int(P), int(P) + 1
        self.prm = params
        self.inv_kn = float(inv_kn)
        self.left, self.right = left, right
        self.coll, self.conserve = coll, conserve
        assert (left.kind == "periodic") == (right.kind == "periodic")
        N, L = params.N, params.L
        self.xi, self.w = dg.gauss_nodes(self.P)
        nodes = self.xi
        self.phiL = dg.lagrange(nodes, -1.0)[:, 0]          # phi_l(-1)
        self.phiR = dg.lagrange(nodes, 1.0)[:, 0]           # phi_l(+1)
        # derivative of each Lagrange polynomial at the nodes: dphi[l, q] = phi_l'(xi_q)
        self.dphi = np.zeros((self.K, self.K))
        for l in range(self.K):
            c = np.polynomial.polynomial.polyfromroots(np.delete(nodes, l))
            c = c / np.polynomial.polynomial.polyval(nodes[l], c)
            self.dphi[l] = np.polynomial.polynomial.polyval(nodes, np.polynomial.polynomial.polyder(c))
        # S_ml = sum_q w_q phi_l(xi_q) phi_m'(xi_q) = w_l phi_m'(xi_l)
        self.S = (self.w[None, :] * self.dphi)              # [m, l] = w_l dphi[m, l]
        self.J = 0.5 * np.diff(self.faces)
        self.xc = 0.5 * (self.faces[1:] + self.faces[:-1])
        c = qd.grid(N, L)
        c1, c2, c3 = np.meshgrid(c, c, c, indexing="ij")
        self.cv = np.stack([c1, c2, c3])                    # [3, N, N, N]
        if coll == "exact":
            self.T, self.Wf, _ = dg.eigen_factors(dg.triple_tensor_1d(self.P))
        self._walls = {}
        for side, bc, nrm in (("L", left, -1.0), ("R", right, 1.0)):
            if bc.kind == "wall":
                cn = (self.cv[0] - bc.u[0]) * nrm           # (c - u_w).n (the wall normal is +-x)
                fw = np.exp(-np.sum((self.cv - bc.u[:, None, None, None]) ** 2, axis=0) / bc.T)
                self._walls[side] = (cn, fw, np.sum(np.where(cn < 0, cn * fw, 0.0)))
            elif bc.kind == "inflow":
                fin = bc.n / (np.pi * bc.T) ** 1.5 * np.exp(
                    -np.sum((self.cv - bc.u[:, None, None, None]) ** 2, axis=0) / bc.T)
                self._walls[side] = (None, fin, None)

    def nodes_x(self):
        return self.xc[:, None] + self.J[:, None] * self.xi[None, :]

    def wall_density(self, side, trace):
        cn, fw, den = self._walls[side]
        num = np.sum(np.where(cn >= 0, cn * trace, 0.0))
        return -num / den

    def _exterior(self, side, trace):
        bc = self.left if side == "L" else self.right
        if bc.kind == "wall":
            return self.wall_density(side, trace) * self._walls[side][1]
        return self._walls[side][1]                          # inflow

    def transport(self, F):
        """c_x-part of the weak form divided by the mass matrix: [I, K, N, N, N]."""
        I, K = self.I, self.K
        cx = self.cv[0]
        fR = np.einsum("l,ilxyz->ixyz", self.phiR, F)       # traces at xi = +1
        fL = np.einsum("l,ilxyz->ixyz", self.phiL, F)       # traces at xi = -1
        # right face of element i: interior fR[i] if c_x >= 0, else exterior fL[i+1]
        ext_R = np.empty_like(fR)
        ext_L = np.empty_like(fL)
        ext_R[:-1] = fL[1:]
        ext_L[1:] = fR[:-1]
        if self.left.kind == "periodic":
            ext_R[-1] = fL[0]
            ext_L[0] = fR[-1]
        else:
            ext_L[0] = self._exterior("L", fL[0])
            ext_R[-1] = self._exterior("R", fR[-1])
        fsR = np.where(cx >= 0, fR, ext_R)
        fsL = np.where(cx > 0, ext_L, fL)                   # left face: normal -x, upwind is the left side if c_x > 0
        R = np.einsum("ml,ilxyz->imxyz", self.S, F) * cx
        R -= self.phiR[None, :, None, None, None] * (cx * fsR)[:, None]
        R += self.phiL[None, :, None, None, None] * (cx * fsL)[:, None]
        return R / (self.J[:, None, None, None, None] * self.w[None, :, None, None, None])

    def _Q(self, f):
        q = spectral.collide(f, self.prm)
        if self.conserve:
            q = oc.project(q[None], self.prm.N, self.prm.L)[0][0]
        return q

    def collision(self, F):
        """(1/Kn) C_m / (J w_m): [I, K, N, N, N]."""
        out = np.zeros_like(F)
        if self.inv_kn == 0.0:
            return out
        for i in range(self.I):
            if self.coll == "collocation":
                for m in range(self.K):
                    out[i, m] = self._Q(F[i, m])
            else:
                h = np.einsum("rk,kxyz->rxyz", self.T, F[i])
                Qh = np.array([self._Q(x) for x in h])
                out[i] = np.einsum("kr,rxyz->kxyz", self.Wf, Qh) / self.w[:, None, None, None]
        return self.inv_kn * out

    def rhs(self, F):
        return self.transport(F) + self.collision(F)

    def step(self, F, dt, rk=3):
        L = self.rhs
        if rk == 1:
            return F + dt * L(F)
        v1 = F + dt * L(F)
        if rk == 2:
            return 0.5 * F + 0.5 * v1 + 0.5 * dt * L(v1)
        v2 = 0.75 * F + 0.25 * v1 + 0.25 * dt * L(v1)
        return F / 3.0 + 2.0 / 3.0 * v2 + 2.0 / 3.0 * dt * L(v2)

    def total_mass(self, F):
        """sum over elements and nodes of J w_m n(F) (mid-point rule in velocity)."""
        dc3 = (2.0 * self.prm.L / self.prm.N) ** 3
        n = F.sum(axis=(2, 3, 4)) * dc3
        return float(np.sum(self.J[:, None] * self.w[None, :] * n))
