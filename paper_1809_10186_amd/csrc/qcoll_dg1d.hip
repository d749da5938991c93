// 1-D RKDG driver (Section 3): nodal DG in x on K = P+1 Gauss-Legendre nodes
// per element, upwind flux (Section 3.2), the weak-form collision term through
// the plan (Section 3.3.1), SSP-RK2/RK3 (Section 3.4), periodic / fully diffuse
// wall / inflow ends (Section 3.5).
//
// State F [I][K][N^3] FP64.  With the K-point rule the mass matrix is
// J w_m delta_ml, so per node
//   dF_m/dt = (c_x sum_l S_ml F_l - phi_m(1) c_x f*_R + phi_m(-1) c_x f*_L) / (J w_m)
//             + inv_kn C_m / (J w_m),
// S_ml = w_l phi_m'(xi_l).  The transport kernel takes one lane per (element,
// velocity point) and all K nodes of it, reading the neighbours' traces for
// the upwind fluxes; the wall densities come from a fixed-order reduction of
// the outgoing flux, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "qcoll_internal.h"

namespace qcoll {
namespace {

constexpr int kMaxK = 8;

// per-end data of the boundary kernels
struct EndDev {
  int kind;        // qcoll_bc_kind
  double ux;       // x-velocity of the wall (for (c - u).n)
  double nrm;      // outward normal: -1 left, +1 right
  double den;      // sum over (c - u).n < 0 of (c - u).n f_w (walls)
  const double *fb;  // [N^3] wall Maxwellian exp(-|c-u|^2/T) or inflow Maxwellian
};

struct Dg1dArgs {
  const double *F;
  double *R;
  const double *C;      // collision term per node (scaled by cscale), or null
  double cscale;
  const double *J;      // [I]
  const double *tab;    // w[K], S[K][K], phiL[K], phiR[K]
  double *nw;           // [2] wall densities
  EndDev end[2];
  int I, K, N;
  long n3;
  double L;
  int periodic;
};

__device__ __forceinline__ double c1_of(long j, int N, double L) {
  const int j1 = int(j / (long(N) * N));
  return -L + (j1 + 0.5) * (2.0 * L / N);
}

// wall densities: block 0 left, block 1 right; n_w = -sum_{(c-u).n >= 0} (c-u).n f_trace / den
__global__ __launch_bounds__(1024) void k_dg1d_wall(Dg1dArgs a) {
  const int side = blockIdx.x;
  const EndDev &E = a.end[side];
  if (E.kind != QCOLL_BC_WALL) return;   // uniform per block
  const int e = side == 0 ? 0 : a.I - 1;
  const double *phi = a.tab + a.K + a.K * a.K + (side == 0 ? 0 : a.K);
  double s = 0.0;
  for (long j = threadIdx.x; j < a.n3; j += 1024) {
    const double cn = (c1_of(j, a.N, a.L) - E.ux) * E.nrm;
    if (cn >= 0.0) {
      double tr = 0.0;
      for (int l = 0; l < a.K; ++l) tr += phi[l] * a.F[(long(e) * a.K + l) * a.n3 + j];
      s += cn * tr;
    }
  }
  __shared__ double red[1024];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.nw[side] = -red[0] / E.den;
}

// exterior state of an end for velocity point j (incoming side of the face)
__device__ __forceinline__ double ext_state(const Dg1dArgs &a, int side, long j) {
  const EndDev &E = a.end[side];
  return E.kind == QCOLL_BC_WALL ? a.nw[side] * E.fb[j] : E.fb[j];
}

__global__ __launch_bounds__(256) void k_dg1d_rhs(Dg1dArgs a) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(a.I) * a.n3) return;
  const int e = int(t / a.n3);
  const long j = t % a.n3;
  const int K = a.K;
  const double *w = a.tab, *S = a.tab + K, *phiL = a.tab + K + K * K, *phiR = phiL + K;
  const double cx = c1_of(j, a.N, a.L);
  auto trace = [&](int el, const double *phi) {
    double s = 0.0;
    for (int l = 0; l < K; ++l) s += phi[l] * a.F[(long(el) * K + l) * a.n3 + j];
    return s;
  };
  double f[kMaxK];
  for (int l = 0; l < K; ++l) f[l] = a.F[(long(e) * K + l) * a.n3 + j];
  double fR = 0.0, fL = 0.0;
  for (int l = 0; l < K; ++l) {
    fR += phiR[l] * f[l];
    fL += phiL[l] * f[l];
  }
  // right face (normal +x): interior if c_x >= 0
  double fsR = fR;
  if (cx < 0.0) {
    if (e + 1 < a.I) fsR = trace(e + 1, phiL);
    else fsR = a.periodic ? trace(0, phiL) : ext_state(a, 1, j);
  }
  // left face (normal -x): interior if c_x <= 0
  double fsL = fL;
  if (cx > 0.0) {
    if (e > 0) fsL = trace(e - 1, phiR);
    else fsL = a.periodic ? trace(a.I - 1, phiR) : ext_state(a, 0, j);
  }
  const double invJ = 1.0 / a.J[e];
  for (int m = 0; m < K; ++m) {
    double v = 0.0;
    for (int l = 0; l < K; ++l) v += S[m * K + l] * f[l];
    double r = (cx * v - phiR[m] * cx * fsR + phiL[m] * cx * fsL) * invJ / w[m];
    const long o = (long(e) * K + m) * a.n3 + j;
    if (a.C) r += a.cscale * a.C[o];
    a.R[o] = r;
  }
}

// out = x a + y b + z c (elementwise; out may alias x)
__global__ __launch_bounds__(256) void k_axpby3(double *out, const double *x, double a, const double *y, double b,
                                                 const double *z, double c, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = a * x[i];
  if (y) v += b * y[i];
  if (z) v += c * z[i];
  out[i] = v;
}

// ---------------------------------------------------------------------------
// host tables
void lagrange_at(const std::vector<double> &xs, double x, std::vector<double> &out) {
  const int K = int(xs.size());
  out.assign(K, 1.0);
  for (int l = 0; l < K; ++l)
    for (int k = 0; k < K; ++k)
      if (k != l) out[l] *= (x - xs[k]) / (xs[l] - xs[k]);
}

// phi_l'(xs[q]) for the Lagrange basis on xs
double lagrange_deriv(const std::vector<double> &xs, int l, int q) {
  const int K = int(xs.size());
  if (q == l) {
    double s = 0.0;
    for (int k = 0; k < K; ++k)
      if (k != l) s += 1.0 / (xs[l] - xs[k]);
    return s;
  }
  double num = 1.0, den = 1.0;
  for (int k = 0; k < K; ++k) {
    if (k != l) den *= xs[l] - xs[k];
    if (k != l && k != q) num *= xs[q] - xs[k];
  }
  return num / den;
}

// cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major);
// on return A holds the eigenvalues on its diagonal and V the eigenvectors in columns
void sym_eigen(std::vector<double> &A, int n, std::vector<double> &V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[size_t(i) * n + j] * A[size_t(i) * n + j];
        if (i != j) off += A[size_t(i) * n + j] * A[size_t(i) * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[size_t(p) * n + q];
        if (apq == 0.0) continue;
        const double app = A[size_t(p) * n + p], aqq = A[size_t(q) * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // A <- A J (columns p, q)
          const double akp = A[size_t(k) * n + p], akq = A[size_t(k) * n + q];
          A[size_t(k) * n + p] = c * akp - s * akq;
          A[size_t(k) * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // A <- J^T A (rows p, q)
          const double apk = A[size_t(p) * n + k], aqk = A[size_t(q) * n + k];
          A[size_t(p) * n + k] = c * apk - s * aqk;
          A[size_t(q) * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {   // V <- V J
          const double vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
          V[size_t(k) * n + p] = c * vkp - s * vkq;
          V[size_t(k) * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

template <class T>
qcoll_status upload_vec(const std::vector<T> &h, T **d) {
  *d = nullptr;
  if (h.empty()) return QCOLL_OK;
  if (hipMalloc(d, h.size() * sizeof(T)) != hipSuccess) {
    *d = nullptr;
    set_error("hipMalloc failed for a driver table");
    return QCOLL_ENOMEM;
  }
  if (hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("hipMemcpy failed for a driver table");
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace qcoll

struct qcoll_dg1d_s {
  qcoll_plan plan = nullptr;
  int I = 0, K = 0, R = 0, coll_form = 0, conserve = 0;
  double inv_kn = 0.0;
  std::vector<double> faces, xnodes, wq;
  qcoll_bc ends[2];
  double den[2] = {1.0, 1.0};
  double *J = nullptr, *tab = nullptr, *T = nullptr, *W = nullptr, *fb = nullptr, *nw = nullptr;
};

namespace {

qcoll_status dfail(qcoll_status s, const char *m) {
  qcoll::set_error(m);
  return s;
}

void free_dg1d(qcoll_dg1d d) {
  (void)hipFree(d->J);
  (void)hipFree(d->tab);
  (void)hipFree(d->T);
  (void)hipFree(d->W);
  (void)hipFree(d->fb);
  (void)hipFree(d->nw);
}

bool bc_ok(const qcoll_bc &b) {
  if (b.kind == QCOLL_BC_PERIODIC) return true;
  if (b.kind != QCOLL_BC_WALL && b.kind != QCOLL_BC_INFLOW) return false;
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(b.u[d])) return false;
  if (!(b.T > 0.0) || !std::isfinite(b.T)) return false;
  if (b.kind == QCOLL_BC_INFLOW && !(b.n > 0.0 && std::isfinite(b.n))) return false;
  return true;
}

struct DgLayout {
  size_t off_c = 0, off_h = 0, off_q = 0, off_ews = 0, off_r = 0, off_v1 = 0, off_v2 = 0, total = 0;
  long items = 0;   // items of the eval (I K collocated, I R exact)
};

DgLayout dg_layout(qcoll_dg1d d, int rk) {
  DgLayout l;
  const long n3 = d->plan->p.n3();
  const size_t vol = size_t(d->I) * d->K * n3 * sizeof(double);
  size_t o = 0;
  l.off_c = o;
  o += qcoll::al256(vol);
  if (d->inv_kn > 0.0) {
    if (d->coll_form == 1) {
      const size_t tv = size_t(d->I) * d->R * n3 * sizeof(double);
      l.off_h = o;
      o += qcoll::al256(tv);
      l.off_q = o;
      o += qcoll::al256(tv);
      l.items = long(d->I) * d->R;
    } else {
      l.items = long(d->I) * d->K;
    }
    l.off_ews = o;
    o += qcoll::al256(qcoll::make_layout(d->plan->p, l.items, 0).total);
  }
  if (rk >= 1) {
    l.off_r = o;
    o += qcoll::al256(vol);
  }
  if (rk >= 2) {
    l.off_v1 = o;
    o += qcoll::al256(vol);
  }
  if (rk >= 3) {
    l.off_v2 = o;
    o += qcoll::al256(vol);
  }
  l.total = o;
  return l;
}

// R = L(F)
qcoll_status dg1d_rhs(qcoll_dg1d d, const double *F, double *Rout, char *ws, const DgLayout &l, hipStream_t st) {
  const qcoll::Plan &p = d->plan->p;
  const long n3 = p.n3();
  qcoll_status s;
  const double *C = nullptr;
  double cscale = 0.0;
  if (d->inv_kn > 0.0) {
    double *Cw = reinterpret_cast<double *>(ws + l.off_c);
    void *ews = ws + l.off_ews;
    const qcoll::Layout lay = qcoll::make_layout(p, l.items, 0);
    if (d->coll_form == 1) {
      double *Hd = reinterpret_cast<double *>(ws + l.off_h);
      double *Qd = reinterpret_cast<double *>(ws + l.off_q);
      if ((s = qcoll::launch_dg_contract(d->T, F, Hd, d->I, d->R, d->K, n3, st)) != QCOLL_OK) return s;
      if ((s = qcoll::launch_eval(p, l.items, Hd, Qd, ews, lay, st)) != QCOLL_OK) return s;
      if (d->conserve && (s = qcoll::launch_conserve(p, l.items, Qd, nullptr, st)) != QCOLL_OK) return s;
      if ((s = qcoll::launch_dg_contract(d->W, Qd, Cw, d->I, d->K, d->R, n3, st)) != QCOLL_OK) return s;
      cscale = 1.0;   // inv_kn / w_m are in W
    } else {
      if ((s = qcoll::launch_eval(p, l.items, F, Cw, ews, lay, st)) != QCOLL_OK) return s;
      if (d->conserve && (s = qcoll::launch_conserve(p, l.items, Cw, nullptr, st)) != QCOLL_OK) return s;
      cscale = d->inv_kn;
    }
    C = Cw;
  }
  qcoll::Dg1dArgs a;
  a.F = F;
  a.R = Rout;
  a.C = C;
  a.cscale = cscale;
  a.J = d->J;
  a.tab = d->tab;
  a.nw = d->nw;
  for (int side = 0; side < 2; ++side) {
    const qcoll_bc &b = d->ends[side];
    a.end[side].kind = b.kind;
    a.end[side].ux = b.u[0];
    a.end[side].nrm = side == 0 ? -1.0 : 1.0;
    a.end[side].den = d->den[side];
    a.end[side].fb = d->fb ? d->fb + size_t(side) * n3 : nullptr;
  }
  a.I = d->I;
  a.K = d->K;
  a.N = p.N;
  a.n3 = n3;
  a.L = p.L;
  a.periodic = d->ends[0].kind == QCOLL_BC_PERIODIC;
  if (!a.periodic) {
    qcoll::TimedLaunch tl("dg1d wall", st);
    hipLaunchKernelGGL(qcoll::k_dg1d_wall, dim3(2), dim3(1024), 0, st, a);
    if (hipGetLastError() != hipSuccess) return dfail(QCOLL_EDEVICE, "dg1d wall launch failed");
  }
  {
    qcoll::TimedLaunch tl("dg1d transport", st);
    const long n = long(d->I) * n3;
    hipLaunchKernelGGL(qcoll::k_dg1d_rhs, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, a);
    if (hipGetLastError() != hipSuccess) return dfail(QCOLL_EDEVICE, "dg1d transport launch failed");
  }
  return QCOLL_OK;
}

qcoll_status axpby3(double *out, const double *x, double a, const double *y, double b, const double *z, double c,
                    long n, hipStream_t st) {
  qcoll::TimedLaunch tl("dg1d rk update", st);
  hipLaunchKernelGGL(qcoll::k_axpby3, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, out, x, a, y, b, z, c, n);
  if (hipGetLastError() != hipSuccess) return dfail(QCOLL_EDEVICE, "dg1d rk update launch failed");
  return QCOLL_OK;
}

}  // namespace

extern "C" {

qcoll_status qcoll_dg1d_create(qcoll_plan plan, const qcoll_dg1d_params *prm, qcoll_dg1d *out) {
  if (!plan || !prm || !out) return dfail(QCOLL_EINVAL, "NULL argument");
  const int I = prm->n_elem, P = prm->order;
  if (I < 1 || I > (1 << 20)) return dfail(QCOLL_EINVAL, "n_elem must be in 1..2^20");
  if (P < 0 || P + 1 > qcoll::kMaxK) return dfail(QCOLL_EINVAL, "order must be in 0..7");
  if (!prm->faces) return dfail(QCOLL_EINVAL, "faces is NULL");
  for (int i = 0; i <= I; ++i)
    if (!std::isfinite(prm->faces[i]) || (i > 0 && !(prm->faces[i] > prm->faces[i - 1])))
      return dfail(QCOLL_EINVAL, "faces must be finite and strictly increasing");
  if (!(prm->inv_kn >= 0.0) || !std::isfinite(prm->inv_kn)) return dfail(QCOLL_EINVAL, "inv_kn must be finite and >= 0");
  if (prm->coll_form != 0 && prm->coll_form != 1) return dfail(QCOLL_EINVAL, "coll_form must be 0 or 1");
  if (!bc_ok(prm->left) || !bc_ok(prm->right)) return dfail(QCOLL_EINVAL, "bad boundary condition");
  if ((prm->left.kind == QCOLL_BC_PERIODIC) != (prm->right.kind == QCOLL_BC_PERIODIC))
    return dfail(QCOLL_EINVAL, "periodic needs both ends periodic");
  auto *d = new (std::nothrow) qcoll_dg1d_s;
  if (!d) return dfail(QCOLL_ENOMEM, "host allocation failed");
  d->plan = plan;
  d->I = I;
  d->K = P + 1;
  d->inv_kn = prm->inv_kn;
  d->coll_form = prm->coll_form;
  d->conserve = prm->conserve != 0;
  d->ends[0] = prm->left;
  d->ends[1] = prm->right;
  d->faces.assign(prm->faces, prm->faces + I + 1);
  const int K = d->K;
  const qcoll::Plan &p = plan->p;
  const int N = p.N;
  const long n3 = p.n3();
  // reference element: Gauss nodes and weights, stiffness, traces
  std::vector<double> xi, w;
  qcoll::gauss_legendre(K, -1.0, 1.0, xi, w);
  std::vector<double> tab(size_t(K) * (K + 3));
  for (int m = 0; m < K; ++m) tab[m] = w[m];
  for (int m = 0; m < K; ++m)
    for (int l = 0; l < K; ++l) tab[K + m * K + l] = w[l] * qcoll::lagrange_deriv(xi, m, l);
  std::vector<double> ph;
  qcoll::lagrange_at(xi, -1.0, ph);
  for (int l = 0; l < K; ++l) tab[K + K * K + l] = ph[l];
  qcoll::lagrange_at(xi, 1.0, ph);
  for (int l = 0; l < K; ++l) tab[2 * K + K * K + l] = ph[l];
  std::vector<double> J(I);
  d->xnodes.resize(size_t(I) * K);
  for (int i = 0; i < I; ++i) {
    J[i] = 0.5 * (d->faces[i + 1] - d->faces[i]);
    const double xc = 0.5 * (d->faces[i + 1] + d->faces[i]);
    for (int m = 0; m < K; ++m) d->xnodes[size_t(i) * K + m] = xc + J[i] * xi[m];
  }
  qcoll_status st;
  if ((st = qcoll::upload_vec(tab, &d->tab)) != QCOLL_OK || (st = qcoll::upload_vec(J, &d->J)) != QCOLL_OK) {
    free_dg1d(d);
    delete d;
    return st;
  }
  // exact triple tensor of the reference element and its eigen factors (Section 3.3.1)
  d->R = K;
  if (prm->coll_form == 1) {
    std::vector<double> xq, wqq;
    qcoll::gauss_legendre(2 * K, -1.0, 1.0, xq, wqq);
    std::vector<std::vector<double>> phq(xq.size());
    for (size_t q = 0; q < xq.size(); ++q) qcoll::lagrange_at(xi, xq[q], phq[q]);
    std::vector<double> Trows, Wcols;   // Trows [R][K]; Wcols per term (m, scaled eigenvalue)
    std::vector<int> Wm;
    for (int m = 0; m < K; ++m) {
      std::vector<double> Hm(size_t(K) * K, 0.0), V;
      for (size_t q = 0; q < xq.size(); ++q)
        for (int a1 = 0; a1 < K; ++a1)
          for (int b1 = 0; b1 < K; ++b1)
            Hm[size_t(a1) * K + b1] += wqq[q] * phq[q][m] * phq[q][a1] * phq[q][b1];
      qcoll::sym_eigen(Hm, K, V);
      double lmax = 0.0;
      for (int r = 0; r < K; ++r) lmax = std::max(lmax, std::fabs(Hm[size_t(r) * K + r]));
      for (int r = 0; r < K; ++r) {
        const double lam = Hm[size_t(r) * K + r];
        if (!(std::fabs(lam) > 1e-13 * lmax)) continue;
        for (int k = 0; k < K; ++k) Trows.push_back(V[size_t(k) * K + r]);
        Wcols.push_back(lam * prm->inv_kn / w[m]);
        Wm.push_back(m);
      }
    }
    d->R = int(Wcols.size());
    std::vector<double> Wfull(size_t(K) * d->R, 0.0);
    for (int r = 0; r < d->R; ++r) Wfull[size_t(Wm[r]) * d->R + r] = Wcols[r];
    if ((st = qcoll::upload_vec(Trows, &d->T)) != QCOLL_OK || (st = qcoll::upload_vec(Wfull, &d->W)) != QCOLL_OK) {
      free_dg1d(d);
      delete d;
      return st;
    }
  }
  // boundary states
  if (prm->left.kind != QCOLL_BC_PERIODIC) {
    std::vector<double> fb(size_t(2) * n3);
    const double dc = 2.0 * p.L / N;
    for (int side = 0; side < 2; ++side) {
      const qcoll_bc &b = d->ends[side];
      const double nrm = side == 0 ? -1.0 : 1.0;
      const double pref = b.kind == QCOLL_BC_INFLOW ? b.n / std::pow(M_PI * b.T, 1.5) : 1.0;
      double den = 0.0;
      for (long j = 0; j < n3; ++j) {
        const int j1 = int(j / (long(N) * N)), j2 = int((j / N) % N), j3 = int(j % N);
        const double c[3] = {-p.L + (j1 + 0.5) * dc, -p.L + (j2 + 0.5) * dc, -p.L + (j3 + 0.5) * dc};
        double r2 = 0.0;
        for (int k = 0; k < 3; ++k) r2 += (c[k] - b.u[k]) * (c[k] - b.u[k]);
        const double v = pref * std::exp(-r2 / b.T);
        fb[size_t(side) * n3 + j] = v;
        const double cn = (c[0] - b.u[0]) * nrm;
        if (cn < 0.0) den += cn * v;
      }
      d->den[side] = den < 0.0 ? den : -1.0;
    }
    if ((st = qcoll::upload_vec(fb, &d->fb)) != QCOLL_OK) {
      free_dg1d(d);
      delete d;
      return st;
    }
  }
  if (hipMalloc(&d->nw, 2 * sizeof(double)) != hipSuccess) {
    free_dg1d(d);
    delete d;
    return dfail(QCOLL_ENOMEM, "hipMalloc failed for the wall densities");
  }
  *out = d;
  return QCOLL_OK;
}

qcoll_status qcoll_dg1d_destroy(qcoll_dg1d d) {
  if (!d) return QCOLL_OK;
  free_dg1d(d);
  delete d;
  return QCOLL_OK;
}

qcoll_status qcoll_dg1d_nodes(qcoll_dg1d d, double *host_x) {
  if (!d || !host_x) return dfail(QCOLL_EINVAL, "NULL argument");
  std::copy(d->xnodes.begin(), d->xnodes.end(), host_x);
  return QCOLL_OK;
}

size_t qcoll_dg1d_workspace_bytes(qcoll_dg1d d, int32_t rk) {
  if (!d || rk < 0 || rk > 3) return 0;
  return dg_layout(d, rk).total;
}

qcoll_status qcoll_dg1d_rhs(qcoll_dg1d d, const double *F, double *R, void *ws, size_t ws_bytes, void *stream) {
  if (!d || !F || !R) return dfail(QCOLL_EINVAL, "NULL argument");
  const size_t vol = size_t(d->I) * d->K * d->plan->p.n3();
  if ((const void *)F < (const void *)(R + vol) && (const void *)R < (const void *)(F + vol))
    return dfail(QCOLL_EINVAL, "R must not overlap F");
  const DgLayout l = dg_layout(d, 0);
  if (!ws || ws_bytes < l.total) return dfail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_dg1d_workspace_bytes(0)");
  return dg1d_rhs(d, F, R, static_cast<char *>(ws), l, static_cast<hipStream_t>(stream));
}

qcoll_status qcoll_dg1d_step(qcoll_dg1d d, double *F, double dt, int32_t rk, void *ws, size_t ws_bytes,
                             void *stream) {
  if (!d || !F) return dfail(QCOLL_EINVAL, "NULL argument");
  if (rk < 1 || rk > 3) return dfail(QCOLL_EINVAL, "rk must be 1, 2 or 3");
  if (!std::isfinite(dt)) return dfail(QCOLL_EINVAL, "dt must be finite");
  const DgLayout l = dg_layout(d, rk);
  if (!ws || ws_bytes < l.total) return dfail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_dg1d_workspace_bytes(rk)");
  char *w = static_cast<char *>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long n = long(d->I) * d->K * d->plan->p.n3();
  double *Rb = reinterpret_cast<double *>(w + l.off_r);
  double *v1 = rk >= 2 ? reinterpret_cast<double *>(w + l.off_v1) : nullptr;
  double *v2 = rk >= 3 ? reinterpret_cast<double *>(w + l.off_v2) : nullptr;
  qcoll_status s;
  if ((s = dg1d_rhs(d, F, Rb, w, l, st)) != QCOLL_OK) return s;
  if (rk == 1) return axpby3(F, F, 1.0, Rb, dt, nullptr, 0.0, n, st);
  // SSP-RK2 / SSP-RK3 (Section 3.4)
  if ((s = axpby3(v1, F, 1.0, Rb, dt, nullptr, 0.0, n, st)) != QCOLL_OK) return s;
  if ((s = dg1d_rhs(d, v1, Rb, w, l, st)) != QCOLL_OK) return s;
  if (rk == 2) return axpby3(F, F, 0.5, v1, 0.5, Rb, 0.5 * dt, n, st);
  if ((s = axpby3(v2, F, 0.75, v1, 0.25, Rb, 0.25 * dt, n, st)) != QCOLL_OK) return s;
  if ((s = dg1d_rhs(d, v2, Rb, w, l, st)) != QCOLL_OK) return s;
  return axpby3(F, F, 1.0 / 3.0, v2, 2.0 / 3.0, Rb, 2.0 / 3.0 * dt, n, st);
}

}  // extern "C"
