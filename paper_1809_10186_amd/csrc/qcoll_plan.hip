// Plan precompute on the host in FP64: quadratures, kernel-mode tables, shift
// tables, optional SVD of the gain-weight table; then upload to the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "qcoll_internal.h"

namespace qcoll {

// Gauss-Legendre nodes/weights on [a, b] (ascending) by Newton iteration on P_n.
void gauss_legendre(int n, double a, double b, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(3.141592653589793238462643383279502884 * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1, pm = (n == 1) ? 1.0 : p0;
    dp = n * (z * pn - pm) / (z * z - 1.0);
    // nodes ascending in [a, b]
    x[n - 1 - i] = 0.5 * (b - a) * z + 0.5 * (b + a);
    w[n - 1 - i] = (b - a) / ((1.0 - z * z) * dp * dp);
  }
}


namespace {

constexpr double kPiD = 3.141592653589793238462643383279502884;

// built-in half-sphere rule: one vertex per antipodal pair of the icosahedron
void icosahedral_half(std::vector<double> &s) {
  const double ph = 0.5 * (1.0 + std::sqrt(5.0));
  const double nrm = std::sqrt(1.0 + ph * ph);
  const double a = 1.0 / nrm, c = ph / nrm;
  const double pts[6][3] = {{0, a, c}, {0, -a, c}, {a, c, 0}, {-a, c, 0}, {c, 0, a}, {c, 0, -a}};
  s.resize(24);
  for (int i = 0; i < 6; ++i) {
    s[4 * i + 0] = pts[i][0];
    s[4 * i + 1] = pts[i][1];
    s[4 * i + 2] = pts[i][2];
    s[4 * i + 3] = 2.0 * kPiD / 6.0;
  }
}

double sinc(double z) { return z == 0.0 ? 1.0 : std::sin(z) / z; }

int kappa(int n, int N) { return n < N / 2 ? n : n - N; }

// One-sided Jacobi: rotate the rows of A [m][n] until pairwise orthogonal.
// On return A holds J A (orthogonal rows) and J [m][m] the accumulated rotation.
void jacobi_rows(std::vector<double> &A, int m, long n, std::vector<double> &J) {
  J.assign(size_t(m) * m, 0.0);
  for (int i = 0; i < m; ++i) J[size_t(i) * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m - 1; ++i) {
      for (int j = i + 1; j < m; ++j) {
        double *ri = &A[size_t(i) * n], *rj = &A[size_t(j) * n];
        double a = 0, b = 0, c = 0;
        for (long k = 0; k < n; ++k) {
          a += ri[k] * ri[k];
          b += rj[k] * rj[k];
          c += ri[k] * rj[k];
        }
        if (a == 0.0 || b == 0.0) continue;
        double rel = std::fabs(c) / std::sqrt(a * b);
        off = std::max(off, rel);
        if (rel < 1e-16) continue;
        double zeta = (b - a) / (2.0 * c);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (long k = 0; k < n; ++k) {
          double x = ri[k], y = rj[k];
          ri[k] = cs * x - sn * y;
          rj[k] = sn * x + cs * y;
        }
        double *Ji = &J[size_t(i) * m], *Jj = &J[size_t(j) * m];
        for (int k = 0; k < m; ++k) {
          double x = Ji[k], y = Jj[k];
          Ji[k] = cs * x - sn * y;
          Jj[k] = sn * x + cs * y;
        }
      }
    }
    if (off < 1e-15) break;
  }
}

template <typename T>
qcoll_status upload(const std::vector<double> &h, void **dptr) {
  std::vector<T> t(h.begin(), h.end());
  if (hipMalloc(dptr, t.size() * sizeof(T)) != hipSuccess) {
    *dptr = nullptr;
    set_error("hipMalloc failed for a plan table");
    return QCOLL_ENOMEM;
  }
  if (hipMemcpy(*dptr, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("hipMemcpy failed for a plan table");
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

}  // namespace

bool supported_N(int N) {
  return N == 8 || N == 12 || N == 16 || N == 24 || N == 32 || N == 48 || N == 64;
}

// d ln(b rho_p^{4-2 omega}) / d omega for every radial node (the omega gradient):
// d ln b / d omega = ln 2 + psi(2.5 - omega) when b follows omega (the VHS and
// VSS constants alike), psi by recurrence and the asymptotic series; else 0
static qcoll_status upload_dlog(Plan &p) {
  std::vector<double> dl(p.N_rho);
  double dlb = 0.0;
  if (p.b_follows_omega) {
    double x = 2.5 - p.omega, acc = 0.0;
    while (x < 8.0) { acc -= 1.0 / x; x += 1.0; }
    const double x2 = 1.0 / (x * x);
    const double psi = acc + std::log(x) - 0.5 / x -
                       x2 * (1.0 / 12 - x2 * (1.0 / 120 - x2 * (1.0 / 252 - x2 * (1.0 / 240 - x2 / 132))));
    dlb = std::log(2.0) + psi;
  }
  for (int r = 0; r < p.N_rho; ++r) dl[r] = dlb - 2.0 * std::log(p.rho[r]);
  return upload<double>(dl, reinterpret_cast<void **>(&p.dlog));
}

// Kernel tables for the current omega/prefactor (alpha_p rows, Lambda, Lambda_p).
static void kernel_tables(const Plan &p, std::vector<double> &alpha, std::vector<double> &lam,
                          std::vector<double> &lam_p) {
  const int N = p.N;
  const long n3 = p.n3();
  double wsum = 0;
  for (int q = 0; q < p.M; ++q) wsum += p.sphere[4 * q + 3];
  alpha.assign(size_t(p.N_rho) * n3, 0.0);
  lam.assign(n3, 0.0);
  lam_p.assign(size_t(p.N_rho) * n3, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) {
        const double k1 = kappa(i, N), k2 = kappa(j, N), k3 = kappa(k, N);
        const double ka = std::sqrt(k1 * k1 + k2 * k2 + k3 * k3);
        const long idx = (long(i) * N + j) * N + k;
        for (int r = 0; r < p.N_rho; ++r) {
          const double rr = p.rho[r], wr = p.w_rho[r];
          const double c = 4.0 * kPiD * p.b * std::pow(rr, 4.0 - 2.0 * p.omega);
          // gain: 2 w_p F(k, rho_p); F = 4 pi b rho^{4-2w} sinc(pi rho |k| / (2L))
          alpha[size_t(r) * n3 + idx] = 2.0 * wr * c * sinc(kPiD * rr * ka / (2.0 * p.L));
          // loss: 2 (sum_q w_q) w_p F(2k, rho_p)
          const double lp = 2.0 * wsum * wr * c * sinc(kPiD * rr * ka / p.L);
          lam_p[size_t(r) * n3 + idx] = lp;
          lam[idx] += lp;
        }
      }
}

// effective per-node gain weights sum_s U[s][p] V_s (already / N^3), for the
// fused schedule, which transforms each A_p on chip and so cannot mix before
// the transform
static std::vector<double> effective_rows(const Plan &p, const std::vector<double> &Vs, const std::vector<double> &U,
                                          int rows) {
  const int m = p.N_rho;
  const long n3 = p.n3();
  std::vector<double> ae(size_t(m) * n3, 0.0);
  for (int s = 0; s < rows; ++s)
    for (int q = 0; q < m; ++q) {
      const double u = U[size_t(s) * m + q];
      if (u == 0.0) continue;
      for (long k = 0; k < n3; ++k) ae[size_t(q) * n3 + k] += u * Vs[size_t(s) * n3 + k];
    }
  return ae;
}

static qcoll_status upload_alpha_eff(Plan &p, const std::vector<double> &Vs, const std::vector<double> &U) {
  if (!fused_gain_supported(p.N, p.precision)) return QCOLL_OK;
  const int m = p.N_rho;
  const long n3 = p.n3();
  std::vector<double> ae(size_t(m) * n3, 0.0);
  for (int s = 0; s < p.nv; ++s)
    for (int q = 0; q < m; ++q) {
      const double u = U[size_t(s) * m + q];
      if (u == 0.0) continue;
      for (long k = 0; k < n3; ++k) ae[size_t(q) * n3 + k] += u * Vs[size_t(s) * n3 + k];
    }
  return p.precision == QCOLL_FP32 ? upload<float>(ae, &p.alpha_eff) : upload<double>(ae, &p.alpha_eff);
}

static qcoll_status upload_kernel_tables(Plan &p) {
  std::vector<double> alpha, lam, lam_p;
  kernel_tables(p, alpha, lam, lam_p);
  const int m = p.N_rho;
  const long n3 = p.n3();
  std::vector<double> V, U;
  p.truncated = false;
  p.mix_identity = true;
  p.rank = m;
  p.nv = m;
  p.sigma_max = p.sigma_min_kept = 0.0;
  V = alpha;
  U.assign(size_t(m) * m, 0.0);
  for (int i = 0; i < m; ++i) U[size_t(i) * m + i] = 1.0;
  // V rows scaled by 1/N^3 (normalised inverse transform), padded to an even count
  const double inv = 1.0 / double(n3);
  const int rows = 2 * p.npair();
  std::vector<double> Vs(size_t(rows) * n3, 0.0);
  for (size_t i = 0; i < size_t(p.nv) * n3; ++i) Vs[i] = V[i] * inv;
  std::vector<double> lams(lam);
  for (auto &x : lams) x *= inv;
  qcoll_status st;
  auto up = [&](const std::vector<double> &h, void **d) {
    return p.precision == QCOLL_FP32 ? upload<float>(h, d) : upload<double>(h, d);
  };
  if ((st = up(Vs, &p.V)) != QCOLL_OK) return st;
  if (p.precision == QCOLL_FP32 && (st = upload<double>(Vs, reinterpret_cast<void **>(&p.V64))) != QCOLL_OK) return st;
  if ((st = upload<double>(lams, &p.lam)) != QCOLL_OK) return st;
  if ((st = up(U, &p.umix_d)) != QCOLL_OK) return st;
  p.umix = U;
  if ((st = upload_alpha_eff(p, Vs, U)) != QCOLL_OK) return st;
  if ((st = upload<double>(lam_p, reinterpret_cast<void **>(&p.lam_p))) != QCOLL_OK) return st;
  return upload_dlog(p);
}

static qcoll_status upload_truncated(Plan &p, int svd_rank, double svd_tol) {
  std::vector<double> alpha, lam, lam_p;
  kernel_tables(p, alpha, lam, lam_p);
  const int m = p.N_rho;
  const long n3 = p.n3();
  std::vector<double> J;
  jacobi_rows(alpha, m, n3, J);
  std::vector<double> nrm(m);
  for (int i = 0; i < m; ++i) {
    double s = 0;
    for (long k = 0; k < n3; ++k) s += alpha[size_t(i) * n3 + k] * alpha[size_t(i) * n3 + k];
    nrm[i] = std::sqrt(s);
  }
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  int r = m;
  if (svd_rank > 0) {
    r = std::min(svd_rank, m);
  } else {
    r = 0;
    for (int i = 0; i < m; ++i)
      if (nrm[ord[i]] > svd_tol * nrm[ord[0]]) ++r;
    r = std::max(r, 1);
  }
  p.truncated = true;
  p.mix_identity = false;
  p.rank = r;
  p.nv = r;
  p.sigma_max = nrm[ord[0]];
  p.sigma_min_kept = nrm[ord[r - 1]];
  const double inv = 1.0 / double(n3);
  std::vector<double> Vs(size_t(r + 1) * n3, 0.0), U(size_t(r) * m);
  for (int s = 0; s < r; ++s) {
    for (long k = 0; k < n3; ++k) Vs[size_t(s) * n3 + k] = alpha[size_t(ord[s]) * n3 + k] * inv;
    for (int q = 0; q < m; ++q) U[size_t(s) * m + q] = J[size_t(ord[s]) * m + q];
  }
  if ((r + 1) / 2 >= (m + 1) / 2) {
    // mixing before the transforms would not save a packed transform: use the
    // truncated table itself, alpha~_p = sum_s U[s][p] V_s, with U = I
    std::vector<double> at = effective_rows(p, Vs, U, r);
    p.nv = m;
    p.mix_identity = true;
    Vs.assign(size_t(m + 1) * n3, 0.0);
    std::copy(at.begin(), at.end(), Vs.begin());
    U.assign(size_t(m) * m, 0.0);
    for (int i = 0; i < m; ++i) U[size_t(i) * m + i] = 1.0;
  }
  Vs.resize(size_t(2 * p.npair()) * n3);
  std::vector<double> lams(lam);
  for (auto &x : lams) x *= inv;
  qcoll_status st;
  auto up = [&](const std::vector<double> &h, void **d) {
    return p.precision == QCOLL_FP32 ? upload<float>(h, d) : upload<double>(h, d);
  };
  if ((st = up(Vs, &p.V)) != QCOLL_OK) return st;
  if (p.precision == QCOLL_FP32 && (st = upload<double>(Vs, reinterpret_cast<void **>(&p.V64))) != QCOLL_OK) return st;
  if ((st = upload<double>(lams, &p.lam)) != QCOLL_OK) return st;
  if ((st = up(U, &p.umix_d)) != QCOLL_OK) return st;
  p.umix = U;
  return upload_alpha_eff(p, Vs, U);
}

// ---------------------------------------------------------------------------
// VSS kernel modes (Section 2 kernel with alpha in (1, 2]; Appendix definition
// of F with the kernel symmetrised in cos chi), by the Funk-Hecke formula.
// With A(t) = ((1+t)^{alpha-1} + (1-t)^{alpha-1}) / 2 and a = pi rho |k| / (2L):
//   F(k, rho, sigma) = 2 rho^2 b rho^{2(1-omega)} int_{S^2+} A(sigma.c) cos(a k^.c) dc
//                    = b rho^{4-2 omega} int_{S^2} A(sigma.c) cos(a k^.c) dc      (even in c).
// The plane wave is sum_n (2n+1) i^n j_n(a) P_n(k^.c); Funk-Hecke turns
// int_{S^2} A(sigma.c) P_n(k^.c) dc into 2 pi (int_{-1}^{1} A P_n dt) P_n(sigma.k^);
// A is even, so only even n remain and int A P_n = c_n := int (1-t)^{alpha-1} P_n dt:
//   F = 2 pi b rho^{4-2 omega} sum_{n even} (2n+1) (-1)^{n/2} c_n j_n(a) P_n(sigma.k^),
// with c_0 = 2^alpha / alpha and c_n = -c_{n-1} (alpha - n) / (alpha + n).  For
// alpha = 1 (or 2) only c_0 survives among even n and F is the VHS closed form.

// j_0..j_nmax(a) by downward recurrence from well above nmax, normalised by
// sum_n (2n+1) j_n(a)^2 = 1 and signed by the larger of j_0, j_1 in closed form.
static void sph_bessel(double a, int nmax, std::vector<double> &j, std::vector<double> &t) {
  j.assign(nmax + 1, 0.0);
  if (a == 0.0) {
    j[0] = 1.0;
    return;
  }
  const int nst = std::max(nmax, int(a)) + 60;
  t.assign(nst + 2, 0.0);
  t[nst] = 1e-30;
  for (int n = nst; n >= 1; --n) {
    t[n - 1] = (2.0 * n + 1.0) / a * t[n] - t[n + 1];
    if (std::fabs(t[n - 1]) > 1e100)
      for (int k = n - 1; k <= nst; ++k) t[k] *= 1e-100;
  }
  // normalise relative to the largest value (neither the squares nor their sum
  // can overflow or underflow)
  double tmax = 0.0;
  for (int n = 0; n <= nst; ++n) tmax = std::max(tmax, std::fabs(t[n]));
  double s = 0.0;
  for (int n = nst; n >= 0; --n) {
    const double u = t[n] / tmax;
    s += (2.0 * n + 1.0) * u * u;
  }
  double scale = 1.0 / (tmax * std::sqrt(s));
  const double j0 = std::sin(a) / a, j1 = std::sin(a) / (a * a) - std::cos(a) / a;
  if (std::fabs(j0) >= std::fabs(j1)) {
    if ((j0 < 0) != (t[0] < 0)) scale = -scale;
  } else if ((j1 < 0) != (t[1] < 0)) {
    scale = -scale;
  }
  for (int n = 0; n <= nmax; ++n) j[n] = t[n] * scale;
}

// terms needed for |k| with argument a: j_n(a) is negligible past a + O(a^{1/3})
static int vss_nmax(double a) { return (int(a + 10.0 * std::cbrt(a) + 30.0) / 2) * 2; }

// F / (b rho^{4-2 omega}) for the given direction cosines mu_q = sigma_q . k^
static void vss_modes(double a, const double *mu, int nq, const std::vector<double> &coef, double *out,
                      std::vector<double> &jn, std::vector<double> &tmp) {
  const int nmax = std::min(vss_nmax(a), int(coef.size()) - 1);
  sph_bessel(a, nmax, jn, tmp);
  for (int q = 0; q < nq; ++q) {
    const double m = mu[q];
    double p0 = 1.0, p1 = m, acc = coef[0] * jn[0];
    for (int n = 2; n <= nmax; n += 2) {
      // advance P_{n-1}, P_n by the three-term recurrence
      const double p2 = ((2.0 * (n - 1) + 1.0) * m * p1 - (n - 1) * p0) / n;
      acc += coef[n] * jn[n] * p2;
      const double p3 = ((2.0 * n + 1.0) * m * p2 - n * p1) / (n + 1);
      p0 = p2;
      p1 = p3;
    }
    out[q] = acc;
  }
}

// alpha_pq half tables (T precision, / N^3) and Lambda (FP64, / N^3) for a VSS plan
static qcoll_status upload_vss_tables(Plan &p) {
  const int N = p.N, Nr = p.N_rho, M = p.M, H1 = N / 2 + 1;
  const long n2 = long(N) * N, n3 = p.n3(), nh = long(H1) * n2;
  const double alpha = p.vss;
  // coefficient of n in the series: 2 pi (2n+1) (-1)^{n/2} c_n (even n; odd entries unused)
  double amax = 0.0;
  for (int r = 0; r < Nr; ++r) amax = std::max(amax, kPiD * p.rho[r] * std::sqrt(3.0) * (N / 2) / p.L);
  const int ncoef = vss_nmax(amax) + 2;
  std::vector<double> cn(ncoef + 1), coef(ncoef + 1, 0.0);
  cn[0] = std::pow(2.0, alpha) / alpha;
  for (int n = 1; n <= ncoef; ++n) cn[n] = -cn[n - 1] * (alpha - n) / (alpha + n);
  for (int n = 0; n <= ncoef; n += 2) coef[n] = 2.0 * kPiD * (2.0 * n + 1.0) * ((n / 2) % 2 ? -1.0 : 1.0) * cn[n];
  std::vector<double> apq(size_t(Nr) * M * nh, 0.0), lam_p(size_t(Nr) * n3, 0.0);
  const double inv = 1.0 / double(n3);
  // The self-paired index N/2 of an axis stands for the frequencies +-N/2: a
  // multiplier acts on it as the average of its two values (for the shift
  // factor this is the cosine rule of the plan's phase tables).  F depends on
  // the signs of the components through k^.sigma, so at indices with Nyquist
  // components it is averaged over their sign patterns; the weights are then
  // even under index reflection and the gain and loss spectra Hermitian.
  auto work = [&](int r) {
    const double rr = p.rho[r], wr = p.w_rho[r];
    const double c = p.b * std::pow(rr, 4.0 - 2.0 * p.omega);
    std::vector<double> mu(M), fq(M), acc(M), jn, tmp;
    for (long idx = 0; idx < n3; ++idx) {
      const int i = int(idx / n2), jj = int((idx / N) % N), kk = int(idx % N);
      const double k1 = kappa(i, N), k2 = kappa(jj, N), k3 = kappa(kk, N);
      const double ka = std::sqrt(k1 * k1 + k2 * k2 + k3 * k3);
      const bool nq1 = (i == N / 2), nq2 = (jj == N / 2), nq3 = (kk == N / 2);
      const int npat = (nq1 || nq2 || nq3) ? 8 : 1;
      // acc[q] = F(arg a, k^.sigma_q) / (b rho^{4-2 omega}), sign-averaged
      auto modes = [&](double a) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int sg = 0; sg < npat; ++sg) {
          const double x1 = (nq1 && (sg & 1)) ? -k1 : k1;
          const double x2 = (nq2 && (sg & 2)) ? -k2 : k2;
          const double x3 = (nq3 && (sg & 4)) ? -k3 : k3;
          for (int q = 0; q < M; ++q) {
            const double *sv = &p.sphere[4 * q];
            mu[q] = ka > 0 ? std::max(-1.0, std::min(1.0, (x1 * sv[0] + x2 * sv[1] + x3 * sv[2]) / ka)) : 1.0;
          }
          vss_modes(a, mu.data(), M, coef, fq.data(), jn, tmp);
          for (int q = 0; q < M; ++q) acc[q] += fq[q] / npat;
        }
      };
      // loss: Lambda_p(k) = sum_q 2 w_p w_q F(2k, rho_p, sigma_q)
      modes(kPiD * rr * ka / p.L);
      double lp = 0.0;
      for (int q = 0; q < M; ++q) lp += 2.0 * wr * p.sphere[4 * q + 3] * c * acc[q];
      lam_p[size_t(r) * n3 + idx] = lp;
      // gain on the planes k1 <= N/2: 2 w_p w_q F(k, rho_p, sigma_q) / N^3
      if (i < H1) {
        modes(kPiD * rr * ka / (2.0 * p.L));
        for (int q = 0; q < M; ++q)
          apq[(size_t(r) * M + q) * nh + idx] = 2.0 * wr * p.sphere[4 * q + 3] * c * acc[q] * inv;
      }
    }
  };
  // radial nodes over host threads; each node writes only its own rows
  const int nth = std::max(1, std::min(Nr, int(std::thread::hardware_concurrency())));
  std::vector<std::thread> th;
  int started = 0;
  try {
    for (int t = 0; t < nth; ++t) {
      th.emplace_back([&, t] {
        for (int r = t; r < Nr; r += nth) work(r);
      });
      ++started;
    }
  } catch (...) {
    // no more threads: the nodes of the threads that did not start run here
  }
  for (int t = started; t < nth; ++t)
    for (int r = t; r < Nr; r += nth) work(r);
  for (auto &x : th) x.join();
  std::vector<double> lam(n3, 0.0);
  for (int r = 0; r < Nr; ++r)
    for (long k = 0; k < n3; ++k) lam[k] += lam_p[size_t(r) * n3 + k];
  for (auto &x : lam) x *= inv;
  p.truncated = false;
  p.mix_identity = true;
  p.rank = p.nv = Nr;
  p.sigma_max = p.sigma_min_kept = 0.0;
  qcoll_status st;
  if ((st = upload<double>(lam, &p.lam)) != QCOLL_OK) return st;
  // per-node loss weights and d ln c_p / d omega: the VJP's omega gradient
  if ((st = upload<double>(lam_p, reinterpret_cast<void **>(&p.lam_p))) != QCOLL_OK) return st;
  if ((st = upload_dlog(p)) != QCOLL_OK) return st;
  return p.precision == QCOLL_FP32 ? upload<float>(apq, &p.alpha_pq) : upload<double>(apq, &p.alpha_pq);
}

static double kernel_constant(double omega, double alpha) {
  // non-dimensional VSS constant alpha / (2^{2-omega+alpha} Gamma(2.5-omega) pi) (Section 2)
  return alpha / (std::pow(2.0, 2.0 - omega + alpha) * std::tgamma(2.5 - omega) * kPiD);
}

static void free_kernel_tables(Plan &p) {
  (void)hipFree(p.V);
  (void)hipFree(p.V64);
  (void)hipFree(p.lam);
  (void)hipFree(p.umix_d);
  (void)hipFree(p.lam_p);
  (void)hipFree(p.dlog);
  (void)hipFree(p.alpha_eff);
  (void)hipFree(p.alpha_pq);
  p.alpha_eff = p.alpha_pq = nullptr;
  p.V = p.lam = p.umix_d = nullptr;
  p.V64 = nullptr;
  p.lam_p = p.dlog = nullptr;
}

qcoll_status plan_build(Plan &p, const qcoll_params &prm) {
  p.N = prm.N;
  p.L = prm.L;
  p.N_rho = prm.N_rho;
  p.omega = prm.omega;
  p.precision = prm.precision;
  p.vss = prm.alpha;
  p.literal = prm.nyquist == QCOLL_NYQ_LITERAL;
  p.b_follows_omega = !(prm.prefactor > 0.0);
  p.b = p.b_follows_omega ? kernel_constant(p.omega, p.vss) : prm.prefactor;
  p.R = 4.0 * p.L / (3.0 + std::sqrt(2.0));
  gauss_legendre(p.N_rho, 0.0, p.R, p.rho, p.w_rho);
  if (prm.sphere) {
    p.M = prm.M;
    p.sphere.assign(prm.sphere, prm.sphere + 4 * size_t(prm.M));
  } else {
    p.M = 6;
    icosahedral_half(p.sphere);
  }
  if (hipGetDevice(&p.device) != hipSuccess) {
    set_error("hipGetDevice failed");
    return QCOLL_EDEVICE;
  }
  const int N = p.N;
  // per-axis shift factors b_d(n) for s = rho_p sigma_q / 2
  std::vector<double> ph(size_t(p.N_rho) * p.M * 3 * N * 2);
  for (int r = 0; r < p.N_rho; ++r)
    for (int q = 0; q < p.M; ++q)
      for (int d = 0; d < 3; ++d) {
        const double s = 0.5 * p.rho[r] * p.sphere[4 * q + d];
        for (int n = 0; n < N; ++n) {
          const double th = kPiD * kappa(n, N) * s / p.L;
          double re = std::cos(th), im = std::sin(th);
          if (n == N / 2 && !p.literal) im = 0.0;  // cosine mode of the real interpolant
          const size_t o = ((((size_t(r) * p.M + q) * 3 + d) * N) + n) * 2;
          ph[o] = re;
          ph[o + 1] = im;
        }
      }
  std::vector<double> wq(p.M);
  for (int q = 0; q < p.M; ++q) wq[q] = p.sphere[4 * q + 3];
  qcoll_status st;
  if (p.precision == QCOLL_FP32) {
    if ((st = upload<float>(ph, &p.phase)) != QCOLL_OK) return st;
    if ((st = upload<float>(wq, &p.wq)) != QCOLL_OK) return st;
  } else {
    if ((st = upload<double>(ph, &p.phase)) != QCOLL_OK) return st;
    if ((st = upload<double>(wq, &p.wq)) != QCOLL_OK) return st;
  }
  // conservation: G = C C^T over the grid, inverted by Gauss-Jordan (5x5)
  {
    const double dc = 2.0 * p.L / N;
    double G[5][5] = {};
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
          const double c1 = -p.L + (i + 0.5) * dc, c2 = -p.L + (j + 0.5) * dc, c3 = -p.L + (k + 0.5) * dc;
          const double v[5] = {1.0, c1, c2, c3, c1 * c1 + c2 * c2 + c3 * c3};
          for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b) G[a][b] += v[a] * v[b];
        }
    double A[5][10] = {};
    for (int a = 0; a < 5; ++a) {
      for (int b = 0; b < 5; ++b) A[a][b] = G[a][b];
      A[a][5 + a] = 1.0;
    }
    for (int c = 0; c < 5; ++c) {
      int piv = c;
      for (int r = c + 1; r < 5; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      for (int k = 0; k < 10; ++k) std::swap(A[c][k], A[piv][k]);
      const double d = A[c][c];
      for (int k = 0; k < 10; ++k) A[c][k] /= d;
      for (int r = 0; r < 5; ++r)
        if (r != c) {
          const double m = A[r][c];
          for (int k = 0; k < 10; ++k) A[r][k] -= m * A[c][k];
        }
    }
    std::vector<double> gi(25);
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) gi[a * 5 + b] = A[a][5 + b];
    if ((st = upload<double>(gi, reinterpret_cast<void **>(&p.ginv))) != QCOLL_OK) return st;
  }
  if (hipMalloc(&p.flag, sizeof(int)) != hipSuccess) {
    set_error("hipMalloc failed for the status flag");
    return QCOLL_ENOMEM;
  }
  if (hipMemset(p.flag, 0, sizeof(int)) != hipSuccess) {
    set_error("hipMemset failed");
    return QCOLL_EDEVICE;
  }
  if (p.is_vss()) return upload_vss_tables(p);
  if (prm.svd_rank < 0) return upload_kernel_tables(p);
  return upload_truncated(p, prm.svd_rank, prm.svd_tol);
}

qcoll_status plan_set_omega(Plan &p, double omega) {
  if (p.truncated) {
    set_error("qcoll_plan_set_omega needs an untruncated plan");
    return QCOLL_ENOTSUP;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("hipDeviceSynchronize failed");
    return QCOLL_EDEVICE;
  }
  // build the new tables beside the old ones and swap them in only on
  // success: a failed rebuild leaves the plan as it was
  Plan t = p;
  t.alpha_eff = t.alpha_pq = nullptr;
  t.V = t.lam = t.umix_d = nullptr;
  t.V64 = nullptr;
  t.lam_p = t.dlog = nullptr;
  t.omega = omega;
  if (t.b_follows_omega) t.b = kernel_constant(t.omega, t.vss);
  const qcoll_status st = t.is_vss() ? upload_vss_tables(t) : upload_kernel_tables(t);
  if (st != QCOLL_OK) {
    free_kernel_tables(t);
    return st;
  }
  free_kernel_tables(p);
  p = t;
  ++p.gen;
  return QCOLL_OK;
}

// Copy a device table back to the host in FP64, undoing the 1/N^3 the kernels fold in.
template <typename T>
static qcoll_status fetch(const void *d, size_t n, std::vector<double> &out) {
  std::vector<T> t(n);
  if (hipMemcpy(t.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("hipMemcpy failed while reading a plan table");
    return QCOLL_EDEVICE;
  }
  out.assign(t.begin(), t.end());
  return QCOLL_OK;
}

qcoll_status plan_table(const Plan &p, int which, double *host, size_t n) {
  const long n3 = p.n3();
  const double scale = double(n3);
  std::vector<double> t;
  qcoll_status st;
  if (which == 0) {
    if (p.is_vss()) {
      set_error("VSS plans have per-(p, q) gain weights, not a per-node table");
      return QCOLL_ENOTSUP;
    }
    if (n != size_t(p.N_rho) * n3) {
      set_error("the gain-weight table has N_rho * N^3 entries");
      return QCOLL_EINVAL;
    }
    const size_t rows = size_t(2 * p.npair());
    st = p.precision == QCOLL_FP32 ? fetch<float>(p.V, rows * n3, t) : fetch<double>(p.V, rows * n3, t);
    if (st != QCOLL_OK) return st;
    // alpha~_p = sum_s U[s][p] V_s (U = I when the plan does not mix)
    for (int q = 0; q < p.N_rho; ++q)
      for (long k = 0; k < n3; ++k) {
        double acc = 0.0;
        if (p.mix_identity) {
          acc = t[size_t(q) * n3 + k];
        } else {
          for (int r = 0; r < p.nv; ++r) acc += p.umix[size_t(r) * p.N_rho + q] * t[size_t(r) * n3 + k];
        }
        host[size_t(q) * n3 + k] = acc * scale;
      }
    return QCOLL_OK;
  }
  if (which == 1) {
    if (n != size_t(n3)) {
      set_error("the loss-weight table has N^3 entries");
      return QCOLL_EINVAL;
    }
    if ((st = fetch<double>(p.lam, n, t)) != QCOLL_OK) return st;
    for (size_t k = 0; k < n; ++k) host[k] = t[k] * scale;
    return QCOLL_OK;
  }
  if (which == 2) {
    if (!p.lam_p) {
      set_error("per-node loss weights exist for untruncated VHS plans only");
      return QCOLL_ENOTSUP;
    }
    if (n != size_t(p.N_rho) * n3) {
      set_error("the per-node loss-weight table has N_rho * N^3 entries");
      return QCOLL_EINVAL;
    }
    if ((st = fetch<double>(p.lam_p, n, t)) != QCOLL_OK) return st;
    std::copy(t.begin(), t.end(), host);
    return QCOLL_OK;
  }
  set_error("unknown table");
  return QCOLL_EINVAL;
}

void plan_free(Plan &p) {
  free_kernel_tables(p);
  (void)hipFree(p.phase);
  (void)hipFree(p.wq);
  (void)hipFree(p.ginv);
  (void)hipFree(p.flag);
  p.phase = p.wq = nullptr;
  p.ginv = nullptr;
  p.flag = nullptr;
}

}  // namespace qcoll
