// C ABI: argument validation, plan lifetime and dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "qcoll_internal.h"

namespace qcoll {
qcoll_status plan_build(Plan &p, const qcoll_params &prm);
qcoll_status plan_set_omega(Plan &p, double omega);
qcoll_status plan_table(const Plan &p, int which, double *host, size_t n);
void plan_free(Plan &p);

static thread_local std::string g_err;
void set_error(const std::string &msg) {
  g_err = msg;
  if (log_on()) log("error: %s", msg.c_str());
}

bool log_on() {
  static const bool on = [] {
    const char *e = std::getenv("QCOLL_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}

void log(const char *fmt, ...) {
  if (!log_on()) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[qcoll] %s\n", buf);
}
}  // namespace qcoll

using qcoll::set_error;

namespace {

qcoll_status fail(qcoll_status s, const std::string &msg) {
  set_error(msg);
  return s;
}

qcoll_status check_device(const qcoll::Plan &p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(QCOLL_EDEVICE, "hipGetDevice failed");
  if (dev != p.device) return fail(QCOLL_EINVAL, "current device differs from the plan's device");
  return QCOLL_OK;
}

}  // namespace

extern "C" {

int32_t qcoll_version(void) { return 1; }

const char *qcoll_status_str(qcoll_status s) {
  // C callers may pass any int: read it as one (no load of an out-of-range enum)
  int v = 0;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case QCOLL_OK: return "QCOLL_OK";
    case QCOLL_EINVAL: return "QCOLL_EINVAL";
    case QCOLL_ENOTSUP: return "QCOLL_ENOTSUP";
    case QCOLL_ENOMEM: return "QCOLL_ENOMEM";
    case QCOLL_EDEVICE: return "QCOLL_EDEVICE";
    case QCOLL_EWORKSPACE: return "QCOLL_EWORKSPACE";
    case QCOLL_ENONFINITE: return "QCOLL_ENONFINITE";
  }
  return "QCOLL_<unknown>";
}

const char *qcoll_last_error(void) { return qcoll::g_err.c_str(); }

qcoll_status qcoll_params_check(const qcoll_params *p) {
  if (!p) return fail(QCOLL_EINVAL, "params is NULL");
  if (!(p->N > 0) || p->N % 2) return fail(QCOLL_EINVAL, "N must be a positive even integer");
  if (!qcoll::supported_N(p->N)) return fail(QCOLL_ENOTSUP, "N must be one of 8, 12, 16, 24, 32, 48, 64");
  if (p->N == 64 && p->alpha != 1.0) return fail(QCOLL_ENOTSUP, "VSS kernels support N <= 48");
  if (!(p->L > 0.0) || !std::isfinite(p->L)) return fail(QCOLL_EINVAL, "L must be finite and > 0");
  if (p->N_rho < 1) return fail(QCOLL_EINVAL, "N_rho must be >= 1");
  if (p->N_rho > 64) return fail(QCOLL_ENOTSUP, "N_rho must be <= 64");
  if (!(p->omega >= 0.5 && p->omega <= 1.0)) return fail(QCOLL_EINVAL, "omega must lie in [0.5, 1]");
  if (!(p->alpha >= 1.0 && p->alpha <= 2.0)) return fail(QCOLL_EINVAL, "alpha must lie in [1, 2] (1: VHS, > 1: VSS)");
  if (p->alpha != 1.0 && p->svd_rank >= 0)
    return fail(QCOLL_ENOTSUP, "VSS plans keep the full kernel-mode table (svd_rank < 0)");
  if (std::isinf(p->prefactor)) return fail(QCOLL_EINVAL, "prefactor must be finite (or NaN/<= 0 for the VHS constant)");
  if (p->precision != QCOLL_FP64 && p->precision != QCOLL_FP32) return fail(QCOLL_EINVAL, "unknown precision");
  if (p->nyquist != QCOLL_NYQ_SYMMETRIC && p->nyquist != QCOLL_NYQ_LITERAL)
    return fail(QCOLL_EINVAL, "nyquist must be QCOLL_NYQ_SYMMETRIC or QCOLL_NYQ_LITERAL");
  if (p->nyquist == QCOLL_NYQ_LITERAL && p->alpha != 1.0)
    return fail(QCOLL_ENOTSUP, "the literal Nyquist convention needs a VHS kernel (alpha = 1)");
  if (p->svd_rank == 0 && !(p->svd_tol > 0.0 && p->svd_tol < 1.0))
    return fail(QCOLL_EINVAL, "svd_rank == 0 needs 0 < svd_tol < 1");
  if (p->svd_rank > p->N_rho) return fail(QCOLL_EINVAL, "svd_rank must be <= N_rho");
  if (p->sphere) {
    if (p->M < 1 || p->M > 256) return fail(QCOLL_EINVAL, "M must be in 1..256");
    double wsum = 0.0;
    for (int q = 0; q < p->M; ++q) {
      const double *s = p->sphere + 4 * q;
      const double n = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
      if (!(std::fabs(n - 1.0) < 1e-12)) return fail(QCOLL_EINVAL, "sphere points must be unit vectors");
      if (!(s[3] > 0.0)) return fail(QCOLL_EINVAL, "sphere weights must be > 0");
      wsum += s[3];
    }
    if (!(std::fabs(wsum - 2.0 * M_PI) < 1e-10))
      return fail(QCOLL_EINVAL, "half-sphere weights must sum to 2*pi");
  } else if (!(p->M == 6 || p->M == 0)) {
    return fail(QCOLL_EINVAL, "sphere is NULL: only the built-in M = 6 rule is available");
  }
  return QCOLL_OK;
}

qcoll_status qcoll_plan_create(const qcoll_params *prm, int32_t device, qcoll_plan *out) {
  if (!out) return fail(QCOLL_EINVAL, "out is NULL");
  qcoll_status st = qcoll_params_check(prm);
  if (st != QCOLL_OK) return st;
  int prev = -1, ndev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipGetDeviceCount(&ndev) != hipSuccess)
    return fail(QCOLL_EDEVICE, "no HIP device");
  if (device >= ndev) return fail(QCOLL_EINVAL, "device index out of range");
  // build with the requested device current, then give the caller back its own
  struct Restore {
    int dev;
    bool on;
    ~Restore() {
      if (on) (void)hipSetDevice(dev);
    }
  } restore{prev, device >= 0 && device != prev};
  if (restore.on && hipSetDevice(device) != hipSuccess) {
    restore.on = false;
    return fail(QCOLL_EDEVICE, "hipSetDevice failed");
  }
  auto *h = new (std::nothrow) qcoll_plan_s;
  if (!h) return fail(QCOLL_ENOMEM, "host allocation failed");
  st = qcoll::plan_build(h->p, *prm);
  if (st != QCOLL_OK) {
    qcoll::plan_free(h->p);
    delete h;
    return st;
  }
  *out = h;
  const auto &p = h->p;
  qcoll::log("plan %p: N=%d L=%g N_rho=%d M=%d omega=%g alpha=%g b=%.10g rank=%d (sigma %.3e..%.3e) %s %s "
             "nyquist=%s device=%d",
             static_cast<void *>(h), p.N, p.L, p.N_rho, p.M, p.omega, p.vss, p.b, p.rank, p.sigma_max,
             p.sigma_min_kept, p.precision == QCOLL_FP32 ? "fp32" : "fp64", p.truncated ? "truncated" : "full",
             p.literal ? "literal" : "symmetric", p.device);
  return QCOLL_OK;
}

qcoll_status qcoll_plan_destroy(qcoll_plan plan) {
  if (!plan) return QCOLL_OK;
  qcoll::plan_free(plan->p);
  delete plan;
  return QCOLL_OK;
}

qcoll_status qcoll_plan_info(qcoll_plan plan, qcoll_plan_info_t *o) {
  if (!plan || !o) return fail(QCOLL_EINVAL, "NULL argument");
  const auto &p = plan->p;
  o->N = p.N;
  o->N_rho = p.N_rho;
  o->M = p.M;
  o->rank = p.rank;
  o->precision = p.precision;
  o->L = p.L;
  o->R = p.R;
  o->omega = p.omega;
  o->prefactor = p.b;
  o->sigma_max = p.sigma_max;
  o->sigma_min_kept = p.sigma_min_kept;
  return QCOLL_OK;
}

qcoll_status qcoll_plan_radial(qcoll_plan plan, double *rho, double *w) {
  if (!plan || !rho || !w) return fail(QCOLL_EINVAL, "NULL argument");
  for (int i = 0; i < plan->p.N_rho; ++i) {
    rho[i] = plan->p.rho[i];
    w[i] = plan->p.w_rho[i];
  }
  return QCOLL_OK;
}

qcoll_status qcoll_plan_table(qcoll_plan plan, int32_t which, double *host_out, size_t n) {
  if (!plan || !host_out) return fail(QCOLL_EINVAL, "NULL argument");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::plan_table(plan->p, which, host_out, n);
}

qcoll_status qcoll_plan_set_omega(qcoll_plan plan, double omega) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (!(omega >= 0.5 && omega <= 1.0)) return fail(QCOLL_EINVAL, "omega must lie in [0.5, 1]");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::plan_set_omega(plan->p, omega);
}

qcoll_status qcoll_plan_set_schedule(qcoll_plan plan, int32_t schedule) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (schedule < 0 || schedule > 2) return fail(QCOLL_EINVAL, "schedule must be 0, 1 or 2");
  if (schedule == 2 && !qcoll::onchip_schedule_supported(plan->p))
    return fail(QCOLL_ENOTSUP, "the on-chip gain kernels need FP32 with N <= 32 or FP64 with N = 16 or 32, "
                               "and the symmetric Nyquist convention");
  plan->p.schedule = schedule;
  plan->p.schedule_user = schedule;
  ++plan->p.gen;
  qcoll::log("plan %p: schedule %d", static_cast<void *>(plan), schedule);
  return QCOLL_OK;
}

size_t qcoll_workspace_bytes(qcoll_plan plan, int64_t batch, int32_t op) {
  if (!plan || batch < 0 || op < 0 || op > 2) return 0;
  return qcoll::make_layout(plan->p, batch, op).total;
}

qcoll_status qcoll_eval(qcoll_plan plan, int64_t batch, const double *f, double *Q, void *ws, size_t ws_bytes,
                        void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return fail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!f || !Q) return fail(QCOLL_EINVAL, "f and Q must be non-NULL");
  const long n3 = plan->p.n3();
  if ((const void *)f < (const void *)(Q + batch * n3) && (const void *)Q < (const void *)(f + batch * n3))
    return fail(QCOLL_EINVAL, "Q must not overlap f");
  const qcoll::Layout lay = qcoll::make_layout(plan->p, batch, 0);
  if (!ws || ws_bytes < lay.total) return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_workspace_bytes");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::launch_eval(plan->p, batch, f, Q, ws, lay, static_cast<hipStream_t>(stream));
}

qcoll_status qcoll_eval_bilinear(qcoll_plan plan, int64_t batch, const double *f, const double *g, double *Q,
                                 void *ws, size_t ws_bytes, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return fail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!f || !g || !Q) return fail(QCOLL_EINVAL, "f, g and Q must be non-NULL");
  if (plan->p.literal) return fail(QCOLL_ENOTSUP, "the bilinear Q needs the symmetric Nyquist convention");
  const long n3 = plan->p.n3();
  auto overlap = [&](const void *a) {
    return a < (const void *)(Q + batch * n3) && (const void *)Q < (const void *)((const double *)a + batch * n3);
  };
  if (overlap(f) || overlap(g)) return fail(QCOLL_EINVAL, "Q must not overlap f or g");
  const qcoll::Layout lay = qcoll::make_layout(plan->p, batch, 2);
  if (!ws || ws_bytes < lay.total) return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_workspace_bytes(op 2)");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::launch_eval2(plan->p, batch, f, g, Q, ws, lay, static_cast<hipStream_t>(stream));
}

qcoll_status qcoll_conserve(qcoll_plan plan, int64_t batch, double *Q, double *moments, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return fail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!Q) return fail(QCOLL_EINVAL, "Q must be non-NULL");
  if (reinterpret_cast<uintptr_t>(Q) % 16) return fail(QCOLL_EINVAL, "Q must be 16-byte aligned");
  if (batch > 0x7fffffff) return fail(QCOLL_EINVAL, "batch too large");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::launch_conserve(plan->p, batch, Q, moments, static_cast<hipStream_t>(stream));
}

qcoll_status qcoll_moments(qcoll_plan plan, int64_t batch, const double *f, double *out, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return fail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!f || !out) return fail(QCOLL_EINVAL, "f and out must be non-NULL");
  if (batch > 0x7fffffff) return fail(QCOLL_EINVAL, "batch too large");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::launch_moments(plan->p, batch, f, out, static_cast<hipStream_t>(stream));
}

qcoll_status qcoll_vjp(qcoll_plan plan, int64_t batch, const double *f, const double *g, double *df,
                       double *domega, int32_t through_conserve, void *ws, size_t ws_bytes, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return fail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!f || !g) return fail(QCOLL_EINVAL, "f and g must be non-NULL");
  if (plan->p.literal) return fail(QCOLL_ENOTSUP, "the VJP needs the symmetric Nyquist convention");
  if (plan->p.N > 48) return fail(QCOLL_ENOTSUP, "the VJP supports N <= 48");
  if (!df && !domega) return QCOLL_OK;
  if (domega && plan->p.truncated)
    return fail(QCOLL_ENOTSUP, "the omega gradient needs an untruncated plan (svd_rank < 0)");
  const qcoll::Layout lay = qcoll::make_layout(plan->p, batch, 1);
  if (!ws || ws_bytes < lay.total) return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_workspace_bytes");
  const long n3 = plan->p.n3();
  if (df && (((const void *)df < (const void *)(f + batch * n3) && (const void *)f < (const void *)(df + batch * n3)) ||
             ((const void *)df < (const void *)(g + batch * n3) && (const void *)g < (const void *)(df + batch * n3))))
    return fail(QCOLL_EINVAL, "df must not overlap f or g");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  return qcoll::launch_vjp(plan->p, batch, f, g, df, domega, through_conserve != 0, ws, lay,
                           static_cast<hipStream_t>(stream));
}

size_t qcoll_dg_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R) {
  if (!plan || n_elem < 0 || K < 1 || R < 1) return 0;
  const size_t n3 = size_t(plan->p.n3());
  const size_t terms = size_t(n_elem) * R;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return 2 * al(terms * n3 * sizeof(double)) + qcoll::make_layout(plan->p, int64_t(terms), 0).total;
}

qcoll_status qcoll_dg_collide(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R, const double *T,
                              const double *W, const double *F, double *C, int32_t conserve, void *ws,
                              size_t ws_bytes, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (n_elem < 0) return fail(QCOLL_EINVAL, "n_elem must be >= 0");
  if (K < 1 || K > 64 || R < 1 || R > 4096) return fail(QCOLL_EINVAL, "need 1 <= K <= 64 and 1 <= R <= 4096");
  if (n_elem == 0) return QCOLL_OK;
  if (!T || !W || !F || !C) return fail(QCOLL_EINVAL, "T, W, F and C must be non-NULL");
  const size_t n3 = size_t(plan->p.n3());
  const size_t terms = size_t(n_elem) * R;
  if (terms > size_t(0x7fffffff)) return fail(QCOLL_EINVAL, "n_elem * R too large");
  const size_t need = qcoll_dg_workspace_bytes(plan, n_elem, K, R);
  if (!ws || ws_bytes < need) return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_dg_workspace_bytes");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  char *w = static_cast<char *>(ws);
  double *Hd = reinterpret_cast<double *>(w);
  double *Qd = reinterpret_cast<double *>(w + al(terms * n3 * sizeof(double)));
  void *ews = w + 2 * al(terms * n3 * sizeof(double));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = qcoll::launch_dg_contract(T, F, Hd, n_elem, R, K, long(n3), s)) != QCOLL_OK) return st;
  const qcoll::Layout lay = qcoll::make_layout(plan->p, int64_t(terms), 0);
  if ((st = qcoll::launch_eval(plan->p, int64_t(terms), Hd, Qd, ews, lay, s)) != QCOLL_OK) return st;
  if (conserve && (st = qcoll::launch_conserve(plan->p, int64_t(terms), Qd, nullptr, s)) != QCOLL_OK) return st;
  return qcoll::launch_dg_contract(W, Qd, C, n_elem, K, R, long(n3), s);
}

size_t qcoll_dg_collocated_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K) {
  if (!plan || n_elem < 0 || K < 1 || K > 64) return 0;
  return 512 + qcoll::make_layout(plan->p, n_elem * K, 0).total;
}

namespace {
struct Weights {
  double w[64];
};

// the K collocation weights into device memory (kernel argument -> workspace)
__global__ void k_fill_weights(Weights wt, int K, double *out) {
#pragma unroll
  for (int k = 0; k < 64; ++k)
    if (k < K && int(threadIdx.x) == k) out[k] = wt.w[k];
}
}  // namespace

qcoll_status qcoll_dg_collide_collocated(qcoll_plan plan, int64_t n_elem, int32_t K, const double *host_w,
                                         const double *F, double *C, int32_t conserve, void *ws, size_t ws_bytes,
                                         void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (n_elem < 0) return fail(QCOLL_EINVAL, "n_elem must be >= 0");
  if (K < 1 || K > 64) return fail(QCOLL_EINVAL, "need 1 <= K <= 64");
  if (n_elem == 0) return QCOLL_OK;
  if (!host_w || !F || !C) return fail(QCOLL_EINVAL, "host_w, F and C must be non-NULL");
  const int64_t items = n_elem * K;
  if (items > 0x7fffffff) return fail(QCOLL_EINVAL, "n_elem * K too large");
  const long n3 = plan->p.n3();
  if ((const void *)F < (const void *)(C + items * n3) && (const void *)C < (const void *)(F + items * n3))
    return fail(QCOLL_EINVAL, "C must not overlap F");
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(host_w[k])) return fail(QCOLL_EINVAL, "collocation weights must be finite");
  if (!ws || ws_bytes < qcoll_dg_collocated_workspace_bytes(plan, n_elem, K))
    return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_dg_collocated_workspace_bytes");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *wd = static_cast<double *>(ws);
  Weights wt{};
  for (int k = 0; k < K; ++k) wt.w[k] = host_w[k];
  hipLaunchKernelGGL(k_fill_weights, dim3(1), dim3(64), 0, s, wt, int(K), wd);
  if (hipGetLastError() != hipSuccess) return fail(QCOLL_EDEVICE, "weight fill launch failed");
  void *ews = static_cast<char *>(ws) + 512;
  const qcoll::Layout lay = qcoll::make_layout(plan->p, items, 0);
  // Q of every (element, node) straight from F (T = I: no contraction), stored
  // scaled by its node weight (W diagonal), or projected first and scaled by
  // the projection (it is linear, so it commutes with the weight)
  if ((st = qcoll::launch_eval(plan->p, items, F, C, ews, lay, s, conserve ? nullptr : wd, K)) != QCOLL_OK)
    return st;
  if (conserve && (st = qcoll::launch_conserve(plan->p, items, C, nullptr, s, wd, K)) != QCOLL_OK) return st;
  return QCOLL_OK;
}

size_t qcoll_dg_svd_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R) {
  if (!plan || n_elem < 0 || K < 1 || R < 1) return 0;
  const size_t n3 = size_t(plan->p.n3());
  const size_t terms = size_t(n_elem) * R;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return 3 * al(terms * n3 * sizeof(double)) + qcoll::make_layout(plan->p, int64_t(terms), 2).total;
}

qcoll_status qcoll_dg_collide_svd(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R, const double *T1,
                                  const double *T2, const double *W, const double *F, double *C, int32_t conserve,
                                  void *ws, size_t ws_bytes, void *stream) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (n_elem < 0) return fail(QCOLL_EINVAL, "n_elem must be >= 0");
  if (K < 1 || K > 64 || R < 1 || R > 4096) return fail(QCOLL_EINVAL, "need 1 <= K <= 64 and 1 <= R <= 4096");
  if (n_elem == 0) return QCOLL_OK;
  if (!T1 || !T2 || !W || !F || !C) return fail(QCOLL_EINVAL, "T1, T2, W, F and C must be non-NULL");
  if (plan->p.literal) return fail(QCOLL_ENOTSUP, "the bilinear Q needs the symmetric Nyquist convention");
  const size_t n3 = size_t(plan->p.n3());
  const size_t terms = size_t(n_elem) * R;
  if (terms > size_t(0x7fffffff)) return fail(QCOLL_EINVAL, "n_elem * R too large");
  if (!ws || ws_bytes < qcoll_dg_svd_workspace_bytes(plan, n_elem, K, R))
    return fail(QCOLL_EWORKSPACE, "workspace missing or smaller than qcoll_dg_svd_workspace_bytes");
  qcoll_status st = check_device(plan->p);
  if (st != QCOLL_OK) return st;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t vol = al(terms * n3 * sizeof(double));
  char *w = static_cast<char *>(ws);
  double *Hf = reinterpret_cast<double *>(w);
  double *Hg = reinterpret_cast<double *>(w + vol);
  double *Qd = reinterpret_cast<double *>(w + 2 * vol);
  void *ews = w + 3 * vol;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = qcoll::launch_dg_contract(T1, F, Hf, n_elem, R, K, long(n3), s)) != QCOLL_OK) return st;
  if ((st = qcoll::launch_dg_contract(T2, F, Hg, n_elem, R, K, long(n3), s)) != QCOLL_OK) return st;
  const qcoll::Layout lay = qcoll::make_layout(plan->p, int64_t(terms), 2);
  if ((st = qcoll::launch_eval2(plan->p, int64_t(terms), Hf, Hg, Qd, ews, lay, s)) != QCOLL_OK) return st;
  if (conserve && (st = qcoll::launch_conserve(plan->p, int64_t(terms), Qd, nullptr, s)) != QCOLL_OK) return st;
  return qcoll::launch_dg_contract(W, Qd, C, n_elem, K, R, long(n3), s);
}

qcoll_status qcoll_poll(qcoll_plan plan) {
  if (!plan) return fail(QCOLL_EINVAL, "plan is NULL");
  if (hipDeviceSynchronize() != hipSuccess) return fail(QCOLL_EDEVICE, "hipDeviceSynchronize failed");
  int h = 0;
  if (hipMemcpy(&h, plan->p.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(QCOLL_EDEVICE, "hipMemcpy failed");
  if (h) {
    if (hipMemset(plan->p.flag, 0, sizeof(int)) != hipSuccess) return fail(QCOLL_EDEVICE, "hipMemset failed");
    return fail(QCOLL_ENONFINITE, "a non-finite value reached the moment sums");
  }
  return QCOLL_OK;
}

}  // extern "C"
