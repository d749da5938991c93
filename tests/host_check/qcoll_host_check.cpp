// Host-side exercise of libqcoll's validation layer, plan precompute, table
// read-back, autotune-cache parser, group and 1-D driver set-up, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code of the
// library's host-heavy sources (see paper_1809_10186_amd/build.py).  Needs one
// GPU (plans own device tables).  Prints "qcoll host check: ok" and exits 0 when
// every expectation holds; a sanitizer report aborts the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "qcoll.h"

static int g_fail = 0;

#define EXPECT(cond)                                                            \
  do {                                                                          \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, \
                   qcoll_last_error());                                         \
      ++g_fail;                                                                 \
    }                                                                           \
  } while (0)

static qcoll_params base(int N) {
  qcoll_params p;
  std::memset(&p, 0, sizeof p);
  p.N = N;
  p.L = 5.0;
  p.N_rho = 4;
  p.M = 6;
  p.sphere = nullptr;
  p.omega = 0.81;
  p.alpha = 1.0;
  p.prefactor = NAN;
  p.svd_rank = -1;
  p.svd_tol = 0.0;
  p.precision = QCOLL_FP64;
  p.nyquist = QCOLL_NYQ_SYMMETRIC;
  return p;
}

static void check_params() {
  qcoll_params p = base(8);
  EXPECT(qcoll_params_check(&p) == QCOLL_OK);
  EXPECT(qcoll_params_check(nullptr) == QCOLL_EINVAL);
  const int Ns[] = {-8, 0, 1, 7, 10, 20, 96, 1 << 20};
  for (int N : Ns) {
    p = base(N);
    EXPECT(qcoll_params_check(&p) != QCOLL_OK);
  }
  const double bad[] = {NAN, INFINITY, -INFINITY, -1.0, 0.0, 1e308};
  for (double x : bad) {
    p = base(8);
    p.L = x;
    if (!(x > 0 && std::isfinite(x))) EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
    p = base(8);
    p.omega = x;
    EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
    p = base(8);
    p.alpha = x;
    EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  }
  // sphere tables: wrong sums, non-unit points, NaN weights, M out of range
  std::vector<double> s(4 * 300, 0.0);
  for (int q = 0; q < 300; ++q) {
    s[4 * q + 2] = 1.0;
    s[4 * q + 3] = 2.0 * M_PI / 6.0;
  }
  p = base(8);
  p.sphere = s.data();
  p.M = 6;
  EXPECT(qcoll_params_check(&p) == QCOLL_OK);
  p.M = 0;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p.M = 257;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p.M = 5;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);   // weights do not sum to 2 pi
  s[3] = NAN;
  p.M = 6;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  s[3] = 2.0 * M_PI / 6.0;
  s[0] = 0.5;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p = base(8);
  p.svd_rank = 0;
  p.svd_tol = 0.0;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p.svd_rank = 99;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p = base(8);
  p.nyquist = 7;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  p = base(8);
  p.precision = -3;
  EXPECT(qcoll_params_check(&p) == QCOLL_EINVAL);
  for (int code = -1; code < 9; ++code) EXPECT(qcoll_status_str(qcoll_status(code)) != nullptr);
}

static void check_plan(const qcoll_params &prm) {
  qcoll_plan plan = nullptr;
  qcoll_plan bad = nullptr;
  EXPECT(qcoll_plan_create(&prm, 1 << 20, &bad) == QCOLL_EINVAL && bad == nullptr);
  EXPECT(qcoll_plan_create(&prm, -1, &plan) == QCOLL_OK);
  if (!plan) return;
  qcoll_plan_info_t info;
  EXPECT(qcoll_plan_info(plan, &info) == QCOLL_OK);
  std::vector<double> r(prm.N_rho), w(prm.N_rho);
  EXPECT(qcoll_plan_radial(plan, r.data(), w.data()) == QCOLL_OK);
  const size_t n3 = size_t(prm.N) * prm.N * prm.N;
  std::vector<double> t(size_t(prm.N_rho) * n3);
  const qcoll_status s0 = qcoll_plan_table(plan, 0, t.data(), t.size());
  EXPECT(s0 == (prm.alpha != 1.0 ? QCOLL_ENOTSUP : QCOLL_OK));
  EXPECT(qcoll_plan_table(plan, 0, t.data(), t.size() - 1) != QCOLL_OK);
  EXPECT(qcoll_plan_table(plan, 1, t.data(), n3) == QCOLL_OK);
  EXPECT(qcoll_plan_table(plan, 9, t.data(), n3) == QCOLL_EINVAL);
  for (int op = 0; op < 3; ++op)
    for (int64_t b : {int64_t(0), int64_t(1), int64_t(7), int64_t(1000)}) (void)qcoll_workspace_bytes(plan, b, op);
  EXPECT(qcoll_workspace_bytes(plan, -1, 0) == 0);
  EXPECT(qcoll_workspace_bytes(plan, 4, 5) == 0);
  for (int sch = -1; sch < 4; ++sch) (void)qcoll_plan_set_schedule(plan, sch);
  EXPECT(qcoll_plan_set_schedule(plan, 0) == QCOLL_OK);
  EXPECT(qcoll_plan_set_chunk(plan, -1) == QCOLL_EINVAL);
  EXPECT(qcoll_plan_set_chunk(plan, 5) == QCOLL_OK);
  if (prm.svd_rank < 0) {
    EXPECT(qcoll_plan_set_omega(plan, 0.7) == QCOLL_OK);
    EXPECT(qcoll_plan_set_omega(plan, 2.0) == QCOLL_EINVAL);
  } else {
    EXPECT(qcoll_plan_set_omega(plan, 0.7) == QCOLL_ENOTSUP);
  }
  // a small evaluation through the workspace entry point and the no-allocation one
  const int64_t batch = 3;
  double *f = nullptr, *Q = nullptr;
  void *ws = nullptr;
  const size_t wsb = qcoll_workspace_bytes(plan, batch, 0);
  if (hipMalloc(&f, batch * n3 * sizeof(double)) == hipSuccess && hipMalloc(&Q, batch * n3 * sizeof(double)) == hipSuccess &&
      hipMalloc(&ws, wsb) == hipSuccess) {
    std::vector<double> h(batch * n3);
    for (size_t i = 0; i < h.size(); ++i) h[i] = 1.0 + 0.01 * double(i % 97);
    (void)hipMemcpy(f, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
    EXPECT(qcoll_eval(plan, batch, f, Q, ws, wsb, nullptr) == QCOLL_OK);
    EXPECT(qcoll_eval(plan, batch, f, Q, ws, wsb - 1, nullptr) == QCOLL_EWORKSPACE);
    EXPECT(qcoll_eval(plan, batch, f, f, ws, wsb, nullptr) == QCOLL_EINVAL);
    EXPECT(qcoll_eval_noalloc(plan, batch, f, Q, nullptr) == QCOLL_OK);
    EXPECT(qcoll_conserve(plan, batch, Q, nullptr, nullptr) == QCOLL_OK);
    EXPECT(qcoll_poll(plan) == QCOLL_OK);
  } else {
    EXPECT(false);
  }
  (void)hipFree(f);
  (void)hipFree(Q);
  (void)hipFree(ws);
  EXPECT(qcoll_plan_destroy(plan) == QCOLL_OK);
}

static void check_autotune_cache(const char *path) {
  qcoll_params prm = base(8);
  prm.precision = QCOLL_FP32;
  qcoll_plan plan = nullptr;
  EXPECT(qcoll_plan_create(&prm, -1, &plan) == QCOLL_OK);
  if (!plan) return;
  // malformed and hostile lines around one valid entry for this plan's key
  FILE *fp = std::fopen(path, "w");
  if (!fp) {
    EXPECT(false);
    return;
  }
  std::fprintf(fp, "\n|\n||||\ngfx950 s2 N=8|\ngfx950 s2 N=8 Nr=4 M=6 prec=1 rank=4 batch<=4|x y\n");
  std::fprintf(fp, "gfx950 s2 N=8 Nr=4 M=6 prec=1 rank=4 batch<=4|999999999999999999999 3\n");
  std::string longline(100000, 'z');
  std::fprintf(fp, "%s|1 2\n", longline.c_str());
  std::fprintf(fp, "gfx950 s2 N=8 Nr=4 M=6 prec=1 rank=4 batch<=4|1 3 0.1\n");
  std::fclose(fp);
  setenv("QCOLL_AUTOTUNE_CACHE", path, 1);
  const int64_t batch = 3;
  const size_t n3 = 512;
  double *f = nullptr, *Q = nullptr;
  void *ws = nullptr;
  const size_t wsb = qcoll_autotune_workspace_bytes(plan, batch);
  if (hipMalloc(&f, batch * n3 * sizeof(double)) == hipSuccess && hipMalloc(&Q, batch * n3 * sizeof(double)) == hipSuccess &&
      hipMalloc(&ws, wsb) == hipSuccess) {
    (void)hipMemset(f, 0, batch * n3 * sizeof(double));
    int32_t sch = -1, ck = -1;
    EXPECT(qcoll_autotune(plan, batch, f, Q, ws, wsb, nullptr, &sch, &ck) == QCOLL_OK);
    EXPECT(sch == 1 && ck == 3);   // the valid line
    EXPECT(qcoll_autotune(plan, batch, f, Q, ws, 1, nullptr, &sch, &ck) == QCOLL_EWORKSPACE);
  } else {
    EXPECT(false);
  }
  unsetenv("QCOLL_AUTOTUNE_CACHE");
  (void)hipFree(f);
  (void)hipFree(Q);
  (void)hipFree(ws);
  // groups and the 1-D driver: argument errors and a create/destroy cycle
  qcoll_group g = nullptr;
  int64_t counts[2] = {2, 0};
  qcoll_plan plans[2] = {plan, plan};
  EXPECT(qcoll_group_create(plans, counts, 0, &g) == QCOLL_EINVAL);
  counts[1] = -1;
  EXPECT(qcoll_group_create(plans, counts, 2, &g) == QCOLL_EINVAL);
  counts[1] = 1;
  EXPECT(qcoll_group_create(plans, counts, 2, &g) == QCOLL_OK);
  (void)qcoll_group_workspace_bytes(g, 0);
  (void)qcoll_group_workspace_bytes(g, 7);
  EXPECT(qcoll_group_destroy(g) == QCOLL_OK);
  double faces[4] = {0.0, 0.5, 0.25, 1.0};
  qcoll_dg1d_params dp;
  std::memset(&dp, 0, sizeof dp);
  dp.n_elem = 3;
  dp.faces = faces;
  dp.order = 2;
  dp.inv_kn = 1.0;
  qcoll_dg1d d = nullptr;
  EXPECT(qcoll_dg1d_create(plan, &dp, &d) == QCOLL_EINVAL);   // faces not increasing
  faces[2] = 0.75;
  dp.order = 99;
  EXPECT(qcoll_dg1d_create(plan, &dp, &d) == QCOLL_EINVAL);
  dp.order = 2;
  EXPECT(qcoll_dg1d_create(plan, &dp, &d) == QCOLL_OK);
  EXPECT(qcoll_dg1d_destroy(d) == QCOLL_OK);
  EXPECT(qcoll_plan_destroy(plan) == QCOLL_OK);
}

int main(int argc, char **argv) {
  check_params();
  qcoll_params p = base(8);
  check_plan(p);
  p.precision = QCOLL_FP32;
  check_plan(p);
  p = base(12);
  p.svd_rank = 0;
  p.svd_tol = 1e-6;
  p.N_rho = 8;
  check_plan(p);
  p = base(8);
  p.alpha = 1.5;
  check_plan(p);
  p = base(8);
  p.nyquist = QCOLL_NYQ_LITERAL;
  check_plan(p);
  check_autotune_cache(argc > 1 ? argv[1] : "qcoll_host_check_cache.txt");
  if (g_fail) {
    std::printf("qcoll host check: %d failures\n", g_fail);
    return 1;
  }
  std::printf("qcoll host check: ok\n");
  return 0;
}
