// Internal plan object and the launchers behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "qcoll.h"

namespace qcoll {

void set_error(const std::string &msg);
// Diagnostics on stderr when the environment variable QCOLL_LOG is set to a
// non-empty value other than "0" (read once): plan creation, schedule and
// chunk choices, autotuner results, group graph captures, argument errors.
bool log_on();
void log(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

struct Plan {
  int device = 0;
  int N = 0, N_rho = 0, M = 0, rank = 0, precision = 0;
  int nv = 0;                    // rows of V / U the kernels use (rank, or N_rho when the mix saves nothing)
  double L = 0, R = 0, omega = 0, b = 0;
  double vss = 1.0;              // VSS scattering exponent alpha (1: VHS, sigma-independent kernel modes)
  bool literal = false;          // literal Nyquist convention: complex shift factor at frequency -N/2
  bool b_follows_omega = true;
  bool truncated = false;        // SVD truncation requested (any svd_rank >= 0)
  bool mix_identity = true;      // B_s = A_s (no SVD rotation)
  int schedule = 0;              // hot-loop schedule: 0 auto, 1 two-pass, 2 fused
  int schedule_user = 0;         // the schedule last requested through the API (the autotuner leaves it)
  int chunk = 0;                 // items per eval chunk (0: default 64)
  uint64_t gen = 0;              // bumped whenever tables, schedule or chunk change (keys cached graphs)
  double sigma_max = 0, sigma_min_kept = 0;

  std::vector<double> rho, w_rho;          // radial rule
  std::vector<double> sphere;              // [M][4]
  std::vector<double> umix;                // [rank][N_rho] (rotation rows kept)

  // device tables, element type = working precision T (float or double)
  void *phase = nullptr;   // [N_rho*M][3][N] complex: per-axis shift factors b_d(n)
  void *wq = nullptr;      // [M] half-sphere weights
  void *V = nullptr;       // [2*npair][N^3] real: spectral factors of the gain / N^3 (zero-padded row)
  double *V64 = nullptr;   // FP32 plans: the same rows in FP64 (two-pass low-rank stage); FP64 plans: NULL, V is FP64
  const double *v64() const { return precision == QCOLL_FP32 ? V64 : static_cast<const double *>(V); }
  void *lam = nullptr;     // [N^3] loss weights / N^3, always FP64
  void *alpha_eff = nullptr;  // [N_rho][N^3] effective gain weights sum_s U_sp V_s / N^3 (fused schedule)
  void *alpha_pq = nullptr;   // VSS: [N_rho][M][(N/2+1) N^2] gain weights 2 w_p w_q F(k, rho_p, sigma_q) / N^3,
                              // planes k1 <= N/2 (the weights are even in k)
  void *umix_d = nullptr;  // [rank][N_rho]
  // FP64 device tables
  double *ginv = nullptr;  // [25] (C C^T)^{-1} of the collision invariants on the grid
  double *lam_p = nullptr; // [N_rho][N^3] per-node loss weights (untruncated plans; omega gradient)
  double *dlog = nullptr;  // [N_rho] d ln(b rho_p^{4-2 omega}) / d omega
  int *flag = nullptr;     // non-finite flag

  int npair() const { return (nv + 1) / 2; }
  bool is_vss() const { return vss != 1.0; }
  long n3() const { return long(N) * N * N; }
};

// workspace layout for one call; sizes in bytes, offsets 256-aligned
// blocks per item of the VJP conservation projection (one partial-moment row
// each) and of the loss part of its omega gradient (one row of N_rho sums each)
constexpr int kProjSeg = 16;
constexpr int kDomSeg = 16;

struct Layout {
  long bc = 0;          // items per chunk
  long pc = 0;          // eval: (item, radial node) pairs per hot-loop launch; vjp: items per sub-chunk
  size_t off_h = 0, off_h64 = 0, off_a = 0, off_b = 0, off_w = 0, off_t = 0, off_l = 0, off_y = 0;
  size_t off_g = 0, off_z = 0, off_hp = 0, off_d = 0, off_pm = 0, off_dp = 0;  // vjp extras
  size_t off_pd = 0;                                    // two-pass vjp: per-pencil omega-gradient parts
  size_t off_yh = 0;                                    // two-pass VSS vjp: paired h_pq volumes
  size_t off_vp = 0;                                    // two-pass VSS eval: partial half spectra
  size_t off_hg = 0, off_h64g = 0, off_yg = 0;          // bilinear extras
  size_t total = 0;
};

// chunk > 0 overrides the plan's items per eval chunk (op 0 and 2)
Layout make_layout(const Plan &p, int64_t batch, int op, long chunk = 0);

// isc: optional device array of K per-item weights; item i of the call is
// stored scaled by isc[i % K] (the collocated DG weak form)
qcoll_status launch_eval(const Plan &p, int64_t batch, const double *f, double *Q, void *ws,
                         const Layout &lay, hipStream_t st, const double *isc = nullptr, int K = 0);
qcoll_status launch_eval2(const Plan &p, int64_t batch, const double *f, const double *g, double *Q, void *ws,
                          const Layout &lay, hipStream_t st);
qcoll_status launch_conserve(const Plan &p, int64_t batch, double *Q, double *mom, hipStream_t st,
                             const double *isc = nullptr, int K = 0);
qcoll_status launch_moments(const Plan &p, int64_t batch, const double *f, double *out,
                            hipStream_t st);
qcoll_status launch_vjp(const Plan &p, int64_t batch, const double *f, const double *g,
                        double *df, double *domega, bool through_conserve, void *ws, const Layout &lay,
                        hipStream_t st);

bool supported_N(int N);
void gauss_legendre(int n, double a, double b, std::vector<double> &x, std::vector<double> &w);
qcoll_status launch_dg_contract(const double *A, const double *X, double *Y, long E, int rows, int cols, long n3,
                                hipStream_t st);
bool fused_gain_supported(int N, int precision);
bool use_fused_gain(const Plan &p);
qcoll_status launch_gain_fused(const Plan &p, const void *H, void *W, long nbp, hipStream_t st);
// FP64 gain loop on chip (N = 16): A_p of every (item, node) pair
bool gain_q64_supported(int N, int precision);
bool use_gain_q64(const Plan &p);
qcoll_status launch_gain_q64(const Plan &p, const void *H, double *A, long nbp, hipStream_t st);
// schedule 2 exists for this grid and precision (FP32 fused kernel or FP64 on-chip gain)
inline bool onchip_schedule_supported(int N, int precision) {
  return fused_gain_supported(N, precision) || gain_q64_supported(N, precision);
}
inline bool onchip_schedule_supported(const Plan &p) {
  return !p.literal && onchip_schedule_supported(p.N, p.precision);
}
// sum over the N_rho per-node spectra of each item (FP32 complex, float4 units)
void launch_sum_nodes(const void *W, void *out, long nitems, int Nr, long n_in, long n_out, hipStream_t st);
// fused gain adjoint of the VJP (FP32, N <= 32, VHS kernels)
bool use_fused_adjoint(const Plan &p);
// two-pass VJP: the largest item count whose adjoint accumulation launch fits
// the device's resident workgroups in one round (0 if the query fails)
long adj_acc_items_per_round(const Plan &p);
// H, G: FP32 spectra of f and g; Hp: scratch for h_p = C_p g (formed on chip)
qcoll_status launch_adjoint_fused(const Plan &p, const void *H, const void *G, float *Hp, void *Zh, double *dwg,
                                  long nbp, hipStream_t st);

// kernel timing (hipEvents on the launch stream) for roofline accounting
bool timing_on();
void timing_begin(const char *name, hipStream_t st);
void timing_end(const char *name, hipStream_t st);

struct TimedLaunch {
  const char *name;
  hipStream_t st;
  bool on;
  TimedLaunch(const char *n, hipStream_t s) : name(n), st(s), on(timing_on()) {
    if (on) timing_begin(name, st);
  }
  ~TimedLaunch() {
    if (on) timing_end(name, st);
  }
};

}  // namespace qcoll

struct qcoll_plan_s {
  qcoll::Plan p;
};
