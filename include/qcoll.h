/*
 * qcoll: batched Boltzmann collision operator Q(f,f) by the fast Fourier
 * spectral method, for AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Jaiswal, Alexeenko and Hu, "A discontinuous
 * Galerkin fast spectral method for the full Boltzmann equation with general
 * collision kernels" (Appendix): f on a uniform N^3 velocity grid is
 * periodised on [-L, L]^3, the kernel modes G(l, m) are separated by a
 * Gauss-Legendre rule in the relative speed and a half-sphere design in the
 * scattering direction, and each separated term becomes an FFT convolution.
 * The library takes the grid values of f and returns the grid values of Q
 * (Section 3.3: the collision solver is a black box from grid values to grid
 * values).  The 1/Kn factor of the non-dimensional equation is NOT applied.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Velocity grid: c_j = -L + (j + 1/2) * 2L/N, j = 0..N-1 per axis.  An item
 *   is a C-order array [N][N][N] of doubles, index (j1, j2, j3) <-> (c1, c2, c3);
 *   a batch is [batch][N][N][N], contiguous.
 * - Pointers named f, g, Q, df, out, moments are DEVICE pointers on the device
 *   the plan was created on, owned by the caller, 16-byte aligned (an item of
 *   a batch starts 16-byte aligned whenever the batch does, N being even).  Host
 *   pointers are named as such.  Workspace (ws) is a caller-owned device
 *   buffer of at least qcoll_workspace_bytes() bytes, 256-byte aligned.
 * - stream is a hipStream_t (NULL = the default stream).  Every compute entry
 *   point is asynchronous on that stream; argument errors are detected before
 *   anything is enqueued and then nothing is enqueued.
 * - Boundary data are FP64 in both precisions; QCOLL_FP32 computes the
 *   transforms and products in FP32 and returns FP64.
 * - Nyquist mode (qcoll_params.nyquist): by default the DFT index N/2
 *   (frequency -N/2) is shifted as the cosine mode of the real trigonometric
 *   interpolant, factor cos(pi (N/2) s_d / L) per axis, so every intermediate
 *   of Q(f,f) is real; the literal convention is available per plan.
 * - Errors: a qcoll_status; qcoll_last_error() gives a thread-local detail
 *   string.  No exception, abort or exit crosses this interface.
 * - Concurrency: a plan is immutable after creation (except through
 *   qcoll_plan_set_omega) and may be used from several streams at once if
 *   each stream has its own workspace.
 */
#ifndef QCOLL_H
#define QCOLL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcoll_plan_s *qcoll_plan;
typedef struct qcoll_group_s *qcoll_group;

typedef enum {
  QCOLL_OK = 0,
  QCOLL_EINVAL = 1,     /* invalid argument */
  QCOLL_ENOTSUP = 2,    /* valid for the method, not supported by this build */
  QCOLL_ENOMEM = 3,     /* device or host allocation failed */
  QCOLL_EDEVICE = 4,    /* a HIP call or a kernel launch failed */
  QCOLL_EWORKSPACE = 5, /* workspace missing or too small */
  QCOLL_ENONFINITE = 6  /* a non-finite value reached the moment sums */
} qcoll_status;

typedef enum { QCOLL_FP64 = 0, QCOLL_FP32 = 1 } qcoll_precision;

/* Plan parameters.
 *   N          points per velocity axis; supported: 8, 12, 16, 24, 32, 48, 64
 *              (64: symmetric or literal VHS plans, no VJP).
 *   L          half-width of the periodic velocity box [-L, L]^3, L > 0.
 *   N_rho      Gauss-Legendre nodes of the radial rule on [0, R],
 *              R = 4L/(3 + sqrt 2) (Appendix: ball truncation); 1..64.
 *   M          points of the half-sphere rule (Appendix: spherical design).
 *   sphere     HOST pointer to [M][4] doubles (x, y, z, weight), unit vectors
 *              with one point per antipodal pair and weights summing to
 *              2*pi; NULL selects the built-in M = 6 rule (one vertex of each
 *              antipodal pair of the regular icosahedron, weights 2*pi/6).
 *   omega      viscosity index, B = b |g|^{2(1-omega)} (1 + cos chi)^{alpha-1}
 *              (Section 2, general kernel); 0.5 <= omega <= 1.
 *   alpha      VSS scattering exponent, 1 <= alpha <= 2.  alpha = 1 is the VHS
 *              kernel (kernel modes independent of sigma).  alpha > 1 makes the
 *              kernel modes F(k, rho_p, sigma_q) depend on the sphere point
 *              (Appendix, F with the kernel symmetrised in cos chi): every
 *              (rho_p, sigma_q) term is then transformed forward and weighted
 *              on its own, about twice the work of alpha = 1.  VSS plans need
 *              svd_rank < 0 and N <= 48.
 *   prefactor  kernel constant b; a value <= 0 or NaN selects the
 *              non-dimensional constant alpha / (2^{2-omega+alpha}
 *              Gamma(2.5-omega) pi) (Section 2.1; 1/(2^{3-omega} Gamma(2.5-omega)
 *              pi) for VHS); the BKW case uses 1/(4 pi).
 *   svd_rank   truncation of the gain-weight table alpha_p(k) = 2 w_p F(k, rho_p)
 *              (rows p) by its SVD: < 0 keeps the full table exactly (no
 *              SVD); > 0 keeps that many singular triplets; 0 keeps those
 *              with sigma_i > svd_tol * sigma_1.
 *   svd_tol    relative truncation threshold used when svd_rank == 0.
 *   precision  qcoll_precision.
 *   nyquist    qcoll_nyquist: how the shift acts on the self-paired DFT index
 *              N/2 (Appendix: the index set k = -N/2 .. N/2 - 1).  SYMMETRIC
 *              takes the real interpolant's cosine factor cos(pi (N/2) s_d / L)
 *              (every intermediate real; the default and the fast path).
 *              LITERAL takes exp(i pi k s_d / L) at k = -N/2 as printed: the
 *              shifted copies t1, t2 and the gain are complex and Q is the real
 *              part.  LITERAL plans run the two-pass schedule with two inverse
 *              transforms per term; qcoll_vjp, qcoll_eval_bilinear and
 *              qcoll_dg_collide_svd return ENOTSUP for them.
 */
typedef enum { QCOLL_NYQ_SYMMETRIC = 0, QCOLL_NYQ_LITERAL = 1 } qcoll_nyquist;

typedef struct {
  int32_t N;
  double L;
  int32_t N_rho;
  int32_t M;
  const double *sphere;
  double omega;
  double alpha;
  double prefactor;
  int32_t svd_rank;
  double svd_tol;
  int32_t precision;
  int32_t nyquist;
} qcoll_params;

/* Plan facts for diagnostics; filled by qcoll_plan_info. */
typedef struct {
  int32_t N, N_rho, M, rank, precision;
  double L, R, omega, prefactor;
  double sigma_max, sigma_min_kept; /* singular values of the gain table (0 if no SVD) */
} qcoll_plan_info_t;

/* Validate parameters without touching any device.  QCOLL_OK, EINVAL or ENOTSUP. */
qcoll_status qcoll_params_check(const qcoll_params *p);

/* Build a plan on HIP device `device` (< 0: the current device): quadratures,
 * kernel-mode tables (Appendix, quadrature form of G), per-axis shift tables,
 * optional SVD, all in FP64 on the host, then copied to device memory owned by
 * the plan.  The caller's current device is left as it was.  Every later call
 * with the plan must run with that device current (EINVAL otherwise).
 * *out is set only on success; EINVAL for a device index out of range. */
qcoll_status qcoll_plan_create(const qcoll_params *p, int32_t device, qcoll_plan *out);

/* Free the plan and its device tables.  The caller must have synchronised
 * every stream that used it.  NULL is accepted. */
qcoll_status qcoll_plan_destroy(qcoll_plan plan);

qcoll_status qcoll_plan_info(qcoll_plan plan, qcoll_plan_info_t *host_out);

/* Copy the radial rule (HOST arrays of N_rho doubles each). */
qcoll_status qcoll_plan_radial(qcoll_plan plan, double *host_rho, double *host_w);

/* Copy one of the plan's kernel-mode tables from the device into a HOST
 * array of exactly n doubles, in FP64 and without the 1/N^3 normalisation
 * the kernels fold in (Appendix, quadrature form of G):
 *   which 0: gain weights alpha_p(k) = 2 w_p F(k, rho_p), [N_rho][N^3] in DFT
 *            index order (after SVD truncation, the truncated table
 *            sum_s U_sp V_s(k)); ENOTSUP for VSS plans;
 *   which 1: loss weights Lambda(k) = 2 sum_{p,q} w_p w_q F(2k, rho_p), [N^3];
 *   which 2: per-node loss weights Lambda_p(k) (their sum over p is Lambda),
 *            [N_rho][N^3]; untruncated VHS plans only (else ENOTSUP).
 * Tables of FP32 plans are stored in FP32 and come back widened.  EINVAL if
 * n does not match the table.  Synchronous. */
qcoll_status qcoll_plan_table(qcoll_plan plan, int32_t which, double *host_out, size_t n);

/* Change omega (and the prefactor if it follows omega) of an untruncated
 * plan; rebuilds the kernel tables synchronously.  ENOTSUP for truncated plans. */
qcoll_status qcoll_plan_set_omega(qcoll_plan plan, double omega);

/* Hot-loop schedule: 0 = automatic (on-chip kernel where it is available:
 * FP32 with N <= 32, FP64 with N = 16 or 32; otherwise two passes over HBM),
 * 1 = force the two-pass schedule, 2 = require the on-chip kernel (ENOTSUP
 * where it is not available).  Results agree to rounding; workspace sizes depend on it.
 * The schedule requested here also selects the gain adjoint of qcoll_vjp
 * (fused unless 1 was requested; the autotuner's choice of the forward
 * schedule does not change it). */
qcoll_status qcoll_plan_set_schedule(qcoll_plan plan, int32_t schedule);

/* Workspace needed by op 0 (qcoll_eval), 1 (qcoll_vjp) or 2 (qcoll_eval_bilinear)
 * for this batch. */
size_t qcoll_workspace_bytes(qcoll_plan plan, int64_t batch, int32_t op);

/* Q(f,f) for every item (Appendix):
 *   Q = sum_p C_p [ sum_q w_q t1_pq t2_pq ] - f * Lam~ f,
 * t1 = f^N(c + rho_p sigma_q / 2), t2 = f^N(c - rho_p sigma_q / 2) evaluated
 * spectrally, C_p the Fourier multiplier by alpha_p (or its truncation),
 * Lam~ the multiplier by the loss weights G(m, m).
 * f: [batch][N^3] input; Q: [batch][N^3] output (may not alias f).
 * batch == 0 is a no-op. */
qcoll_status qcoll_eval(qcoll_plan plan, int64_t batch, const double *f, double *Q,
                        void *ws, size_t ws_bytes, void *stream);

/* qcoll_eval for callers that cannot allocate device memory or pass a
 * workspace: code under hipGraph stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same result as qcoll_eval (same kernels;
 * every item's result is independent of the chunking).  The scratch is one
 * static device array of 256 MiB, one copy per GPU the library runs on, held
 * until the process ends; the batch runs in chunks whose workspace fits it
 * (at most the plan's chunk).  Calls no allocator.  EWORKSPACE if a single
 * item of this plan needs more scratch than the array holds.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (different
 * streams or threads without ordering between them) race and give undefined
 * results; order them on one stream. */
qcoll_status qcoll_eval_noalloc(qcoll_plan plan, int64_t batch, const double *f, double *Q, void *stream);

/* Bilinear collision operator Q(f, g) (Appendix: the operator form
 * Q(f,g) = int int B_sym [f(c') g(c'_*) - f(c) g(c_*)] evaluated with the same
 * quadrature form of the kernel modes): per (rho_p, sigma_q) the gain takes
 * (t1_f t2_g + t2_f t1_g) / 2 (for VSS kernels each term's product is weighted
 * by its own alpha_pq after its transform), the loss is f * Lam~ g.  Q(f, f)
 * equals qcoll_eval.  Two inverse transforms per term (two-pass schedule in both
 * precisions).  f, g, Q: [batch][N^3]; workspace: qcoll_workspace_bytes(op 2).
 * ENOTSUP for literal-Nyquist plans. */
qcoll_status qcoll_eval_bilinear(qcoll_plan plan, int64_t batch, const double *f, const double *g,
                                 double *Q, void *ws, size_t ws_bytes, void *stream);

/* FP64 conservation projection, in place:
 *   Q <- Q - C^T (C C^T)^{-1} C Q,  rows of C = 1, c1, c2, c3, |c|^2 on the grid,
 * the nearest grid function (Euclidean) with zero discrete mass, momentum and
 * energy production.  Not part of the paper's method.
 * moments: [batch][5] device output of the pre-projection sums
 * sum_j Q_j phi_i(c_j) dc^3, or NULL.  Non-finite sums raise a device flag
 * reported by qcoll_poll. */
qcoll_status qcoll_conserve(qcoll_plan plan, int64_t batch, double *Q, double *moments,
                            void *stream);

/* Midpoint-rule moments (Section 3.3): out [batch][14] =
 * n, u1, u2, u3, T, P11, P12, P13, P22, P23, P33, q1, q2, q3 of the
 * non-dimensional definitions. */
qcoll_status qcoll_moments(qcoll_plan plan, int64_t batch, const double *f, double *out,
                           void *stream);

/* Vector-Jacobian product of Q(f,f) with cotangent g:
 *   df = J_f^T g  ([batch][N^3], may be NULL),
 *   domega[b] = g_b . dQ(f_b)/d omega ([batch], may be NULL; needs an
 *   untruncated plan, else ENOTSUP).
 * VHS and VSS kernels (VSS: the two-pass adjoint, one inverse transform of
 * alpha_pq g^ per sphere point); N <= 48, symmetric Nyquist convention.
 * through_conserve != 0 differentiates the projected operator (g is first
 * projected; the projection is symmetric).  Not part of the paper's method. */
qcoll_status qcoll_vjp(qcoll_plan plan, int64_t batch, const double *f, const double *g,
                       double *df, double *domega, int32_t through_conserve,
                       void *ws, size_t ws_bytes, void *stream);

/* Per-kernel timing for roofline accounting.  While enabled, every kernel
 * launch is bracketed by a pair of hipEvents recorded on its own stream, keyed
 * by the kernel's role name ("gain slab", "gain pencil", ...).  Process-wide;
 * not thread-safe while enabled.
 * qcoll_timing_read synchronises the recorded events and returns the summed
 * duration (ms) and launch count for one name (0 and 0 if never launched);
 * qcoll_timing_names writes a '\n'-separated list of the names seen into a
 * HOST buffer of cap bytes (truncated, NUL-terminated).
 * qcoll_timing_select restricts the events to one role (a HOST string,
 * copied; NULL or "" = every role), so that a timed region can carry the
 * events of its dominant kernel only.  qcoll_timing_reset keeps the event
 * objects for reuse, so launches after the first round create none. */
qcoll_status qcoll_timing_enable(int32_t on);
qcoll_status qcoll_timing_select(const char *host_name);
qcoll_status qcoll_timing_reset(void);
qcoll_status qcoll_timing_read(const char *name, double *host_ms, int64_t *host_count);
qcoll_status qcoll_timing_names(char *host_buf, size_t cap);

/* DG collision term of the weak form (Section 3.3.1, the collision double sum
 * and its SVD variant):
 *   C[e][m] = sum_r W[m][r] Q( sum_l T[r][l] F[e][l] ),   m < K, r < R,
 * for every element e.  With T the stacked eigenvectors u_{m,r} of the
 * symmetric triple-tensor slices H_m and W[m][(m,r)] their eigenvalues this
 * is sum_{l1,l2} H_{m l1 l2} Q(F_l1, F_l2); with T the basis values at
 * quadrature points and W the weighted basis values it is the quadrature
 * form.  The two contractions run on MFMA (FP64).
 *   T: [R][K], W: [K][R] device FP64; F, C: [n_elem][K][N^3] device FP64.
 *   conserve != 0 applies qcoll_conserve to every Q term before W.
 * Workspace from qcoll_dg_workspace_bytes (includes the eval workspace). */
size_t qcoll_dg_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R);
qcoll_status qcoll_dg_collide(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R, const double *T,
                              const double *W, const double *F, double *C, int32_t conserve, void *ws,
                              size_t ws_bytes, void *stream);

/* The collocated form of the same DG collision term (nodal basis on the K
 * quadrature points of the element, Section 3.3.1 with the K-point rule): T is
 * the identity and W = diag(w), so
 *   C[e][m] = w_m Q(F[e][m]),   m < K,
 * e.g. w_m = J times the Gauss weight of node m.  No contraction runs: F is
 * evaluated as a batch of n_elem*K items and each item's weight is applied
 * in the store of the last pass (after the projection when conserve != 0;
 * the projection is linear).  host_w: HOST [K] finite weights; F, C device
 * FP64 [n_elem][K][N^3], C must not overlap F.  Workspace from
 * qcoll_dg_collocated_workspace_bytes. */
size_t qcoll_dg_collocated_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K);
qcoll_status qcoll_dg_collide_collocated(qcoll_plan plan, int64_t n_elem, int32_t K, const double *host_w,
                                         const double *F, double *C, int32_t conserve, void *ws, size_t ws_bytes,
                                         void *stream);

/* Items per chunk of the eval pipeline (0 = default 64); workspace sizes
 * depend on it.  Results do not. */
qcoll_status qcoll_plan_set_chunk(qcoll_plan plan, int32_t items);

/* Autotuner: times the candidate schedules of this plan (fused / two-pass hot
 * loop x 32, 64, 96, 128, 192, 256 items per chunk, each balanced over the
 * batch as ceil(batch / ceil(batch / c)); best of two timed runs each) with qcoll_eval on the caller's f and Q (Q is overwritten), keeps the
 * fastest in the plan and returns it in
 * *host_schedule, *host_chunk (either may be NULL).  Synchronous.  If the
 * environment variable QCOLL_AUTOTUNE_CACHE names a file, choices are read
 * from and appended to it, keyed by (arch, the library's schedule set, N,
 * N_rho, M, precision, rank, batch rounded up to a power of two); entries of
 * an older schedule set are timed again. */
size_t qcoll_autotune_workspace_bytes(qcoll_plan plan, int64_t batch);
qcoll_status qcoll_autotune(qcoll_plan plan, int64_t batch, const double *f, double *Q, void *ws,
                            size_t ws_bytes, void *stream, int32_t *host_schedule, int32_t *host_chunk);

/* Groups of plans (several velocity grids / kernels / ranks) with their item
 * counts, evaluated as one launch: each plan's pipeline runs on its own
 * stream between a fork and a join on the caller's stream, ordered by model
 * cost (largest first).  With use_graph != 0 the fork/join is captured into
 * a hipGraph the first time a given set of pointers is used (stream must not
 * be the legacy default stream) and replayed with one hipGraphLaunch after
 * that; the graph holds kernel nodes only.
 *   plans, counts: HOST arrays of nplans entries (plans outlive the group).
 *   f, Q, g, df, domega: HOST arrays of nplans DEVICE pointers, entry i laid
 *   out as for the single-plan calls with counts[i] items (domega may be NULL,
 *   or have NULL entries).
 * Workspace from qcoll_group_workspace_bytes(group, op) (op 0 eval, 1 vjp).
 * Calls on one group must not overlap (they share its streams and graphs). */
qcoll_status qcoll_group_create(const qcoll_plan *plans, const int64_t *counts, int32_t nplans,
                                qcoll_group *out);
qcoll_status qcoll_group_destroy(qcoll_group group);
size_t qcoll_group_workspace_bytes(qcoll_group group, int32_t op);
qcoll_status qcoll_group_eval(qcoll_group group, const double *const *f, double *const *Q,
                              int32_t conserve, void *ws, size_t ws_bytes, void *stream,
                              int32_t use_graph);
qcoll_status qcoll_group_vjp(qcoll_group group, const double *const *f, const double *const *g,
                             double *const *df, double *const *domega, int32_t through_conserve,
                             void *ws, size_t ws_bytes, void *stream, int32_t use_graph);
/* Autotune every member plan on its own inputs (qcoll_autotune with the
 * plan's item count; Q entries are overwritten), so that a later captured
 * graph records the tuned schedules.  Synchronous.  Workspace from
 * qcoll_group_autotune_workspace_bytes (the largest member's need). */
size_t qcoll_group_autotune_workspace_bytes(qcoll_group group);
qcoll_status qcoll_group_autotune(qcoll_group group, const double *const *f, double *const *Q, void *ws,
                                  size_t ws_bytes, void *stream);

/* The paper's SVD variant of the DG collision term with general factors:
 *   C[e][m] = sum_r W[m][r] Q( sum_l T1[r][l] F[e][l], sum_l T2[r][l] F[e][l] )
 * with the bilinear Q (f_r = U^m F, g_r = V^m F of the SVD H_m = U V).
 * T1, T2: [R][K], W: [K][R] device FP64.  Workspace from
 * qcoll_dg_svd_workspace_bytes. */
size_t qcoll_dg_svd_workspace_bytes(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R);
qcoll_status qcoll_dg_collide_svd(qcoll_plan plan, int64_t n_elem, int32_t K, int32_t R,
                                  const double *T1, const double *T2, const double *W, const double *F,
                                  double *C, int32_t conserve, void *ws, size_t ws_bytes, void *stream);

/* 1-D RKDG driver (Section 3): DG in x on the K = P+1 Gauss-Legendre nodes of
 * every element (diagonal mass matrix), the upwind flux of Section 3.2, the
 * collision term of the weak form through the plan, SSP-RK2/RK3 of Section
 * 3.4 and the boundary conditions of Section 3.5.  The walls are normal to x.
 *   F, R: device FP64 [n_elem][K][N^3] nodal values (item order of qcoll_eval);
 *   dF_m/dt = (c_x (S F)_m - face terms) / (J w_m) + inv_kn * C_m / (J w_m),
 *   C_m = sum_{l1,l2} H_{m l1 l2} Q(F_l1, F_l2) with H exact (eigen form of the
 *   triple tensor, coll_form 1) or from the K-point rule (C_m = J w_m Q(F_m),
 *   coll_form 0).  The plan's precision applies to Q; the transport is FP64. */
typedef struct qcoll_dg1d_s *qcoll_dg1d;

typedef enum { QCOLL_BC_PERIODIC = 0, QCOLL_BC_WALL = 1, QCOLL_BC_INFLOW = 2 } qcoll_bc_kind;

/* One end of the interval.  PERIODIC: both ends or neither.  WALL: fully
 * diffuse at velocity u and temperature T; incoming velocities ((c - u).n < 0)
 * see n_w exp(-|c - u|^2 / T) with n_w from zero net mass flux (discrete sums
 * over the velocity grid).  INFLOW: incoming velocities (c.n < 0) see the
 * Maxwellian n (pi T)^{-3/2} exp(-|c - u|^2 / T). */
typedef struct {
  int32_t kind;
  double n;
  double u[3];
  double T;
} qcoll_bc;

typedef struct {
  int32_t n_elem;        /* >= 1 */
  const double *faces;   /* HOST [n_elem + 1], strictly increasing */
  int32_t order;         /* P, 0..7 */
  double inv_kn;         /* >= 0; 0 = free streaming (no collision term) */
  int32_t coll_form;     /* 0 collocated, 1 exact triple tensor */
  int32_t conserve;      /* project every Q evaluation (qcoll_conserve) */
  qcoll_bc left, right;
} qcoll_dg1d_params;

/* The driver keeps the plan pointer (not owned: destroy the driver first) and
 * small device tables.  EINVAL for bad parameters. */
qcoll_status qcoll_dg1d_create(qcoll_plan plan, const qcoll_dg1d_params *p, qcoll_dg1d *out);
qcoll_status qcoll_dg1d_destroy(qcoll_dg1d d);
/* Node positions, HOST [n_elem][K]. */
qcoll_status qcoll_dg1d_nodes(qcoll_dg1d d, double *host_x);
/* Workspace for qcoll_dg1d_rhs (rk = 0) or qcoll_dg1d_step (rk = 1, 2, 3). */
size_t qcoll_dg1d_workspace_bytes(qcoll_dg1d d, int32_t rk);
/* R = L(F), the right-hand side of the semi-discrete system.  R must not
 * overlap F. */
qcoll_status qcoll_dg1d_rhs(qcoll_dg1d d, const double *F, double *R, void *ws, size_t ws_bytes, void *stream);
/* One time step in place: rk = 1 forward Euler, 2 SSP-RK2, 3 SSP-RK3. */
qcoll_status qcoll_dg1d_step(qcoll_dg1d d, double *F, double dt, int32_t rk, void *ws, size_t ws_bytes,
                             void *stream);

/* Synchronise the device, then report and clear the non-finite flag. */
qcoll_status qcoll_poll(qcoll_plan plan);

const char *qcoll_status_str(qcoll_status s);
const char *qcoll_last_error(void);
int32_t qcoll_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QCOLL_H */
