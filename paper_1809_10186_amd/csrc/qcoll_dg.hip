// DG collision term of the weak form (Section 3.3.1):
//   C[e][m] = sum_r W[m][r] Q( sum_l T[r][l] F[e][l] ),
// which covers the paper's SVD (eigen) variant (T = stacked eigenvectors of the
// triple tensor H_m, W = their eigenvalues) and the quadrature form (T = basis
// values at quadrature points, W = weighted basis values).  The two small
// contractions run on MFMA: v_mfma_f64_16x16x4f64 tiles of 16 output rows x 16
// velocity points, the inner (basis) dimension in steps of 4.
#include <hip/hip_runtime.h>

#include "qcoll_internal.h"

namespace qcoll {

typedef double d4 __attribute__((ext_vector_type(4)));

// Y[e][i][j] = sum_k A[i][k] X[e][k][j]; A is [rows][cols] row-major (device),
// X is [E][cols][n3], Y is [E][rows][n3].  One wave per (e, 16-row tile,
// 16-point tile).  Operand layout of the 16x16x4 FP64 MFMA (lane l):
//   A: row l % 16, k = l / 16;  B: column l % 16, k = l / 16;
//   D: 4 values v, row (l / 16) + 4 v, column l % 16 (rows interleaved across
//   the four 16-lane groups; checked by the DG parity tests).
__global__ __launch_bounds__(256) void k_dg_contract(const double *__restrict__ A, const double *__restrict__ X,
                                                     double *__restrict__ Y, long E, int rows, int cols, long n3) {
  const long wave = (long(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  const long ptiles = n3 / 16;
  const int rtiles = (rows + 15) / 16;
  const long total = E * rtiles * ptiles;
  if (wave >= total) return;  // uniform per wave
  const long e = wave / (rtiles * ptiles);
  const long rest = wave % (rtiles * ptiles);
  const int rt = int(rest / ptiles);
  const long j0 = (rest % ptiles) * 16;
  const int li = lane % 16, lk = lane / 16;
  const int i = rt * 16 + li;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < cols; k0 += 4) {
    const int k = k0 + lk;
    const double a = (i < rows && k < cols) ? A[long(i) * cols + k] : 0.0;
    const double b = (k < cols) ? X[(e * cols + k) * n3 + j0 + li] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  for (int v = 0; v < 4; ++v) {
    const int io = rt * 16 + lk + 4 * v;
    if (io < rows) Y[(e * rows + io) * n3 + j0 + li] = acc[v];
  }
}

qcoll_status launch_dg_contract(const double *A, const double *X, double *Y, long E, int rows, int cols, long n3,
                                hipStream_t st) {
  const long waves = E * ((rows + 15) / 16) * (n3 / 16);
  const long threads = waves * 64;
  TimedLaunch tl("dg contract", st);
  hipLaunchKernelGGL(k_dg_contract, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, st, A, X, Y, E, rows, cols,
                     n3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("dg contract: ") + hipGetErrorString(e));
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

}  // namespace qcoll
