// Shared building blocks of the batched transforms: the slab pass (two inner
// axes in LDS), the pencil pass (outer axis in registers), common prologue and
// epilogue functors, and launch helpers.
//
// Every 3-D transform is split in two passes over HBM:
//   slab pass   : one workgroup holds SPB slabs (fixed first index) in LDS and
//                 transforms the two inner axes (rows in registers, then
//                 columns), with coalesced loads/stores of whole slabs;
//   pencil pass : one lane holds one pencil along the outer axis (stride N^2,
//                 coalesced across lanes) and transforms it in registers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "qcoll_fft.hpp"
#include "qcoll_internal.h"

namespace qcoll {

template <typename T>
using C = cplx<T>;

// slabs per workgroup: keep the LDS tile (re + im, padded rows) within 64 KiB
template <typename T, int N>
constexpr int spb() {
  constexpr int by_lds = 65536 / (2 * N * (N + 1) * int(sizeof(T)));
  constexpr int by_threads = 256 / N;
  constexpr int s = by_lds < by_threads ? by_lds : by_threads;
  return s < 1 ? 1 : s;
}

// 2-D transform of the SPB slabs held in LDS: rows (last axis), then columns.
template <typename T, int N, int SPB, int SIGN>
__device__ __forceinline__ void lds_slab_fft(T (*sre)[N][N + 1], T (*sim)[N][N + 1]) {
  const int tid = threadIdx.x;
  const int s = tid / N, r = tid % N;
  T xr[N], xi[N];
  static_for<0, N>([&](auto c) {
    xr[decltype(c)::value] = sre[s][r][decltype(c)::value];
    xi[decltype(c)::value] = sim[s][r][decltype(c)::value];
  });
  fft_reg<N, SIGN, T>(xr, xi);
  static_for<0, N>([&](auto c) {
    sre[s][r][decltype(c)::value] = xr[decltype(c)::value];
    sim[s][r][decltype(c)::value] = xi[decltype(c)::value];
  });
  __syncthreads();
  static_for<0, N>([&](auto rr) {
    xr[decltype(rr)::value] = sre[s][decltype(rr)::value][r];
    xi[decltype(rr)::value] = sim[s][decltype(rr)::value][r];
  });
  fft_reg<N, SIGN, T>(xr, xi);
  static_for<0, N>([&](auto rr) {
    sre[s][decltype(rr)::value][r] = xr[decltype(rr)::value];
    sim[s][decltype(rr)::value][r] = xi[decltype(rr)::value];
  });
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Generic slab kernel: Src(g, r, c) -> C<T> loads element (r, c) of slab g with
// any prologue; Dst(g, r, c, v) stores.  Slabs g >= nslab are skipped.
template <typename T, int N, int SIGN, class Src, class Dst>
__global__ __launch_bounds__(256) void k_slab(Src src, Dst dst, long nslab) {
  constexpr int SPB = spb<T, N>();
  __shared__ T sre[SPB][N][N + 1];
  __shared__ T sim[SPB][N][N + 1];
  const long g0 = long(blockIdx.x) * SPB;
  for (int e = threadIdx.x; e < SPB * N * N; e += SPB * N) {
    const int s = e / (N * N), rc = e % (N * N), r = rc / N, c = rc % N;
    const long g = g0 + s;
    C<T> v{T(0), T(0)};
    if (g < nslab) v = src(g, r, c);
    sre[s][r][c] = v.re;
    sim[s][r][c] = v.im;
  }
  __syncthreads();
  lds_slab_fft<T, N, SPB, SIGN>(sre, sim);
  for (int e = threadIdx.x; e < SPB * N * N; e += SPB * N) {
    const int s = e / (N * N), rc = e % (N * N), r = rc / N, c = rc % N;
    const long g = g0 + s;
    if (g < nslab) dst(g, r, c, C<T>{sre[s][r][c], sim[s][r][c]});
  }
}

// generic pencil kernel: Op(pencil_group, r) with r = j2*N + j3
template <int N, class Op>
__global__ __launch_bounds__(256) void k_pencil(Op op, long npencil) {
  const long pid = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (pid >= npencil) return;
  op(pid / (N * N), int(pid % (N * N)));
}

// ----------------------------------------------------------------------------
// functors

// real FP64 input -> complex T, slab g = item*N + j1
template <typename T, int N>
struct SrcReal {
  const double *f;
  __device__ C<T> operator()(long g, int r, int c) const {
    return C<T>{T(f[(g * N + r) * N + c]), T(0)};
  }
};

template <typename T, int N>
struct DstCplx {
  C<T> *out;
  __device__ void operator()(long g, int r, int c, C<T> v) const { out[(g * N + r) * N + c] = v; }
};

template <typename T, int N>
struct SrcCplx {
  const C<T> *in;
  __device__ C<T> operator()(long g, int r, int c) const { return in[(g * N + r) * N + c]; }
};

// hot loop, slab pass: task t = (bp_local, q) with bp = bp0 + bp_local,
// b = bp / N_rho, p = bp % N_rho; slab g = t*N + k1.  Loads H[b] times the
// real multiplier c_s = Re beta_s + Im beta_s, beta_s = b1(k1) b2(k2) b3(k3),
// scaled by 1/N^3 (normalised inverse).
template <typename T, int N>
struct SrcShift {
  const C<T> *H;
  const C<T> *phase;
  long bp0;
  int M, Nr;
  T scale;
  __device__ C<T> operator()(long g, int r, int c) const {
    const long t = g / N;
    const int k1 = int(g % N);
    const long bp = bp0 + t / M;
    const int q = int(t % M);
    const long b = bp / Nr;
    const int p = int(bp % Nr);
    const C<T> *ph = phase + size_t(p * M + q) * 3 * N;
    const C<T> b1 = ph[k1], b2 = ph[N + r], b3 = ph[2 * N + c];
    const T x12 = b1.re * b2.re - b1.im * b2.im, y12 = b1.re * b2.im + b1.im * b2.re;
    const T x = x12 * b3.re - y12 * b3.im, y = x12 * b3.im + y12 * b3.re;
    const T m = (x + y) * scale;
    const C<T> h = H[((b * N + k1) * N + r) * N + c];
    return C<T>{h.re * m, h.im * m};
  }
};

// forward pencil pass in place (first axis)
template <typename T, int N, int SIGN>
struct OpPencilInPlace {
  C<T> *X;
  __device__ void operator()(long v, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    C<T> *x = X + v * n3 + r;
    T xr[N], xi[N];
    static_for<0, N>([&](auto k) {
      const C<T> e = x[decltype(k)::value * n2];
      xr[decltype(k)::value] = e.re;
      xi[decltype(k)::value] = e.im;
    });
    fft_reg<N, SIGN, T>(xr, xi);
    static_for<0, N>([&](auto k) { x[decltype(k)::value * n2] = C<T>{xr[decltype(k)::value], xi[decltype(k)::value]}; });
  }
};

// FP64 spectrum -> working precision
template <typename T>
__global__ void k_cast(const C<double> *in, C<T> *out, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = C<T>{T(in[i].re), T(in[i].im)};
}

inline unsigned nblk(long n, int b) { return unsigned((n + b - 1) / b); }

#define QC_LAUNCH_CHECK(what)                                           \
  do {                                                                  \
    hipError_t e_ = hipGetLastError();                                  \
    if (e_ != hipSuccess) {                                             \
      set_error(std::string(what) + ": " + hipGetErrorString(e_));      \
      return QCOLL_EDEVICE;                                             \
    }                                                                   \
  } while (0)

template <typename T, int N>
struct Passes {
  static constexpr int SPB = spb<T, N>();
  static constexpr long n3 = long(N) * N * N;

  template <class Src, class Dst, int SIGN>
  static qcoll_status slab(Src s, Dst d, long nslab, hipStream_t st, const char *what) {
    if (nslab <= 0) return QCOLL_OK;
    TimedLaunch tl(what, st);
    hipLaunchKernelGGL((k_slab<T, N, SIGN, Src, Dst>), dim3(nblk(nslab, SPB)), dim3(SPB * N), 0, st, s, d, nslab);
    QC_LAUNCH_CHECK(what);
    return QCOLL_OK;
  }
  template <class Op>
  static qcoll_status pencil(Op op, long npencil, hipStream_t st, const char *what) {
    if (npencil <= 0) return QCOLL_OK;
    TimedLaunch tl(what, st);
    hipLaunchKernelGGL((k_pencil<N, Op>), dim3(nblk(npencil, 256)), dim3(256), 0, st, op, npencil);
    QC_LAUNCH_CHECK(what);
    return QCOLL_OK;
  }

  // forward transform of nb real items into H (complex)
  static qcoll_status forward(const double *f, C<T> *H, long nb, hipStream_t st) {
    qcoll_status s;
    if ((s = slab<SrcReal<T, N>, DstCplx<T, N>, -1>(SrcReal<T, N>{f}, DstCplx<T, N>{H}, nb * N, st, "forward slab")))
      return s;
    return pencil(OpPencilInPlace<T, N, -1>{H}, nb * N * N, st, "forward pencil");
  }

};

}  // namespace qcoll
