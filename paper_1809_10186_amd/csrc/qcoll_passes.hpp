// Shared building blocks of the batched transforms: the slab pass (two inner
// axes in LDS), the pencil pass (outer axis in registers), common prologue and
// epilogue functors, and launch helpers.
//
// Every 3-D transform is split in two passes over HBM:
//   slab pass   : one workgroup holds SPB slabs (fixed first index) and
//                 transforms the two inner axes (columns in registers from
//                 the loads, rows through LDS), with coalesced loads/stores;
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

// Slabs per block of the slab kernels, for bytes_per_slab of LDS: the first
// count whose lanes fill whole waves, else the one that leaves the fewest lanes
// idle, with the LDS tile within 64 KiB and at most 256 lanes.
constexpr int spb_for(int N, int bytes_per_slab) {
  int best = 1, best_num = 0, best_den = 1;
  for (int s = 1; s * N <= 256 && s * bytes_per_slab <= 65536; ++s) {
    const int lanes = s * N, waves = (lanes + 63) / 64;
    if (lanes % 64 == 0) return s;
    if (lanes * best_den > best_num * (64 * waves)) {
      best = s;
      best_num = lanes;
      best_den = 64 * waves;
    }
  }
  return best;
}

constexpr int lane_use_pct(int N, int spb) { return 100 * spb * N / (64 * ((spb * N + 63) / 64)); }

// both components of the slab in LDS at once
template <typename T, int N>
constexpr int slab_spb2() {
  return spb_for(N, 2 * N * (N + 1) * int(sizeof(T)));
}

// resident waves per CU that the LDS tile of a slab block allows (160 KiB per CU)
constexpr int slab_lds_waves(int N, int spb, int bytes_per_slab) {
  return (163840 / (spb * bytes_per_slab)) * ((spb * N + 63) / 64);
}

// k_slab moves one component at a time through LDS (more barriers, half the
// tile) where that turns blocks with idle lanes into whole waves (N = 48 in
// FP32), where both components of one slab exceed 64 KiB (N = 64 in FP64), or
// where blocks with idle lanes leave fewer than two waves per SIMD resident and
// the split tile more (FP64 at N = 24 and 48).  Whole-wave FP64 blocks at
// N = 32 keep both components: split, their shifted-spectrum slab pass ran
// slower despite twice the resident waves.
template <typename T, int N>
constexpr bool slab_split() {
  constexpr int b2 = 2 * N * (N + 1) * int(sizeof(T)), b1 = N * (N + 1) * int(sizeof(T));
  constexpr int s2 = slab_spb2<T, N>(), s1 = spb_for(N, b1);
  return b2 > 65536 || (lane_use_pct(N, s2) < 80 && lane_use_pct(N, s1) == 100) ||
         (lane_use_pct(N, s2) < 100 && slab_lds_waves(N, s2, b2) < 8 &&
          slab_lds_waves(N, s1, b1) > slab_lds_waves(N, s2, b2));
}

template <typename T, int N>
constexpr int slab_spb() {
  return slab_split<T, N>() ? spb_for(N, N * (N + 1) * int(sizeof(T))) : slab_spb2<T, N>();
}

// Sources that declare kGroupedLoads provide raw(g, r, c), the element in its
// stored precision; k_slab then issues the loads of a group of rows together
// and widens them afterwards (left to itself, the compiler reuses a few
// registers for the raw values and waits for every load on its own).
template <class S, class = void>
struct grouped_loads : std::false_type {};
template <class S>
struct grouped_loads<S, std::void_t<decltype(S::kGroupedLoads)>> : std::bool_constant<S::kGroupedLoads> {};

// Generic slab kernel: Src(g, r, c) -> C<T> loads element (r, c) of slab g with
// any prologue; Dst(g, r, c, v) stores.  Slabs g >= nslab are skipped.
//
// Lane (s, c) owns column c of local slab s: it loads the column (consecutive
// lanes read consecutive c, so every load is coalesced), transforms it along
// r in registers, and passes it through LDS once for the row transforms; the
// result goes back through LDS so that the stores are column-wise again.  The
// slab index is fixed per lane, so whatever Src and Dst derive from it is
// computed once.  Lanes of a slab past the end read slab nslab - 1 (always
// valid) and store nothing.  With SPLIT the real and imaginary parts take
// turns in one tile.
template <typename T, int N, int SIGN, class Src, class Dst, int SPB = slab_spb<T, N>(),
          bool SPLIT = slab_split<T, N>()>
__global__ __launch_bounds__(256) void k_slab(Src src, Dst dst, long nslab) {
  const int s = int(threadIdx.x) / N, c = int(threadIdx.x) % N;
  const long g = long(blockIdx.x) * SPB + s;
  const long gl = g < nslab ? g : nslab - 1;
  T xr[N], xi[N];
  if constexpr (grouped_loads<Src>::value) {
    constexpr int LG = (N % 16 == 0) ? 16 : ((N % 8 == 0) ? 8 : 4);
    static_for<0, N / LG>([&](auto gg) {
      constexpr int r0 = decltype(gg)::value * LG;
      decltype(src.raw(gl, 0, c)) v[LG];
      static_for<0, LG>([&](auto ii) { v[decltype(ii)::value] = src.raw(gl, r0 + decltype(ii)::value, c); });
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, LG>([&](auto ii) {
        xr[r0 + decltype(ii)::value] = T(v[decltype(ii)::value].re);
        xi[r0 + decltype(ii)::value] = T(v[decltype(ii)::value].im);
      });
    });
  } else {
    static_for<0, N>([&](auto r) {
      const C<T> v = src(gl, decltype(r)::value, c);
      xr[decltype(r)::value] = v.re;
      xi[decltype(r)::value] = v.im;
    });
  }
  fft_reg<N, SIGN, T>(xr, xi);
  if constexpr (SPLIT) {
    // one tile, one component at a time: column -> row, row FFT, row -> column
    __shared__ T sb[SPB][N][N + 1];
    const int row = c;
    auto to_rows = [&](T *x) {
      static_for<0, N>([&](auto r) { sb[s][decltype(r)::value][c] = x[decltype(r)::value]; });
      __syncthreads();
      static_for<0, N>([&](auto k) { x[decltype(k)::value] = sb[s][row][decltype(k)::value]; });
      __syncthreads();
    };
    auto to_cols = [&](T *x) {
      static_for<0, N>([&](auto k) { sb[s][row][decltype(k)::value] = x[decltype(k)::value]; });
      __syncthreads();
      static_for<0, N>([&](auto r) { x[decltype(r)::value] = sb[s][decltype(r)::value][c]; });
      __syncthreads();
    };
    to_rows(xr);
    to_rows(xi);
    fft_reg<N, SIGN, T>(xr, xi);
    to_cols(xr);
    to_cols(xi);
    if (g < nslab) {
      static_for<0, N>([&](auto r) {
        dst(g, decltype(r)::value, c, C<T>{xr[decltype(r)::value], xi[decltype(r)::value]});
      });
    }
    return;
  } else {
    __shared__ T sre[SPB][N][N + 1];
    __shared__ T sim[SPB][N][N + 1];
    static_for<0, N>([&](auto r) {
      sre[s][decltype(r)::value][c] = xr[decltype(r)::value];
      sim[s][decltype(r)::value][c] = xi[decltype(r)::value];
    });
    __syncthreads();
    const int row = c;
    static_for<0, N>([&](auto k) {
      xr[decltype(k)::value] = sre[s][row][decltype(k)::value];
      xi[decltype(k)::value] = sim[s][row][decltype(k)::value];
    });
    fft_reg<N, SIGN, T>(xr, xi);
    static_for<0, N>([&](auto k) {
      sre[s][row][decltype(k)::value] = xr[decltype(k)::value];
      sim[s][row][decltype(k)::value] = xi[decltype(k)::value];
    });
    __syncthreads();
    if (g < nslab) {
      static_for<0, N>([&](auto r) {
        dst(g, decltype(r)::value, c, C<T>{sre[s][decltype(r)::value][c], sim[s][decltype(r)::value][c]});
      });
    }
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
    // a slab block never straddles two terms when its slab count divides N
    // (the N slabs of a term are consecutive and every launch holds whole
    // terms): the term is then uniform over the wave, and its phase rows are
    // read with scalar loads instead of one vector load per element
    constexpr bool UNIFORM = (N % slab_spb<T, N>()) == 0;
    long t = g / N;
    if constexpr (UNIFORM) t = __builtin_amdgcn_readfirstlane(int(t));
    const int k1 = int(g % N);
    const long bp = bp0 + t / M;
    const int q = int(t % M);
    const long b = bp / Nr;
    const int p = int(bp % Nr);
    const C<T> *ph = phase + size_t(p * M + q) * 3 * N;
    // m = Re(b1 b2 b3) + Im(b1 b2 b3) = b2.re P + b2.im Q with P, Q from b1 b3,
    // which do not depend on the row r (computed once per lane and column)
    const C<T> b1 = ph[k1], b2 = ph[N + r], b3 = ph[2 * N + c];
    const T x13 = b1.re * b3.re - b1.im * b3.im, y13 = b1.re * b3.im + b1.im * b3.re;
    const T P = (x13 + y13) * scale, Q = (x13 - y13) * scale;
    const T m = b2.re * P + b2.im * Q;
    const C<T> h = H[((b * N + k1) * N + r) * N + c];
    return C<T>{h.re * m, h.im * m};
  }
};

// forward pencil pass in place (first axis), plus a copy rounded to U
template <typename T, typename U, int N>
struct OpPencilForwardTo {
  C<T> *X;
  C<U> *XU;
  __device__ void operator()(long v, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    C<T> *x = X + v * n3 + r;
    C<U> *xu = XU + v * n3 + r;
    T xr[N], xi[N];
    static_for<0, N>([&](auto k) {
      const C<T> e = x[decltype(k)::value * n2];
      xr[decltype(k)::value] = e.re;
      xi[decltype(k)::value] = e.im;
    });
    fft_reg<N, -1, T>(xr, xi);
    static_for<0, N>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      x[kk * n2] = C<T>{xr[kk], xi[kk]};
      xu[kk * n2] = C<U>{U(xr[kk]), U(xi[kk])};
    });
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

inline unsigned nblk(long n, int b) { return unsigned((n + b - 1) / b); }

// register width of the low-rank mixing kernels for n (<= 64) radial nodes:
// the next of 8, 16, 24, 32, 48, 64
inline int mix_width(int n) { return n <= 32 ? ((n + 7) / 8) * 8 : (n <= 48 ? 48 : 64); }

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
  static constexpr long n3 = long(N) * N * N;

  template <class Src, class Dst, int SIGN>
  static qcoll_status slab(Src s, Dst d, long nslab, hipStream_t st, const char *what) {
    if (nslab <= 0) return QCOLL_OK;
    TimedLaunch tl(what, st);
    constexpr int SPB = slab_spb<T, N>();
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

  // the same, also storing a copy of the spectrum rounded to U (the pencil
  // pass writes both, so the copy costs no extra read)
  template <typename U>
  static qcoll_status forward_to(const double *f, C<T> *H, C<U> *HU, long nb, hipStream_t st) {
    qcoll_status s;
    if ((s = slab<SrcReal<T, N>, DstCplx<T, N>, -1>(SrcReal<T, N>{f}, DstCplx<T, N>{H}, nb * N, st, "forward slab")))
      return s;
    return pencil(OpPencilForwardTo<T, U, N>{H, HU}, nb * N * N, st, "forward pencil");
  }

};

// Half spectra: slab g of a pass over the planes k1 <= N/2 of every item is
// plane g % (N/2 + 1) of item g / (N/2 + 1), kept in the full [item][k1][k2][k3]
// layout (the planes k1 > N/2 follow by Hermitian symmetry).
template <int N>
__device__ __forceinline__ long half_slab(long g) {
  constexpr int H1 = N / 2 + 1;
  return (g / H1) * N + g % H1;
}

template <typename T, int N>
struct SrcCplxHalf {
  const C<T> *in;
  __device__ C<T> operator()(long g, int r, int c) const { return in[(half_slab<N>(g) * N + r) * N + c]; }
};

template <typename T, int N>
struct DstCplxHalf {
  C<T> *out;
  __device__ void operator()(long g, int r, int c, C<T> v) const { out[(half_slab<N>(g) * N + r) * N + c] = v; }
};

}  // namespace qcoll
