// Batched evaluation of the fast spectral collision operator (gfx950), built
// on the slab and pencil passes of qcoll_passes.hpp.
// The pointwise work of the method is fused into these passes:
//   - the shift multiplier of each (rho_p, sigma_q) term into the slab load,
//   - the product t1 t2 and the sphere sum into the pencil pass,
//   - the low-rank weights, the loss multiplier and the final assembly into
//     the last passes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <type_traits>

#include "qcoll_passes.hpp"

namespace qcoll {

// complex input in T widened to U (the literal convention's low-rank stage)
template <typename T, int N, typename U>
struct SrcCplxWide {
  const C<T> *in;
  __device__ C<U> operator()(long g, int r, int c) const {
    const C<T> v = in[(g * N + r) * N + c];
    return C<U>{U(v.re), U(v.im)};
  }
};

// hot loop, pencil pass: for each (b, p) and pencil (j2, j3), inverse
// transform along the first axis for every q and accumulate
// A_p += w_q (u_re^2 - u_im^2)  (= w_q t1 t2 with t1 = re - im, t2 = re + im).
template <typename T, int N>
struct OpGainAcc {
  const C<T> *Y;
  const T *wq;
  T *A;
  long bp0;
  int M;
  __device__ void operator()(long bpl, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    T acc[N];
    static_for<0, N>([&](auto j) { acc[decltype(j)::value] = T(0); });
    for (int q = 0; q < M; ++q) {
      const C<T> *y = Y + (bpl * M + q) * n3 + r;
      T xr[N], xi[N];
      static_for<0, N>([&](auto k) {
        const C<T> v = y[decltype(k)::value * n2];
        xr[decltype(k)::value] = v.re;
        xi[decltype(k)::value] = v.im;
      });
      fft_reg<N, +1, T>(xr, xi);
      const T w = wq[q];
      static_for<0, N>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        acc[jj] += w * (xr[jj] * xr[jj] - xi[jj] * xi[jj]);
      });
    }
    T *a = A + (bp0 + bpl) * n3 + r;
    static_for<0, N>([&](auto j) { a[decltype(j)::value * n2] = acc[decltype(j)::value]; });
  }
};

// The same pencil pass with the M terms of each pencil split in kGainParts
// fixed parts, one wave per part: a workgroup owns 64 consecutive pencils (so
// every wave's loads stay one coalesced run), waves 1.. leave their sums in
// LDS and wave 0 adds them in order, ((part 0 + part 1) + ...), and stores.
// A launch of 32 pairs at 32^3 (or 18 at 48^3) otherwise runs about two waves
// per CU.  The split is fixed by M, so a pair's result does not depend on the
// launch sizes.  Needs N^2 to be a multiple of 64 and the parts' sums to fit
// 48 KiB of LDS (not FP64 at 48^3).
constexpr int kGainParts = 4;

template <typename T, int N>
__global__ __launch_bounds__(64 * kGainParts) void k_gain_pencil_parts(const C<T> *Y, const T *wq, T *A, long bp0,
                                                                       int M) {
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  __shared__ T part_acc[kGainParts - 1][N][64];
  const int lane = int(threadIdx.x) % 64, part = int(threadIdx.x) / 64;
  const long pen = long(blockIdx.x) * 64 + lane;   // the grid covers whole groups of 64 pencils
  const long bpl = pen / n2;
  const int r = int(pen % n2);
  T acc[N];
  static_for<0, N>([&](auto j) { acc[decltype(j)::value] = T(0); });
  const int q0 = (part * M) / kGainParts, q1 = ((part + 1) * M) / kGainParts;
  for (int q = q0; q < q1; ++q) {
    const C<T> *y = Y + (bpl * M + q) * n3 + r;
    T xr[N], xi[N];
    static_for<0, N>([&](auto k) {
      const C<T> v = y[decltype(k)::value * n2];
      xr[decltype(k)::value] = v.re;
      xi[decltype(k)::value] = v.im;
    });
    fft_reg<N, +1, T>(xr, xi);
    const T w = wq[q];
    static_for<0, N>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      acc[jj] += w * (xr[jj] * xr[jj] - xi[jj] * xi[jj]);
    });
  }
  if (part > 0) static_for<0, N>([&](auto j) { part_acc[part - 1][decltype(j)::value][lane] = acc[decltype(j)::value]; });
  __syncthreads();
  if (part == 0) {
#pragma unroll
    for (int k = 0; k < kGainParts - 1; ++k)
      static_for<0, N>([&](auto j) { acc[decltype(j)::value] += part_acc[k][decltype(j)::value][lane]; });
    T *a = A + (bp0 + bpl) * n3 + r;
    static_for<0, N>([&](auto j) { a[decltype(j)::value * n2] = acc[decltype(j)::value]; });
  }
}

template <typename T, int N>
constexpr bool gain_pencil_parts() {
  return (long(N) * N) % 64 == 0 && size_t(kGainParts - 1) * N * 64 * sizeof(T) <= 48 * 1024;
}

// bilinear hot loop, pencil pass: u_f and u_g inverse along axis 1 for every
// q; A_p += w_q Re(u_f u_g)  (= w_q (t1_f t2_g + t2_f t1_g) / 2)
template <typename T, int N>
struct OpGainAcc2 {
  const C<T> *Yf, *Yg;
  const T *wq;
  T *A;
  long bp0;
  int M;
  __device__ void operator()(long bpl, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    T acc[N];
    static_for<0, N>([&](auto j) { acc[decltype(j)::value] = T(0); });
    for (int q = 0; q < M; ++q) {
      const C<T> *yf = Yf + (bpl * M + q) * n3 + r;
      const C<T> *yg = Yg + (bpl * M + q) * n3 + r;
      T fr[N], fi[N], gr[N], gi[N];
      static_for<0, N>([&](auto k) {
        const C<T> a = yf[decltype(k)::value * n2], c = yg[decltype(k)::value * n2];
        fr[decltype(k)::value] = a.re;
        fi[decltype(k)::value] = a.im;
        gr[decltype(k)::value] = c.re;
        gi[decltype(k)::value] = c.im;
      });
      fft_reg<N, +1, T>(fr, fi);
      fft_reg<N, +1, T>(gr, gi);
      const T w = wq[q];
      static_for<0, N>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        acc[jj] += w * (fr[jj] * gr[jj] - fi[jj] * gi[jj]);
      });
    }
    T *a = A + (bp0 + bpl) * n3 + r;
    static_for<0, N>([&](auto j) { a[decltype(j)::value * n2] = acc[decltype(j)::value]; });
  }
};

// low-rank mixing: B[b][s] = sum_p U[s][p] A[b][p]
template <typename T, int NRM>
__global__ __launch_bounds__(256) void k_mix(const T *A, const T *U, T *B, long nitems, int S, int Nr, long n3) {
  // one point per lane: its Nr (<= NRM) node values are loaded once into
  // registers; U (S x Nr, S <= Nr) is staged per block in LDS, zero-padded to
  // NRM columns, and read at one address per wave (broadcast)
  __shared__ T us[NRM * NRM];
  for (int t = threadIdx.x; t < S * NRM; t += blockDim.x) {
    const int s = t / NRM, q = t % NRM;
    us[t] = (q < Nr) ? U[s * Nr + q] : T(0);
  }
  __syncthreads();
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nitems * n3) return;
  const long b = i / n3, j = i % n3;
  const T *a0 = A + b * Nr * n3 + j;
  T a[NRM];
#pragma unroll
  for (int q = 0; q < NRM; ++q) a[q] = (q < Nr) ? a0[q * n3] : T(0);
  T *b0 = B + b * S * n3 + j;
  for (int s = 0; s < S; ++s) {
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < NRM; ++q) acc += us[s * NRM + q] * a[q];
    b0[s * n3] = acc;
  }
}

template <typename T>
static void launch_mix(const T *A, const T *U, T *B, long nitems, int S, int Nr, long n3, hipStream_t st) {
  const dim3 g(nblk(nitems * n3, 256)), blk(256);
  switch (mix_width(Nr)) {
    case 8: hipLaunchKernelGGL((k_mix<T, 8>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
    case 16: hipLaunchKernelGGL((k_mix<T, 16>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
    case 24: hipLaunchKernelGGL((k_mix<T, 24>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
    case 32: hipLaunchKernelGGL((k_mix<T, 32>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
    case 48: hipLaunchKernelGGL((k_mix<T, 48>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
    default: hipLaunchKernelGGL((k_mix<T, 64>), g, blk, 0, st, A, U, B, nitems, S, Nr, n3); break;
  }
}

// low-rank stage, slab pass: slab g = (b*npair + s)*N + j1, Z = B[2s] + i B[2s+1];
// the rows are read in the working precision T and transformed in U (FP64:
// the forward transform of the gain accumulators is where FP32 rounding costs
// most once gain and loss cancel)
template <typename T, int N, typename U = T>
struct SrcPair {
  const T *B;
  int S, npair;
  static constexpr bool kGroupedLoads = true;
  __device__ C<U> operator()(long g, int r, int c) const {
    const C<T> v = raw(g, r, c);
    return C<U>{U(v.re), U(v.im)};
  }
  __device__ C<T> raw(long g, int r, int c) const {
    constexpr long n3 = long(N) * N * N;
    const long t = g / N;
    const int j1 = int(g % N);
    const long b = t / npair;
    const int s = int(t % npair);
    const long o = (long(j1) * N + r) * N + c;
    // the odd row of the last pair may be missing (S odd): load the even row
    // again and select zero, so that every load is unconditional (a branch
    // per element would make each load wait for the previous one)
    const bool has_im = 2 * s + 1 < S;
    const T re = B[(b * S + 2 * s) * n3 + o];
    const T im_raw = B[(b * S + 2 * s + (has_im ? 1 : 0)) * n3 + o];
    const T im = has_im ? im_raw : T(0);
    return C<T>{re, im};
  }
};

// low-rank stage, pencil pass: forward along the first axis for each pair s,
// accumulating T += (V_2s - i V_2s+1) Z^_s (V already carries 1/N^3).
// With Z = B_2s + i B_2s+1 and V real and even, Re ifft(T) = sum_s C_s B_s.
// The low-rank stage (this pass and the slab pass before it) runs in FP64 in
// both precisions: gain and loss cancel by up to two orders of magnitude in Q,
// and an FP32 gain spectrum and inverse transform cost about 2e-5 of ||Q||, an
// FP32 forward transform of the accumulators about half of that.
template <typename T, int N>
struct OpLowRank {
  const C<double> *W;
  const T *V;
  C<double> *TA;
  int npair;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    T tr[N], ti[N];
    static_for<0, N>([&](auto k) { tr[decltype(k)::value] = T(0); ti[decltype(k)::value] = T(0); });
    for (int s = 0; s < npair; ++s) {
      const C<double> *w = W + (b * npair + s) * n3 + r;
      T xr[N], xi[N];
      static_for<0, N>([&](auto k) {
        const C<double> e = w[decltype(k)::value * n2];
        xr[decltype(k)::value] = T(e.re);
        xi[decltype(k)::value] = T(e.im);
      });
      fft_reg<N, -1, T>(xr, xi);
      const T *v0 = V + (2 * s) * n3 + r;
      const T *v1 = V + (2 * s + 1) * n3 + r;
      // the V rows in groups of KV values, each group's loads issued together
      // before its products (otherwise every pair of loads is waited for
      // alone); at N = 64 the accumulator and the pencil already fill the
      // register file, and the groups only add spills
      constexpr int KV = (N >= 64) ? N : ((N % 8 == 0) ? 8 : ((N % 6 == 0) ? 6 : 4));
      if constexpr (KV == N) {
        static_for<0, N>([&](auto k) {
          constexpr int kk = decltype(k)::value;
          const T a = v0[kk * n2], c = v1[kk * n2];
          tr[kk] += a * xr[kk] + c * xi[kk];
          ti[kk] += a * xi[kk] - c * xr[kk];
        });
      } else
      static_for<0, N / KV>([&](auto gg) {
        constexpr int k0 = decltype(gg)::value * KV;
        T av[KV], cv[KV];
        static_for<0, KV>([&](auto ii) {
          av[decltype(ii)::value] = v0[(k0 + decltype(ii)::value) * n2];
          cv[decltype(ii)::value] = v1[(k0 + decltype(ii)::value) * n2];
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, KV>([&](auto ii) {
          constexpr int kk = k0 + decltype(ii)::value;
          const T a = av[decltype(ii)::value], c = cv[decltype(ii)::value];
          // (a - i c)(xr + i xi) = (a xr + c xi) + i (a xi - c xr)
          tr[kk] += a * xr[kk] + c * xi[kk];
          ti[kk] += a * xi[kk] - c * xr[kk];
        });
      });
    }
    C<double> *o = TA + b * n3 + r;
    static_for<0, N>([&](auto k) {
      o[decltype(k)::value * n2] = C<double>{double(tr[decltype(k)::value]), double(ti[decltype(k)::value])};
    });
  }
};

// fused schedule: gain spectrum = sum over the radial nodes of the per-node
// half spectra W[b][p] (n_in float4 each) into the item's spectrum (n_out
// float4 apart); two complex values per lane (16-byte loads), node loop
// unrolled so that the loads of several nodes are in flight together
__global__ __launch_bounds__(256) void k_sum_nodes(const float4 *__restrict__ W, float4 *__restrict__ out,
                                                   long nitems, int Nr, long n_in, long n_out) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nitems * n_in) return;
  const long b = i / n_in, o = i % n_in;
  // each half spectrum is read once: streaming loads
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v *w = reinterpret_cast<const f4v *>(W + b * Nr * n_in + o);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
  for (int p = 0; p < Nr; ++p) {
    const f4v v = __builtin_nontemporal_load(w + p * n_in);
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  out[b * n_out + o] = acc;
}

// the same node sum of FP32 half spectra, accumulated and stored in FP64 (two
// complex values per lane: one 16-byte load per node, two 16-byte stores), so
// that the gain spectrum and its inverse transform stay in FP64
__global__ __launch_bounds__(256) void k_sum_nodes_wide(const float4 *__restrict__ W, double2 *__restrict__ out,
                                                        long nitems, int Nr, long n_in, long n_out) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nitems * n_in) return;
  const long b = i / n_in, o = i % n_in;
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v *w = reinterpret_cast<const f4v *>(W + b * Nr * n_in + o);
  double ax = 0.0, ay = 0.0, az = 0.0, aw = 0.0;
#pragma unroll 8
  for (int p = 0; p < Nr; ++p) {
    const f4v v = __builtin_nontemporal_load(w + p * n_in);
    ax += double(v.x);
    ay += double(v.y);
    az += double(v.z);
    aw += double(v.w);
  }
  double2 *d = out + 2 * (b * n_out + o);
  d[0] = make_double2(ax, ay);
  d[1] = make_double2(az, aw);
}

void launch_sum_nodes(const void *W, void *out, long nitems, int Nr, long n_in, long n_out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_nodes, dim3(nblk(nitems * n_in, 256)), dim3(256), 0, st,
                     static_cast<const float4 *>(W), static_cast<float4 *>(out), nitems, Nr, n_in, n_out);
}

// the same node sum for FP64 spectra: one complex value (16 bytes) per lane
__global__ __launch_bounds__(256) void k_sum_nodes64(const double2 *__restrict__ W, double2 *__restrict__ out,
                                                     long nitems, int Nr, long n_in, long n_out) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nitems * n_in) return;
  const long b = i / n_in, o = i % n_in;
  const double2 *w = W + b * Nr * n_in + o;
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
  for (int p = 0; p < Nr; ++p) {
    const double2 v = w[p * n_in];
    acc.x += v.x;
    acc.y += v.y;
  }
  out[b * n_out + o] = acc;
}

// Half spectra.  The gain and loss spectra are Hermitian (their inverse
// transforms are real), so the fused schedule keeps only the planes
// k1 <= N/2 of each item (half_slab, SrcCplxHalf, DstCplxHalf).

// loss, slab pass (FP64): Lambda * H64, slab g = item*N + k1
template <int N>
struct SrcLoss {
  const C<double> *H;
  const double *lam;
  __device__ C<double> operator()(long g, int r, int c) const {
    const long o = (g * N + r) * N + c;
    const double l = lam[((g % N) * N + r) * N + c];
    const C<double> h = H[o];
    return C<double>{h.re * l, h.im * l};
  }
};

// loss, slab pass over the half spectrum (FP64)
template <int N>
struct SrcLossHalf {
  const C<double> *H;
  const double *lam;
  __device__ C<double> operator()(long g, int r, int c) const {
    const long gf = half_slab<N>(g);
    const long o = (gf * N + r) * N + c;
    const double l = lam[((gf % N) * N + r) * N + c];
    const C<double> h = H[o];
    return C<double>{h.re * l, h.im * l};
  }
};

// final pencil pass: inverse along the first axis of the gain accumulator (T)
// and of the loss spectrum (FP64), then Q = Re(gain) - f * Re(loss) in FP64.
// With isc set, item b0 + b of the call is scaled by isc[(b0 + b) % K] (the
// collocation weights of the DG weak form, folded into this store).
// Second half of the assembly along one axis-1 pencil: Q = sc * (gain - f *
// ifft(L)) with gain the pencil's transformed gain spectrum, L the loss
// spectrum (all N planes, or with HALF the planes k1 <= N/2 of a Hermitian
// spectrum, completed in registers).  Up to N = 32 the gain values stay in
// registers; from N = 48 on (a pencil of N complex doubles is then 192 and more
// registers) they go to Q first and are read back by the same lane after the
// loss transform, which keeps one pencil live at a time instead of spilling.
template <int N, bool HALF = false>
__device__ __forceinline__ void assemble_loss(double (&out)[N], const C<double> *x1, const double *fb, double *qb,
                                              double sc) {
  constexpr long n2 = long(N) * N;
  constexpr int H1 = N / 2 + 1;
  constexpr bool SPLIT = N >= 48;
  if constexpr (SPLIT) static_for<0, N>([&](auto j) { qb[decltype(j)::value * n2] = out[decltype(j)::value]; });
  double lr[N], li[N];
  static_for<0, HALF ? H1 : N>([&](auto k) {
    const C<double> l = x1[decltype(k)::value * n2];
    lr[decltype(k)::value] = l.re;
    li[decltype(k)::value] = l.im;
  });
  if constexpr (HALF) {
    static_for<H1, N>([&](auto k) {
      lr[decltype(k)::value] = lr[N - decltype(k)::value];
      li[decltype(k)::value] = -li[N - decltype(k)::value];
    });
  }
  fft_reg<N, +1, double>(lr, li);
  // groups of G points: the group's loads of f (and of the stored gain) are
  // issued before its stores (Q may alias f as far as the compiler knows, so
  // a load after a store would wait for it)
  constexpr int G = (N % 8 == 0) ? 8 : 4;
  static_for<0, N / G>([&](auto gg) {
    constexpr int j0 = decltype(gg)::value * G;
    double fv[G], gv[G];
    static_for<0, G>([&](auto i) {
      constexpr int jj = j0 + decltype(i)::value;
      fv[decltype(i)::value] = fb[jj * n2];
      gv[decltype(i)::value] = SPLIT ? qb[jj * n2] : out[jj];
    });
    static_for<0, G>([&](auto i) {
      constexpr int jj = j0 + decltype(i)::value;
      double o = gv[decltype(i)::value];
      o -= fv[decltype(i)::value] * lr[jj];
      qb[jj * n2] = sc * o;
    });
  });
}

template <typename T, int N>
struct OpAssemble {
  const C<T> *TA;
  const C<double> *LH;
  const double *f;
  double *Q;
  const double *isc;
  int K;
  long b0;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    double out[N];
    {
      T ar[N], ai[N];
      const C<T> *x0 = TA + b * n3 + r;
      static_for<0, N>([&](auto k) {
        const C<T> a = x0[decltype(k)::value * n2];
        ar[decltype(k)::value] = a.re;
        ai[decltype(k)::value] = a.im;
      });
      fft_reg<N, +1, T>(ar, ai);
      static_for<0, N>([&](auto j) { out[decltype(j)::value] = double(ar[decltype(j)::value]); });
    }
    assemble_loss<N>(out, LH + b * n3 + r, f + b * n3 + r, Q + b * n3 + r, isc ? isc[(b0 + b) % K] : 1.0);
  }
};

// the same assembly from half spectra: after the slab passes, plane N - k1
// of a Hermitian spectrum is the complex conjugate of plane k1 at the same
// (j2, j3), so each pencil is completed in registers before its transform
template <typename T, int N>
struct OpAssembleHalf {
  const C<T> *TA;
  const C<double> *LH;
  const double *f;
  double *Q;
  const double *isc;
  int K;
  long b0;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    constexpr int H1 = N / 2 + 1;
    double out[N];
    {
      T ar[N], ai[N];
      const C<T> *x0 = TA + b * n3 + r;
      static_for<0, H1>([&](auto k) {
        const C<T> a = x0[decltype(k)::value * n2];
        ar[decltype(k)::value] = a.re;
        ai[decltype(k)::value] = a.im;
      });
      static_for<H1, N>([&](auto k) {
        ar[decltype(k)::value] = ar[N - decltype(k)::value];
        ai[decltype(k)::value] = -ai[N - decltype(k)::value];
      });
      fft_reg<N, +1, T>(ar, ai);
      static_for<0, N>([&](auto j) { out[decltype(j)::value] = double(ar[decltype(j)::value]); });
    }
    assemble_loss<N, true>(out, LH + b * n3 + r, f + b * n3 + r, Q + b * n3 + r, isc ? isc[(b0 + b) % K] : 1.0);
  }
};

// ----------------------------------------------------------------------------
// VSS kernels (sigma-dependent kernel modes): every (item, p, q) term is
// transformed forward and weighted by its own alpha_pq before the sums.
//
// Pencil pass over Y[(pair, q)] (after the shifted slab pass): inverse along
// axis 1, the product t = Re(u)^2 - Im(u)^2 = t1 t2 (the weights w_p w_q sit
// in alpha_pq), then the forward transform of the real t along axis 1; only
// the planes k1 <= N/2 are written back (t is real, so its spectrum is
// Hermitian and the slab pass below needs no other plane).
template <typename T, int N>
struct OpGainVss {
  C<T> *Y;
  int M;
  __device__ void operator()(long v, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    C<T> *y = Y + v * n3 + r;
    T xr[N], xi[N];
    static_for<0, N>([&](auto k) {
      const C<T> e = y[decltype(k)::value * n2];
      xr[decltype(k)::value] = e.re;
      xi[decltype(k)::value] = e.im;
    });
    fft_reg<N, +1, T>(xr, xi);
    static_for<0, N>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      const T t = xr[jj] * xr[jj] - xi[jj] * xi[jj];
      xr[jj] = t;
      xi[jj] = T(0);
    });
    fft_reg<N, -1, T>(xr, xi);
    static_for<0, N / 2 + 1>([&](auto k) {
      y[decltype(k)::value * n2] = C<T>{xr[decltype(k)::value], xi[decltype(k)::value]};
    });
  }
};

// The same pass for the bilinear Q(f, g): Yf and Yg hold the shifted volumes
// of f and g; the product is Re(u_f u_g) = (t1_f t2_g + t2_f t1_g) / 2, stored
// (forward along axis 1, planes k1 <= N/2) in Yf.
template <typename T, int N>
struct OpGainVss2 {
  C<T> *Yf;
  const C<T> *Yg;
  int M;
  __device__ void operator()(long v, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    C<T> *y = Yf + v * n3 + r;
    const C<T> *yg = Yg + v * n3 + r;
    T xr[N], xi[N];
    {
      T gr[N], gi[N];
      static_for<0, N>([&](auto k) {
        const C<T> e = yg[decltype(k)::value * n2];
        gr[decltype(k)::value] = e.re;
        gi[decltype(k)::value] = e.im;
      });
      fft_reg<N, +1, T>(gr, gi);
      static_for<0, N>([&](auto k) {
        const C<T> e = y[decltype(k)::value * n2];
        xr[decltype(k)::value] = e.re;
        xi[decltype(k)::value] = e.im;
      });
      fft_reg<N, +1, T>(xr, xi);
      static_for<0, N>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        const T t = xr[jj] * gr[jj] - xi[jj] * gi[jj];
        xr[jj] = t;
        xi[jj] = T(0);
      });
    }
    fft_reg<N, -1, T>(xr, xi);
    static_for<0, N / 2 + 1>([&](auto k) {
      y[decltype(k)::value * n2] = C<T>{xr[decltype(k)::value], xi[decltype(k)::value]};
    });
  }
};

// Slab accumulation: W[pair] plane k1 (<= N/2) = sum_q alpha_pq(k) fft2(Y[(pair, q)] plane k1)
// over the (j2, j3) axes.  The M terms of a plane are split in kVssParts fixed
// parts (blockIdx.y): part 0's sum goes to W, part i's to Wp[i - 1] (launch
// relative), and k_vss_acc_add forms ((part 0 + part 1) + ...), so several
// workgroups share a plane's loads while every pair's result is independent of
// the launch sizes.  One workgroup owns SPB planes; lane (s, c) owns column c of
// plane s (as in the generic slab kernel: column transform from the coalesced
// loads, row transform through LDS) and keeps that column's sums in registers.
constexpr int kVssParts = 4;

template <typename T, int N>
__global__ __launch_bounds__(256) void k_vss_acc(const C<T> *Y, const T *apq, C<T> *W, C<T> *Wp, long bp0,
                                                 long npair, int M, int Nr) {
  constexpr int SPB = slab_spb2<T, N>();
  constexpr int H1 = N / 2 + 1;
  constexpr long n2 = long(N) * N, n3 = n2 * N, nh = long(H1) * n2;
  __shared__ T sre[SPB][N][N + 1];
  __shared__ T sim[SPB][N][N + 1];
  const int s = int(threadIdx.x) / N, c = int(threadIdx.x) % N;
  const long nz = npair * H1;
  const long z = long(blockIdx.x) * SPB + s;   // (pair, k1) plane
  const long zl = z < nz ? z : nz - 1;
  const long pl = zl / H1;
  const int k1 = int(zl % H1);
  const int p = int((bp0 + pl) % Nr);
  T ar[N], ai[N];
  static_for<0, N>([&](auto k) { ar[decltype(k)::value] = T(0); ai[decltype(k)::value] = T(0); });
  const int part = int(blockIdx.y);
  const int q0 = (part * M) / kVssParts, q1 = ((part + 1) * M) / kVssParts;
  for (int q = q0; q < q1; ++q) {
    const C<T> *y = Y + (pl * M + q) * n3 + long(k1) * n2 + c;
    T xr[N], xi[N];
    static_for<0, N>([&](auto r) {
      const C<T> v = y[decltype(r)::value * N];
      xr[decltype(r)::value] = v.re;
      xi[decltype(r)::value] = v.im;
    });
    // the term's weights for this column, loaded before the two transforms
    // hide their latency (loaded where they are used, each was waited for
    // alone); not where the extra registers cost occupancy or spill (FP64
    // at N = 24 and 48)
    constexpr bool PRE = (sizeof(T) == 4) ? (N <= 48) : (N == 32);
    const T *a = apq + (size_t(p) * M + q) * nh + long(k1) * n2 + c;
    T wv[PRE ? N : 1];
    if constexpr (PRE) static_for<0, N>([&](auto r) { wv[decltype(r)::value] = a[decltype(r)::value * N]; });
    fft_reg<N, -1, T>(xr, xi);
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
    fft_reg<N, -1, T>(xr, xi);
    static_for<0, N>([&](auto k) {
      sre[s][row][decltype(k)::value] = xr[decltype(k)::value];
      sim[s][row][decltype(k)::value] = xi[decltype(k)::value];
    });
    __syncthreads();
    static_for<0, N>([&](auto r) {
      constexpr int rr = decltype(r)::value;
      T w;
      if constexpr (PRE) w = wv[rr];
      else w = a[rr * N];
      ar[rr] += w * sre[s][rr][c];
      ai[rr] += w * sim[s][rr][c];
    });
    __syncthreads();
  }
  if (z < nz) {
    C<T> *wo = (part == 0 ? W : Wp + (part - 1) * npair * nh) + pl * nh + long(k1) * n2 + c;
    static_for<0, N>([&](auto r) { wo[decltype(r)::value * N] = C<T>{ar[decltype(r)::value], ai[decltype(r)::value]}; });
  }
}

// W[i] = ((W[i] + Wp[0][i]) + Wp[1][i]) + ... for the n values of a launch
template <typename T>
__global__ __launch_bounds__(256) void k_vss_acc_add(C<T> *W, const C<T> *Wp, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  C<T> a = W[i];
#pragma unroll
  for (int k = 0; k < kVssParts - 1; ++k) {
    const C<T> b = Wp[k * n + i];
    a.re += b.re;
    a.im += b.im;
  }
  W[i] = a;
}

// ----------------------------------------------------------------------------
// Literal Nyquist convention: the shift factor at frequency -N/2 is the complex
// exp(i pi k s / L), so beta_s X is no longer Hermitian and the shifted copies
// t1 = ifft(beta_s X), t2 = ifft(conj(beta_s) X) are complex.  With
// a = ifft(Re(beta_s) X) and b = ifft(Im(beta_s) X) (each complex now),
// t1 t2 = (a + i b)(a - i b) = a a + b b, the Appendix's cos/sin form, so each
// term takes two inverse transforms and a complex product; the gain
// accumulators A_p and the low-rank stage are complex, and Q = Re(Q+ - Q-).

// slab pass: H times Re(beta_s) (IM = false) or Im(beta_s) (IM = true), with
// beta_s = b1 b2 b3 formed from b1 b3 once per lane and column (as SrcShift)
template <typename T, int N, bool IM>
struct SrcShiftPart {
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
    const T x13 = (b1.re * b3.re - b1.im * b3.im) * scale, y13 = (b1.re * b3.im + b1.im * b3.re) * scale;
    const T m = IM ? (b2.re * y13 + b2.im * x13) : (b2.re * x13 - b2.im * y13);
    const C<T> h = H[((b * N + k1) * N + r) * N + c];
    return C<T>{h.re * m, h.im * m};
  }
};

// pencil pass: inverse along axis 1 of the a and b volumes of every q (one
// pencil held at a time), A_p += w_q (a a + b b), complex A_p stored
template <typename T, int N>
struct OpGainAccLit {
  const C<T> *Ya, *Yb;
  const T *wq;
  C<T> *A;
  long bp0;
  int M;
  __device__ void operator()(long bpl, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    T accr[N], acci[N];
    static_for<0, N>([&](auto j) { accr[decltype(j)::value] = T(0); acci[decltype(j)::value] = T(0); });
    for (int q = 0; q < M; ++q) {
      const T w = wq[q];
      for (int part = 0; part < 2; ++part) {
        const C<T> *y = (part ? Yb : Ya) + (bpl * M + q) * n3 + r;
        T xr[N], xi[N];
        static_for<0, N>([&](auto k) {
          const C<T> v = y[decltype(k)::value * n2];
          xr[decltype(k)::value] = v.re;
          xi[decltype(k)::value] = v.im;
        });
        fft_reg<N, +1, T>(xr, xi);
        static_for<0, N>([&](auto j) {
          constexpr int jj = decltype(j)::value;
          accr[jj] += w * (xr[jj] * xr[jj] - xi[jj] * xi[jj]);
          acci[jj] += T(2) * w * (xr[jj] * xi[jj]);
        });
      }
    }
    C<T> *a = A + (bp0 + bpl) * n3 + r;
    static_for<0, N>([&](auto j) { a[decltype(j)::value * n2] = C<T>{accr[decltype(j)::value], acci[decltype(j)::value]}; });
  }
};

// low-rank stage for complex accumulators: forward along axis 1 of each of
// the S complex volumes B_s of an item (after the forward slab pass), times
// the real weights V_s (already / N^3), summed into the FP64 gain spectrum
template <typename T, int N>
struct OpLowRankC {
  const C<T> *W;
  const T *V;
  C<double> *TA;
  int S;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    double tr[N], ti[N];
    static_for<0, N>([&](auto k) { tr[decltype(k)::value] = 0.0; ti[decltype(k)::value] = 0.0; });
    for (int s = 0; s < S; ++s) {
      const C<T> *w = W + (b * S + s) * n3 + r;
      T xr[N], xi[N];
      static_for<0, N>([&](auto k) {
        const C<T> e = w[decltype(k)::value * n2];
        xr[decltype(k)::value] = e.re;
        xi[decltype(k)::value] = e.im;
      });
      fft_reg<N, -1, T>(xr, xi);
      const T *v = V + s * n3 + r;
      static_for<0, N>([&](auto k) {
        constexpr int kk = decltype(k)::value;
        const T a = v[kk * n2];
        tr[kk] += double(a * xr[kk]);
        ti[kk] += double(a * xi[kk]);
      });
    }
    C<double> *o = TA + b * n3 + r;
    static_for<0, N>([&](auto k) {
      o[decltype(k)::value * n2] = C<double>{tr[decltype(k)::value], ti[decltype(k)::value]};
    });
  }
};

// ----------------------------------------------------------------------------
template <typename T, int N>
struct Engine {
  using P = Passes<T, N>;
  static constexpr long n3 = P::n3;
  template <class Src, class Dst, int SIGN>
  static qcoll_status slab(Src s, Dst d, long nslab, hipStream_t st, const char *what) {
    return P::template slab<Src, Dst, SIGN>(s, d, nslab, st, what);
  }
  template <class Op>
  static qcoll_status pencil(Op op, long npencil, hipStream_t st, const char *what) {
    return P::pencil(op, npencil, st, what);
  }

  // A[b][p] for items of this chunk: (b, p) pairs bp in [0, nb*Nr)
  static qcoll_status gain_terms(const Plan &p, const C<T> *H, T *A, C<T> *Y, long nb, long pc,
                                 hipStream_t st) {
    const long nbp = nb * p.N_rho;
    if constexpr (std::is_same<T, double>::value) {
      if (use_gain_q64(p)) return launch_gain_q64(p, H, A, nbp, st);
    }
    const T scale = T(1.0 / double(n3));
    for (long bp0 = 0; bp0 < nbp; bp0 += pc) {
      const long cnt = (nbp - bp0 < pc) ? (nbp - bp0) : pc;
      SrcShift<T, N> src{H, reinterpret_cast<const C<T> *>(p.phase), bp0, p.M, p.N_rho, scale};
      qcoll_status s;
      if ((s = slab<SrcShift<T, N>, DstCplx<T, N>, +1>(src, DstCplx<T, N>{Y}, cnt * p.M * N, st, "gain slab")))
        return s;
      if constexpr (gain_pencil_parts<T, N>()) {
        TimedLaunch tl("gain pencil", st);
        hipLaunchKernelGGL((k_gain_pencil_parts<T, N>), dim3(unsigned(cnt * N * N / 64)), dim3(64 * kGainParts), 0,
                           st, Y, reinterpret_cast<const T *>(p.wq), A, bp0, p.M);
        QC_LAUNCH_CHECK("gain pencil");
      } else {
        OpGainAcc<T, N> op{Y, reinterpret_cast<const T *>(p.wq), A, bp0, p.M};
        if ((s = pencil(op, cnt * N * N, st, "gain pencil"))) return s;
      }
    }
    return QCOLL_OK;
  }

  // bilinear gain terms: both spectra through the slab pass, products in the pencil pass
  static qcoll_status gain_terms2(const Plan &p, const C<T> *Hf, const C<T> *Hg, T *A, C<T> *Yf, C<T> *Yg, long nb,
                                  long pc, hipStream_t st) {
    const long nbp = nb * p.N_rho;
    const T scale = T(1.0 / double(n3));
    for (long bp0 = 0; bp0 < nbp; bp0 += pc) {
      const long cnt = (nbp - bp0 < pc) ? (nbp - bp0) : pc;
      qcoll_status s;
      SrcShift<T, N> sf{Hf, reinterpret_cast<const C<T> *>(p.phase), bp0, p.M, p.N_rho, scale};
      SrcShift<T, N> sg{Hg, reinterpret_cast<const C<T> *>(p.phase), bp0, p.M, p.N_rho, scale};
      if ((s = slab<SrcShift<T, N>, DstCplx<T, N>, +1>(sf, DstCplx<T, N>{Yf}, cnt * p.M * N, st, "gain slab")))
        return s;
      if ((s = slab<SrcShift<T, N>, DstCplx<T, N>, +1>(sg, DstCplx<T, N>{Yg}, cnt * p.M * N, st, "gain slab")))
        return s;
      OpGainAcc2<T, N> op{Yf, Yg, reinterpret_cast<const T *>(p.wq), A, bp0, p.M};
      if ((s = pencil(op, cnt * N * N, st, "gain pencil"))) return s;
    }
    return QCOLL_OK;
  }

  // VSS: per (item, node) pair, the shifted slab pass, the pencil pass to the
  // product and back to the spectrum along axis 1, and the weighted slab
  // accumulation over q into the pair's half spectrum W; then the node sum and
  // the half-spectrum tail of the fused schedule.
  // (Hg, H64g, Yg non-null: the bilinear Q(f, g), two-pass in both precisions)
  static qcoll_status eval_vss(const Plan &p, const C<T> *H, const C<double> *H64, T *A, C<T> *Y, C<double> *TA,
                               C<T> *VP, C<double> *LH, const double *fb, double *Qb, long nb, long pc,
                               hipStream_t st, const double *isc, int K, long b0, const C<T> *Hg = nullptr,
                               const C<double> *H64g = nullptr, C<T> *Yg = nullptr) {
    constexpr int H1 = N / 2 + 1;
    constexpr long nh = long(H1) * N * N;
    constexpr int SPB = slab_spb2<T, N>();
    C<T> *Wp = reinterpret_cast<C<T> *>(A);
    const long nbp = nb * p.N_rho;
    const T scale = T(1.0 / double(n3));
    qcoll_status s;
    // FP32 with N <= 32: the whole per-pair loop on chip (fused kernel, VSS mode)
    const bool fused = std::is_same<T, float>::value && use_fused_gain(p) && !Hg;
    if (fused && (s = launch_gain_fused(p, H, Wp, nbp, st))) return s;
    for (long bp0 = 0; !fused && bp0 < nbp; bp0 += pc) {
      const long cnt = (nbp - bp0 < pc) ? (nbp - bp0) : pc;
      SrcShift<T, N> src{H, reinterpret_cast<const C<T> *>(p.phase), bp0, p.M, p.N_rho, scale};
      if ((s = slab<SrcShift<T, N>, DstCplx<T, N>, +1>(src, DstCplx<T, N>{Y}, cnt * p.M * N, st, "gain slab")))
        return s;
      if (Hg) {
        SrcShift<T, N> sg{Hg, reinterpret_cast<const C<T> *>(p.phase), bp0, p.M, p.N_rho, scale};
        if ((s = slab<SrcShift<T, N>, DstCplx<T, N>, +1>(sg, DstCplx<T, N>{Yg}, cnt * p.M * N, st, "gain slab")))
          return s;
        if ((s = pencil(OpGainVss2<T, N>{Y, Yg, p.M}, cnt * p.M * N * N, st, "vss pencil"))) return s;
      } else if ((s = pencil(OpGainVss<T, N>{Y, p.M}, cnt * p.M * N * N, st, "vss pencil"))) {
        return s;
      }
      TimedLaunch tl("vss acc", st);
      hipLaunchKernelGGL((k_vss_acc<T, N>), dim3(nblk(cnt * H1, SPB), kVssParts), dim3(SPB * N), 0, st, Y,
                         reinterpret_cast<const T *>(p.alpha_pq), Wp + bp0 * nh, VP, bp0, cnt, p.M, p.N_rho);
      hipLaunchKernelGGL((k_vss_acc_add<T>), dim3(nblk(cnt * nh, 256)), dim3(256), 0, st, Wp + bp0 * nh, VP,
                         cnt * nh);
      QC_LAUNCH_CHECK("vss acc");
    }
    {
      TimedLaunch tl("sum nodes", st);
      if constexpr (std::is_same<T, float>::value) {
        hipLaunchKernelGGL(k_sum_nodes_wide, dim3(nblk(nb * (nh / 2), 256)), dim3(256), 0, st,
                           reinterpret_cast<const float4 *>(Wp), reinterpret_cast<double2 *>(TA), nb, p.N_rho, nh / 2,
                           n3 / 2);
      } else {
        hipLaunchKernelGGL(k_sum_nodes64, dim3(nblk(nb * nh, 256)), dim3(256), 0, st,
                           reinterpret_cast<const double2 *>(Wp), reinterpret_cast<double2 *>(TA), nb, p.N_rho, nh,
                           n3);
      }
      QC_LAUNCH_CHECK("sum nodes");
    }
    if ((s = Passes<double, N>::template slab<SrcCplxHalf<double, N>, DstCplxHalf<double, N>, +1>(
             SrcCplxHalf<double, N>{TA}, DstCplxHalf<double, N>{TA}, nb * H1, st, "gain inverse slab")))
      return s;
    if ((s = Passes<double, N>::template slab<SrcLossHalf<N>, DstCplxHalf<double, N>, +1>(
             SrcLossHalf<N>{H64g ? H64g : H64, reinterpret_cast<const double *>(p.lam)}, DstCplxHalf<double, N>{LH},
             nb * H1, st, "loss slab")))
      return s;
    return pencil(OpAssembleHalf<double, N>{TA, LH, fb, Qb, isc, K, b0}, nb * N * N, st, "assemble");
  }

  // literal Nyquist convention (two-pass, complex intermediates), see above
  static qcoll_status eval_literal(const Plan &p, const C<T> *H, const C<double> *H64, T *Ar, T *Br, C<T> *W,
                                   C<double> *TA, C<double> *LH, C<T> *Ya, C<T> *Yb, const double *fb, double *Qb,
                                   long nb, long pc, hipStream_t st, const double *isc, int K, long b0) {
    C<T> *A = reinterpret_cast<C<T> *>(Ar);
    const long nbp = nb * p.N_rho;
    const T scale = T(1.0 / double(n3));
    const C<T> *ph = reinterpret_cast<const C<T> *>(p.phase);
    qcoll_status s;
    for (long bp0 = 0; bp0 < nbp; bp0 += pc) {
      const long cnt = (nbp - bp0 < pc) ? (nbp - bp0) : pc;
      SrcShiftPart<T, N, false> sa{H, ph, bp0, p.M, p.N_rho, scale};
      SrcShiftPart<T, N, true> sb{H, ph, bp0, p.M, p.N_rho, scale};
      if ((s = slab<SrcShiftPart<T, N, false>, DstCplx<T, N>, +1>(sa, DstCplx<T, N>{Ya}, cnt * p.M * N, st,
                                                                   "gain slab")))
        return s;
      if ((s = slab<SrcShiftPart<T, N, true>, DstCplx<T, N>, +1>(sb, DstCplx<T, N>{Yb}, cnt * p.M * N, st,
                                                                  "gain slab")))
        return s;
      OpGainAccLit<T, N> op{Ya, Yb, reinterpret_cast<const T *>(p.wq), A, bp0, p.M};
      if ((s = pencil(op, cnt * N * N, st, "gain pencil"))) return s;
    }
    // rows of the low-rank stage: B_s = sum_p U_sp A_p (complex: re and im mixed alike)
    const C<T> *Bsrc = A;
    const int S = p.nv;
    if (!p.mix_identity) {
      TimedLaunch tl("mix", st);
      launch_mix<T>(Ar, reinterpret_cast<const T *>(p.umix_d), Br, nb, S, p.N_rho, 2 * n3, st);
      QC_LAUNCH_CHECK("mix");
      Bsrc = reinterpret_cast<const C<T> *>(Br);
    }
    // the low-rank stage in FP64 (the workspace row W holds FP64 volumes)
    C<double> *Wd = reinterpret_cast<C<double> *>(W);
    if ((s = Passes<double, N>::template slab<SrcCplxWide<T, N, double>, DstCplx<double, N>, -1>(
             SrcCplxWide<T, N, double>{Bsrc}, DstCplx<double, N>{Wd}, nb * S * N, st, "low-rank slab")))
      return s;
    if ((s = pencil(OpLowRankC<double, N>{Wd, p.v64(), TA, S}, nb * N * N, st, "low-rank pencil"))) return s;
    if ((s = Passes<double, N>::template slab<SrcCplx<double, N>, DstCplx<double, N>, +1>(
             SrcCplx<double, N>{TA}, DstCplx<double, N>{TA}, nb * N, st, "gain inverse slab")))
      return s;
    if ((s = Passes<double, N>::template slab<SrcLoss<N>, DstCplx<double, N>, +1>(
             SrcLoss<N>{H64, reinterpret_cast<const double *>(p.lam)}, DstCplx<double, N>{LH}, nb * N, st,
             "loss slab")))
      return s;
    return pencil(OpAssemble<double, N>{TA, LH, fb, Qb, isc, K, b0}, nb * N * N, st, "assemble");
  }

  // Q(f, f), or the bilinear Q(f, g) when g is non-null (two-pass schedule)
  static qcoll_status eval(const Plan &p, int64_t batch, const double *f, const double *g, double *Q, void *ws,
                           const Layout &lay, hipStream_t st, const double *isc, int K) {
    char *w = static_cast<char *>(ws);
    C<T> *Hg = reinterpret_cast<C<T> *>(w + lay.off_hg);
    C<double> *H64g = reinterpret_cast<C<double> *>(w + lay.off_h64g);
    C<T> *Yg = reinterpret_cast<C<T> *>(w + lay.off_yg);
    C<T> *H = reinterpret_cast<C<T> *>(w + lay.off_h);
    C<double> *H64 = reinterpret_cast<C<double> *>(w + lay.off_h64);
    T *A = reinterpret_cast<T *>(w + lay.off_a);
    T *B = reinterpret_cast<T *>(w + lay.off_b);
    C<T> *W = reinterpret_cast<C<T> *>(w + lay.off_w);
    C<double> *TA = reinterpret_cast<C<double> *>(w + lay.off_t);   // gain spectrum, FP64 in both precisions
    C<double> *LH = reinterpret_cast<C<double> *>(w + lay.off_l);
    C<T> *Y = reinterpret_cast<C<T> *>(w + lay.off_y);
    C<T> *VP = reinterpret_cast<C<T> *>(w + lay.off_vp);
    const int S = p.nv, np = p.npair();
    for (long b0 = 0; b0 < batch; b0 += lay.bc) {
      const long nb = (batch - b0 < lay.bc) ? (batch - b0) : lay.bc;
      const double *fb = f + b0 * n3;
      qcoll_status s;
      // spectrum of f in FP64 (shared by the gain and the loss), and its copy
      // in the working precision for the gain
      if constexpr (!std::is_same<T, double>::value) {
        if ((s = Passes<double, N>::template forward_to<T>(fb, H64, H, nb, st))) return s;
      } else {
        if ((s = Passes<double, N>::forward(fb, H64, nb, st))) return s;
      }
      if constexpr (N <= 48) {   // VSS kernels: N <= 48 (the plan refuses larger grids)
        if (p.is_vss()) {
          if (g && (s = Passes<double, N>::template forward_to<T>(g + b0 * n3, H64g, Hg, nb, st))) return s;
          if ((s = eval_vss(p, H, H64, A, Y, TA, VP, LH, fb, Q + b0 * n3, nb, lay.pc, st, isc, K, b0,
                            g ? Hg : nullptr, g ? H64g : nullptr, g ? Yg : nullptr)))
            return s;
          continue;
        }
      }
      if (p.literal) {
        if ((s = eval_literal(p, H, H64, A, B, W, TA, LH, Y, Yg, fb, Q + b0 * n3, nb, lay.pc, st, isc, K, b0)))
          return s;
        continue;
      }
      if (g) {
        // bilinear Q(f, g): gain from both spectra, loss f * ifft(Lambda g^)
        const double *gb = g + b0 * n3;
        if ((s = Passes<double, N>::template forward_to<T>(gb, H64g, Hg, nb, st))) return s;
        if ((s = gain_terms2(p, H, Hg, A, Y, Yg, nb, lay.pc, st))) return s;
      } else if constexpr (std::is_same<T, float>::value) {
        if (use_fused_gain(p)) {
          // gain terms and the low-rank stage on chip; W[b][p] = alpha_p fft3(A_p)
          C<T> *Wp = reinterpret_cast<C<T> *>(A);
          if ((s = launch_gain_fused(p, H, Wp, nb * p.N_rho, st))) return s;
          // half spectra from here on: planes k1 <= N/2 of every item
          constexpr long nh = long(N / 2 + 1) * N * N;
          constexpr int H1 = N / 2 + 1;
          {
            // nh and n3 are even for every supported N, so the float4 view is exact
            TimedLaunch tl("sum nodes", st);
            hipLaunchKernelGGL(k_sum_nodes_wide, dim3(nblk(nb * (nh / 2), 256)), dim3(256), 0, st,
                               reinterpret_cast<const float4 *>(Wp), reinterpret_cast<double2 *>(TA), nb, p.N_rho,
                               nh / 2, n3 / 2);
            QC_LAUNCH_CHECK("sum nodes");
          }
          if ((s = Passes<double, N>::template slab<SrcCplxHalf<double, N>, DstCplxHalf<double, N>, +1>(
                   SrcCplxHalf<double, N>{TA}, DstCplxHalf<double, N>{TA}, nb * H1, st, "gain inverse slab")))
            return s;
          if ((s = Passes<double, N>::template slab<SrcLossHalf<N>, DstCplxHalf<double, N>, +1>(
                   SrcLossHalf<N>{H64, reinterpret_cast<const double *>(p.lam)}, DstCplxHalf<double, N>{LH}, nb * H1,
                   st, "loss slab")))
            return s;
          if ((s = pencil(OpAssembleHalf<double, N>{TA, LH, fb, Q + b0 * n3, isc, K, b0}, nb * N * N, st, "assemble")))
            return s;
          continue;
        }
        if ((s = gain_terms(p, H, A, Y, nb, lay.pc, st))) return s;
      } else {
        if ((s = gain_terms(p, H, A, Y, nb, lay.pc, st))) return s;
      }
      const T *Bsrc = A;
      if (!p.mix_identity) {
        TimedLaunch tl("mix", st);
        launch_mix<T>(A, reinterpret_cast<const T *>(p.umix_d), B, nb, S, p.N_rho, n3, st);
        QC_LAUNCH_CHECK("mix");
        Bsrc = B;
      }
      // the low-rank stage in FP64 in both precisions (W holds FP64 volumes)
      C<double> *Wd = reinterpret_cast<C<double> *>(W);
      if ((s = Passes<double, N>::template slab<SrcPair<T, N, double>, DstCplx<double, N>, -1>(
               SrcPair<T, N, double>{Bsrc, S, np}, DstCplx<double, N>{Wd}, nb * np * N, st, "low-rank slab")))
        return s;
      OpLowRank<double, N> lr{Wd, p.v64(), TA, np};
      if ((s = pencil(lr, nb * N * N, st, "low-rank pencil"))) return s;
      if ((s = Passes<double, N>::template slab<SrcCplx<double, N>, DstCplx<double, N>, +1>(
               SrcCplx<double, N>{TA}, DstCplx<double, N>{TA}, nb * N, st, "gain inverse slab")))
        return s;
      if ((s = Passes<double, N>::template slab<SrcLoss<N>, DstCplx<double, N>, +1>(
               SrcLoss<N>{g ? H64g : H64, reinterpret_cast<const double *>(p.lam)}, DstCplx<double, N>{LH}, nb * N,
               st, "loss slab")))
        return s;
      if ((s = pencil(OpAssemble<double, N>{TA, LH, fb, Q + b0 * n3, isc, K, b0}, nb * N * N, st, "assemble")))
        return s;
    }
    return QCOLL_OK;
  }
};

// ----------------------------------------------------------------------------
// FP64 conservation projection: one 1024-lane workgroup per item.  Each lane
// walks pairs of consecutive points along the last axis (16-byte loads); the
// velocity of a point is rebuilt from its index.  The five sums are reduced
// in a fixed order, so the result is deterministic.  With PPT > 0 (grids up
// to 32^3: at most 16 pairs per lane) a lane keeps its PPT pairs in registers
// between the sums and the correction, so Q is read once; PPT = 0 reads it
// twice.  Both visit a lane's pairs in the same order: the results are
// bit-identical.  NC > 0 fixes N at compile time, so that rebuilding a point's
// indices takes shifts and multiplications instead of integer divisions by a
// runtime value (which dominated the kernel's instruction count).
constexpr int kConserveBlock = 1024;   // lanes per workgroup of k_conserve

template <int PPT, int NC = 0>
__global__ __launch_bounds__(kConserveBlock) void k_conserve(double *Q, double *mom, const double *ginv, int Nrt, double L,
                                                   int *flag, double dc3, const double *isc, int K) {
  const int N = NC > 0 ? NC : Nrt;
  const long n3 = long(N) * N * N;
  const long b = blockIdx.x;
  double2 *q = reinterpret_cast<double2 *>(Q + b * n3);
  const double dc = 2.0 * L / N;
  const long nh = n3 / 2;   // N is even: a pair never crosses a row
  auto coords = [&](long h, double &c1, double &c2, double &c3a, double &c3b) {
    const long j = 2 * h;
    const int i1 = int(j / (N * N)), i2 = int((j / N) % N), i3 = int(j % N);
    c1 = -L + (i1 + 0.5) * dc;
    c2 = -L + (i2 + 0.5) * dc;
    c3a = -L + (i3 + 0.5) * dc;
    c3b = c3a + dc;
  };
  double s[5] = {0, 0, 0, 0, 0};
  auto add = [&](long h, double2 v) {
    double c1, c2, c3a, c3b;
    coords(h, c1, c2, c3a, c3b);
    const double sv = v.x + v.y;
    const double r12 = c1 * c1 + c2 * c2;
    s[0] += sv;
    s[1] += sv * c1;
    s[2] += sv * c2;
    s[3] += v.x * c3a + v.y * c3b;
    s[4] += v.x * (r12 + c3a * c3a) + v.y * (r12 + c3b * c3b);
  };
  double2 keep[PPT > 0 ? PPT : 1];
  if constexpr (PPT > 0) {
    // every load is issued before the first sum: the index is clamped instead
    // of guarded (a guarded load sits in a branch of its own, and the compiler
    // then waits for each load before the next one is issued)
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const long h = threadIdx.x + long(i) * kConserveBlock;
      keep[i] = q[h < nh ? h : nh - 1];
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const long h = threadIdx.x + long(i) * kConserveBlock;
      if (h < nh) add(h, keep[i]);
    }
  } else {
    for (long h = threadIdx.x; h < nh; h += blockDim.x) add(h, q[h]);
  }
  __shared__ double red[5][1024];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  double m[5], lam[5];
  for (int k = 0; k < 5; ++k) m[k] = red[k][0];
  const double sc = isc ? isc[b % K] : 1.0;   // projection first, then the item's weight
  for (int a = 0; a < 5; ++a) {
    double acc = 0;
    for (int c = 0; c < 5; ++c) acc += ginv[a * 5 + c] * m[c];
    lam[a] = acc;
  }
  bool finite = true;
  for (int k = 0; k < 5; ++k) finite = finite && isfinite(m[k]);
  if (threadIdx.x == 0) {
    if (mom)
      for (int k = 0; k < 5; ++k) mom[b * 5 + k] = m[k] * dc3;
    if (!finite) atomicOr(flag, 1);
  }
  auto fix = [&](long h, double2 v) {
    double c1, c2, c3a, c3b;
    coords(h, c1, c2, c3a, c3b);
    const double base = lam[0] + lam[1] * c1 + lam[2] * c2 + lam[4] * (c1 * c1 + c2 * c2);
    v.x -= base + lam[3] * c3a + lam[4] * c3a * c3a;
    v.y -= base + lam[3] * c3b + lam[4] * c3b * c3b;
    v.x *= sc;
    v.y *= sc;
    q[h] = v;
  };
  if constexpr (PPT > 0) {
    // The lane index goes through an empty asm statement, so that the
    // coordinates are rebuilt here instead of being held in registers from
    // the first pass (64 more live doubles at PPT = 16: they spilled).
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const long h = lane + long(i) * kConserveBlock;
      if (h < nh) fix(h, keep[i]);
    }
  } else {
    for (long h = threadIdx.x; h < nh; h += blockDim.x) fix(h, q[h]);
  }
}

// Midpoint-rule moments, FP64, one workgroup per item, two passes.
__global__ __launch_bounds__(256) void k_moments(const double *F, double *out, int N, double L) {
  const long n3 = long(N) * N * N;
  const long b = blockIdx.x;
  const double *f = F + b * n3;
  const double dc = 2.0 * L / N, dc3 = dc * dc * dc;
  __shared__ double red[10][256];
  double s[10];
  for (int k = 0; k < 4; ++k) s[k] = 0;
  for (long j = threadIdx.x; j < n3; j += blockDim.x) {
    const int i1 = int(j / (N * N)), i2 = int((j / N) % N), i3 = int(j % N);
    const double v = f[j];
    s[0] += v;
    s[1] += v * (-L + (i1 + 0.5) * dc);
    s[2] += v * (-L + (i2 + 0.5) * dc);
    s[3] += v * (-L + (i3 + 0.5) * dc);
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  const double n = red[0][0] * dc3;
  const double u1 = red[1][0] * dc3 / n, u2 = red[2][0] * dc3 / n, u3 = red[3][0] * dc3 / n;
  __syncthreads();
  for (int k = 0; k < 10; ++k) s[k] = 0;
  for (long j = threadIdx.x; j < n3; j += blockDim.x) {
    const int i1 = int(j / (N * N)), i2 = int((j / N) % N), i3 = int(j % N);
    const double v = f[j];
    const double d1 = -L + (i1 + 0.5) * dc - u1, d2 = -L + (i2 + 0.5) * dc - u2, d3 = -L + (i3 + 0.5) * dc - u3;
    const double d2s = d1 * d1 + d2 * d2 + d3 * d3;
    s[0] += v * d2s;
    s[1] += v * d1 * d1;
    s[2] += v * d1 * d2;
    s[3] += v * d1 * d3;
    s[4] += v * d2 * d2;
    s[5] += v * d2 * d3;
    s[6] += v * d3 * d3;
    s[7] += v * d1 * d2s;
    s[8] += v * d2 * d2s;
    s[9] += v * d3 * d2s;
  }
  for (int k = 0; k < 10; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 10; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = out + b * 14;
    o[0] = n;
    o[1] = u1;
    o[2] = u2;
    o[3] = u3;
    o[4] = 2.0 / (3.0 * n) * red[0][0] * dc3;
    for (int k = 0; k < 6; ++k) o[5 + k] = 2.0 * red[1 + k][0] * dc3;
    for (int k = 0; k < 3; ++k) o[11 + k] = red[7 + k][0] * dc3;
  }
}

// ----------------------------------------------------------------------------
bool use_fused_gain(const Plan &p) {
  return p.schedule != 1 && !p.literal && fused_gain_supported(p.N, p.precision);
}

Layout make_layout(const Plan &p, int64_t batch, int op, long chunk) {
  Layout l;
  const size_t es = (p.precision == QCOLL_FP32) ? sizeof(float) : sizeof(double);
  const long n3 = p.n3();
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t o = 0;
  if (op == 1) {
    // vjp: items per chunk and per gain sub-chunk (Y holds N_rho*M complex volumes per item).
    // The two-pass adjoint accumulation runs two workgroups (task halves) per
    // group of slabs of the sub-chunk's items, so the sub-chunk must hold enough
    // items to fill the GPU (32 items at N = 32 in FP64: 1024 workgroups); Y is
    // capped at 4 GiB.
    // The fused adjoint has no sub-chunks: its chunks hold up to 256 items
    // (fewer, larger launches of the small passes around it).
    const long cap = use_fused_adjoint(p) ? 256 : 32;
    l.bc = batch < cap ? (batch > 0 ? batch : 1) : cap;
    // (VSS kernels add the paired h_pq volumes, ceil(M/2) complex volumes per pair)
    const size_t per_item_y = size_t(p.N_rho) * p.M * n3 * 2 * es;
    const size_t per_item_yh = p.is_vss() ? size_t(p.N_rho) * ((p.M + 1) / 2) * n3 * 2 * es : 0;
    long pc = long((size_t(4) << 30) / (per_item_y + per_item_yh));
    l.pc = pc < 1 ? 1 : (pc > l.bc ? l.bc : pc);
    if (!use_fused_adjoint(p)) {
      // sub-chunks that fill the accumulation kernel's resident workgroups in
      // whole rounds, and chunks of whole sub-chunks (no small tail launch per
      // chunk); the chunking does not change any item's result
      const long round = adj_acc_items_per_round(p);
      if (round >= 1 && round < l.pc) l.pc = round * (l.pc / round);
      if (l.pc < l.bc) l.bc = l.pc * (l.bc / l.pc);
    }
    const size_t c64 = size_t(l.bc) * n3 * 2 * sizeof(double), cT = size_t(l.bc) * n3 * 2 * es;
    l.off_h64 = o; o += al(c64);
    l.off_g = o; o += al(c64);
    l.off_z = o; o += al(c64);
    l.off_h = o; o += al(cT);
    l.off_w = o; o += al(cT);
    l.off_b = o; o += al(size_t(l.bc) * p.npair() * n3 * 2 * es);
    l.off_hp = o; o += al(size_t(l.bc) * p.N_rho * n3 * es);
    // the fused adjoint keeps its per-term volumes on chip: Y holds only the
    // pairs' half spectra
    const size_t y_bytes = use_fused_adjoint(p) ? size_t(l.bc) * p.N_rho * (p.N / 2 + 1) * p.N * p.N * 2 * es
                                                : size_t(l.pc) * per_item_y;
    l.off_y = o; o += al(y_bytes);
    l.off_t = o; o += al(cT);
    l.off_l = o; o += al(c64);
    l.off_a = o; o += al(size_t(l.bc) * n3 * sizeof(double));
    l.off_d = o; o += al(size_t(l.bc) * p.N_rho * sizeof(double));
    l.off_pm = o; o += al(size_t(l.bc) * kProjSeg * 5 * sizeof(double));
    l.off_dp = o; o += al(size_t(l.bc) * kDomSeg * p.N_rho * sizeof(double));
    l.off_pd = o; o += use_fused_adjoint(p) ? 0 : al(size_t(l.bc) * p.N_rho * p.N * p.N * sizeof(double));
    l.off_yh = o; o += al(size_t(l.pc) * per_item_yh);
    l.total = o;
    return l;
  }
  const long cmax = chunk > 0 ? chunk : (p.chunk > 0 ? p.chunk : 64);
  l.bc = batch < cmax ? (batch > 0 ? batch : 1) : cmax;
  const bool bil = (op == 2);
  // two-pass hot loop: (item, node) pairs per launch such that the launch's
  // intermediate volume Y (M complex volumes per pair) stays near 192 MiB and
  // is mostly served from the 256 MiB Infinity Cache when the pencil pass
  // reads it back (FP64 at N = 32: 32 pairs)
  const bool lit = p.literal && !bil;
  {
    // (the literal convention writes two volumes per term)
    const size_t per_pair = size_t(p.M) * n3 * 2 * es * (lit ? 2 : 1);
    long pc = long((size_t(192) << 20) / per_pair);
    l.pc = pc < 8 ? 8 : (pc > 128 ? 128 : pc);
  }
  if (l.pc > l.bc * p.N_rho) l.pc = l.bc * p.N_rho;
  l.off_h = o; o += al(size_t(l.bc) * n3 * 2 * es);
  l.off_h64 = l.off_h;
  if (p.precision == QCOLL_FP32) { l.off_h64 = o; o += al(size_t(l.bc) * n3 * 2 * sizeof(double)); }
  const bool fused = use_fused_gain(p) && !bil;
  const bool vss = p.is_vss();
  // fused and VSS: W, the complex half spectra ((N/2 + 1) N^2 values) of every (item, node)
  const bool half = fused || vss;
  // literal: complex accumulators and one complex low-rank row per kept term
  const size_t per_node = half ? size_t(p.N / 2 + 1) * p.N * p.N * 2 : size_t(n3) * (lit ? 2 : 1);
  l.off_a = o; o += al(size_t(l.bc) * p.N_rho * per_node * es);
  l.off_b = o; o += (p.mix_identity || half) ? 0 : al(size_t(l.bc) * p.nv * n3 * es * (lit ? 2 : 1));
  l.off_w = o; o += half ? 0 : al(size_t(l.bc) * (lit ? p.nv : p.npair()) * n3 * 2 * sizeof(double));
  l.off_t = o; o += al(size_t(l.bc) * n3 * 2 * sizeof(double));   // gain spectrum, FP64
  l.off_l = o; o += al(size_t(l.bc) * n3 * 2 * sizeof(double));
  const bool q64 = use_gain_q64(p) && !bil;   // FP64 gain on chip: no per-term volumes
  l.off_y = o; o += (fused || q64) ? 0 : al(size_t(l.pc) * p.M * n3 * 2 * es);
  // two-pass VSS: the partial half spectra of the accumulation's parts 1.. of a launch
  l.off_vp = o;
  o += (vss && !fused) ? al(size_t(kVssParts - 1) * l.pc * (p.N / 2 + 1) * p.N * p.N * 2 * es) : 0;
  if (lit) {
    l.off_yg = o; o += al(size_t(l.pc) * p.M * n3 * 2 * es);   // the Im(beta) volumes
  }
  if (bil) {
    l.off_hg = o; o += al(size_t(l.bc) * n3 * 2 * es);
    l.off_h64g = o; o += al(size_t(l.bc) * n3 * 2 * sizeof(double));
    l.off_yg = o; o += al(size_t(l.pc) * p.M * n3 * 2 * es);
  }
  l.total = o;
  return l;
}

template <typename T>
static qcoll_status eval_dispatch(const Plan &p, int64_t batch, const double *f, const double *g, double *Q, void *ws,
                                  const Layout &lay, hipStream_t st, const double *isc, int K) {
  switch (p.N) {
    case 8: return Engine<T, 8>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 12: return Engine<T, 12>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 16: return Engine<T, 16>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 24: return Engine<T, 24>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 32: return Engine<T, 32>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 48: return Engine<T, 48>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    case 64: return Engine<T, 64>::eval(p, batch, f, g, Q, ws, lay, st, isc, K);
    default: set_error("unsupported N"); return QCOLL_ENOTSUP;
  }
}

qcoll_status launch_eval(const Plan &p, int64_t batch, const double *f, double *Q, void *ws,
                         const Layout &lay, hipStream_t st, const double *isc, int K) {
  if (p.precision == QCOLL_FP32) return eval_dispatch<float>(p, batch, f, nullptr, Q, ws, lay, st, isc, K);
  return eval_dispatch<double>(p, batch, f, nullptr, Q, ws, lay, st, isc, K);
}

qcoll_status launch_eval2(const Plan &p, int64_t batch, const double *f, const double *g, double *Q, void *ws,
                          const Layout &lay, hipStream_t st) {
  if (p.precision == QCOLL_FP32) return eval_dispatch<float>(p, batch, f, g, Q, ws, lay, st, nullptr, 0);
  return eval_dispatch<double>(p, batch, f, g, Q, ws, lay, st, nullptr, 0);
}

qcoll_status launch_conserve(const Plan &p, int64_t batch, double *Q, double *mom, hipStream_t st, const double *isc,
                             int K) {
  const double dc = 2.0 * p.L / p.N;
  TimedLaunch tl("conserve", st);
  // pairs per lane of the register-resident variant: N^3 / 2 / 1024, rounded up
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(unsigned(batch)), dim3(kConserveBlock), 0, st, Q, mom, p.ginv, p.N, p.L, p.flag,
                       dc * dc * dc, isc, K);
  };
  switch (p.N) {
    case 8: go(k_conserve<1, 8>); break;
    case 12: go(k_conserve<1, 12>); break;
    case 16: go(k_conserve<2, 16>); break;
    case 24: go(k_conserve<7, 24>); break;
    case 32: go(k_conserve<16, 32>); break;
    case 48: go(k_conserve<0, 48>); break;
    case 64: go(k_conserve<0, 64>); break;
    default: go(k_conserve<0>); break;
  }
  QC_LAUNCH_CHECK("conserve");
  return QCOLL_OK;
}

qcoll_status launch_moments(const Plan &p, int64_t batch, const double *f, double *out, hipStream_t st) {
  TimedLaunch tl("moments", st);
  hipLaunchKernelGGL(k_moments, dim3(unsigned(batch)), dim3(256), 0, st, f, out, p.N, p.L);
  QC_LAUNCH_CHECK("moments");
  return QCOLL_OK;
}

}  // namespace qcoll
