// Vector-Jacobian product of Q(f,f) with respect to f and omega.
//
// With u_pq = ifft3[c_s fft3 f] (the same transform as the forward hot loop),
// h_p = C_p g (multiplier alpha_p, or its truncation) and the loss multiplier
// Lam:
//   J^T g = 2 Re ifft3[ sum_pq w_q c_s fft3( h_p conj(u_pq) ) ]
//           - g * ifft3[Lam fft3 f] - ifft3[Lam fft3(f g)],
// which follows from the forward form Q = sum_p C_p sum_q w_q t1 t2 - f Lam~ f
// with t1 + i t2 = (1 + i) u, the adjoint of a shift being the opposite shift
// and C_p, Lam~ self-adjoint.  omega enters through b(omega) rho_p^{4-2 omega}:
//   g . dQ/d omega = sum_p dlog_p ( <h_p, A_p> - <f g, Lam~_p f> ),
// A_p = sum_q w_q t1 t2, and the loss part is a Fourier-space dot product.
//
// The gain adjoint runs on chip per (item, p) pair for FP32 plans with N <= 32
// (k_adj_fused, qcoll_adj_fused.hip).  Otherwise (FP64, N = 48, or the two-pass
// schedule requested) it takes three passes per (item, p, q): the forward slab
// pass of the hot loop, a pencil pass that inverts along axis 1, forms
// w_q h_p conj(u), accumulates <h_p, A_p> and transforms back along axis 1, and
// a slab pass that transforms the two inner axes forward and accumulates
// c_s * (.) for every (p, q) of the item.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "qcoll_passes.hpp"

namespace qcoll {

// f * g as a complex FP64 volume, slab g = item*N + j1
template <int N>
struct SrcProd {
  const double *f, *g;
  __device__ C<double> operator()(long s, int r, int c) const {
    const long o = (s * N + r) * N + c;
    return C<double>{f[o] * g[o], 0.0};
  }
};

// (V_2s + i V_2s+1) * G^ for pair s of item b, slab = (b*npair + s)*N + k1
template <typename T, int N>
struct SrcVPair {
  const C<T> *G;
  const T *V;
  int npair;
  __device__ C<T> operator()(long g, int r, int c) const {
    constexpr long n3 = long(N) * N * N;
    const long t = g / N;
    const int k1 = int(g % N);
    const long b = t / npair;
    const int s = int(t % npair);
    const long o = (long(k1) * N + r) * N + c;
    const C<T> x = G[b * n3 + o];
    const T a = V[(2 * s) * n3 + o], d = V[(2 * s + 1) * n3 + o];
    return C<T>{x.re * a - x.im * d, x.re * d + x.im * a};
  }
};

// h_p = sum_s U[s][p] R_s, R_s = Re/Im of the packed pair buffer
template <typename T, int NRM>
__global__ __launch_bounds__(256) void k_unpack_mix(const C<T> *R, const T *U, T *Hp, long nitems, int S, int Nr,
                                                    int npair, long n3) {
  // the S (<= Nr <= NRM) packed values of the point are loaded once into
  // registers; U (S x Nr) is staged per block in LDS, transposed and
  // zero-padded to NRM rows, and read at one address per wave (broadcast)
  __shared__ T ut[NRM * NRM];
  for (int t = threadIdx.x; t < Nr * NRM; t += blockDim.x) {
    const int q = t / NRM, s = t % NRM;
    ut[t] = (s < S) ? U[s * Nr + q] : T(0);
  }
  __syncthreads();
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nitems * n3) return;
  const long b = i / n3, j = i % n3;
  const C<T> *r0 = R + b * npair * n3 + j;
  T rv[NRM];
#pragma unroll
  for (int k = 0; k < NRM / 2; ++k) {
    C<T> x{T(0), T(0)};
    if (2 * k < S) x = r0[k * n3];
    rv[2 * k] = x.re;
    rv[2 * k + 1] = x.im;
  }
  T *h0 = Hp + b * Nr * n3 + j;
  for (int q = 0; q < Nr; ++q) {
    T acc = T(0);
#pragma unroll
    for (int s = 0; s < NRM; ++s) acc += ut[q * NRM + s] * rv[s];
    h0[q * n3] = acc;
  }
}

template <typename T>
static void launch_unpack_mix(const C<T> *R, const T *U, T *Hp, long nitems, int S, int Nr, int npair, long n3,
                              hipStream_t st) {
  const dim3 g(nblk(nitems * n3, 256)), blk(256);
  switch (mix_width(Nr)) {
    case 8: hipLaunchKernelGGL((k_unpack_mix<T, 8>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
    case 16: hipLaunchKernelGGL((k_unpack_mix<T, 16>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
    case 24: hipLaunchKernelGGL((k_unpack_mix<T, 24>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
    case 32: hipLaunchKernelGGL((k_unpack_mix<T, 32>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
    case 48: hipLaunchKernelGGL((k_unpack_mix<T, 48>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
    default: hipLaunchKernelGGL((k_unpack_mix<T, 64>), g, blk, 0, st, R, U, Hp, nitems, S, Nr, npair, n3); break;
  }
}

// adjoint pencil pass: per (item, p) pair and pencil (j2, j3), for every q:
// u = inverse along axis 1; y = w_q h_p conj(u); the pencil's part of
// <h_p, sum_q w_q t1 t2> is stored per pencil (summed per pair in a fixed order
// by k_pair_dot_sum); y transformed forward along axis 1 and stored back in place.
template <typename T, int N>
struct OpAdjPencil {
  C<T> *Y;
  const T *Hp;
  const T *wq;
  double *dots;    // [pairs][N^2] per-pencil parts of <h_p, A_p>, or null
  long bp0;        // first (item, p) pair of this launch (within the chunk)
  int M;
  __device__ void operator()(long bpl, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    const T *h = Hp + (bp0 + bpl) * n3 + r;
    T hv[N];
    static_for<0, N>([&](auto j) { hv[decltype(j)::value] = h[decltype(j)::value * n2]; });
    double dot = 0.0;
    for (int q = 0; q < M; ++q) {
      C<T> *y = Y + (bpl * M + q) * n3 + r;
      T xr[N], xi[N];
      static_for<0, N>([&](auto k) {
        const C<T> v = y[decltype(k)::value * n2];
        xr[decltype(k)::value] = v.re;
        xi[decltype(k)::value] = v.im;
      });
      fft_reg<N, +1, T>(xr, xi);
      const T w = wq[q];
      T part = T(0);
      static_for<0, N>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        part += hv[jj] * (xr[jj] * xr[jj] - xi[jj] * xi[jj]);
        const T s = w * hv[jj];
        xr[jj] = s * xr[jj];
        xi[jj] = -s * xi[jj];
      });
      dot += double(w) * double(part);
      fft_reg<N, -1, T>(xr, xi);
      static_for<0, N>([&](auto k) { y[decltype(k)::value * n2] = C<T>{xr[decltype(k)::value], xi[decltype(k)::value]}; });
    }
    if (dots) dots[(bp0 + bpl) * n2 + r] = dot;
  }
};

// VSS kernels: h_pq = C_pq g differs per sphere point.  Slab pass of the
// cotangent's weighted spectra, two sphere points per complex volume:
// alpha_pq0 G + i alpha_pq1 G (slab g = ((pair * MH + qq) * N + k1), MH = ceil(M/2),
// q0 = 2 qq, q1 = 2 qq + 1 or none), transformed along axes 2 and 3; the adjoint
// pencil pass inverts it along axis 1 to h_pq0 + i h_pq1 (both real: alpha_pq
// is even and G Hermitian).  alpha_pq holds the planes k1 <= N/2 (already / N^3);
// a plane k1 > N/2 reads the reflected index.
template <typename T, int N>
struct SrcVssG {
  const C<T> *G;
  const T *apq;
  long bp0;
  int M, Nr;
  __device__ C<T> operator()(long g, int r, int c) const {
    constexpr long n2 = long(N) * N, nh = long(N / 2 + 1) * n2;
    const int MH = (M + 1) / 2;
    const long t = g / N;
    const int k1 = int(g % N);
    const long bp = bp0 + t / MH;
    const int qq = int(t % MH);
    const long b = bp / Nr;
    const int p = int(bp % Nr);
    const long o = k1 <= N / 2 ? (long(k1) * N + r) * N + c
                               : (long(N - k1) * N + (N - r) % N) * N + (N - c) % N;
    const int q0 = 2 * qq, q1 = 2 * qq + 1;
    const T a0 = apq[(size_t(p) * M + q0) * nh + o];
    const T a1 = q1 < M ? apq[(size_t(p) * M + q1) * nh + o] : T(0);
    const C<T> x = G[b * n2 * N + (long(k1) * N + r) * N + c];
    return C<T>{a0 * x.re - a1 * x.im, a0 * x.im + a1 * x.re};
  }
};

// adjoint pencil pass for VSS kernels: as OpAdjPencil with h_pq (from the
// paired volumes Yh) in place of w_q h_p (alpha_pq carries w_p w_q).  Where the
// pencil's four rows (h_pq0, h_pq1 and the term's u) would not fit in the
// registers (FP64 at N >= 32) the pair's h volume is transformed once per
// sphere point instead of once per pair.
template <typename T, int N>
struct OpAdjPencilVss {
  C<T> *Y;
  const C<T> *Yh;
  double *dots;    // [pairs][N^2] per-pencil parts of sum_q <h_pq, t1 t2>, or null
  long bp0;
  int M;
  static constexpr bool kBothH = sizeof(T) * N < 256;
  // y = h conj(u) along the pencil, and the pencil's part of <h, Re u^2 - Im u^2>
  __device__ static T term(C<T> *y, const T (&hv)[N]) {
    constexpr long n2 = long(N) * N;
    T xr[N], xi[N];
    static_for<0, N>([&](auto k) {
      const C<T> v = y[decltype(k)::value * n2];
      xr[decltype(k)::value] = v.re;
      xi[decltype(k)::value] = v.im;
    });
    fft_reg<N, +1, T>(xr, xi);
    T part = T(0);
    static_for<0, N>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      part += hv[jj] * (xr[jj] * xr[jj] - xi[jj] * xi[jj]);
      xr[jj] = hv[jj] * xr[jj];
      xi[jj] = -hv[jj] * xi[jj];
    });
    fft_reg<N, -1, T>(xr, xi);
    static_for<0, N>([&](auto k) { y[decltype(k)::value * n2] = C<T>{xr[decltype(k)::value], xi[decltype(k)::value]}; });
    return part;
  }
  __device__ void operator()(long bpl, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    const int MH = (M + 1) / 2;
    double dot = 0.0;
    for (int qq = 0; qq < MH; ++qq) {
      const C<T> *yh = Yh + (bpl * MH + qq) * n3 + r;
      if constexpr (kBothH) {
        T hr[N], hi[N];
        static_for<0, N>([&](auto k) {
          const C<T> v = yh[decltype(k)::value * n2];
          hr[decltype(k)::value] = v.re;
          hi[decltype(k)::value] = v.im;
        });
        fft_reg<N, +1, T>(hr, hi);
        dot += double(term(Y + (bpl * M + 2 * qq) * n3 + r, hr));
        if (2 * qq + 1 < M) dot += double(term(Y + (bpl * M + 2 * qq + 1) * n3 + r, hi));
      } else {
        for (int e = 0; e < 2 && 2 * qq + e < M; ++e) {
          T hr[N], hi[N];
          static_for<0, N>([&](auto k) {
            const C<T> v = yh[decltype(k)::value * n2];
            hr[decltype(k)::value] = v.re;
            hi[decltype(k)::value] = v.im;
          });
          fft_reg<N, +1, T>(hr, hi);
          T hv[N];
          static_for<0, N>([&](auto k) { hv[decltype(k)::value] = e ? hi[decltype(k)::value] : hr[decltype(k)::value]; });
          dot += double(term(Y + (bpl * M + 2 * qq + e) * n3 + r, hv));
        }
      }
    }
    if (dots) dots[(bp0 + bpl) * n2 + r] = dot;
  }
};

// dwg[pair] = sum of the pair's n per-pencil parts, in a fixed order (strided
// per-thread sums, wave butterflies, then the four waves in order)
__global__ __launch_bounds__(256) void k_pair_dot_sum(const double *dots, double *dwg, long n) {
  const long bp = blockIdx.x;
  double v = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) v += dots[bp * n + i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __shared__ double red[4];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) dwg[bp] = ((red[0] + red[1]) + red[2]) + red[3];
}

// adjoint accumulation: Z[b] slab k1 = sum_{p,q} c_s(k) * fft2d(Y_(b,p,q) slab k1)
// over the items [ib0, ib0 + ni) of the sub-chunk.  The N_rho*M tasks (p, q)
// of a slab are split in two fixed halves (blockIdx.y): the first half's sum
// goes to Z, the second half's to Zp (sub-chunk relative), and k_adj_acc_add
// forms Z = first + second, so twice as many workgroups hide the loads' latency
// while every item's result is the same whatever the chunking.  One workgroup
// owns SPB slabs of Z (possibly of two items).  Lane (s, c) owns column c of
// slab s, as in the generic slab kernel: the column transform runs in registers
// straight from the coalesced loads, the row transform through LDS, and the
// accumulators hold the lane's column.
// waves per SIMD the register budget must allow: at 48^3 in FP32 a one-wave
// workgroup needs 18.8 KiB of LDS, so eight fit a CU once the registers do
template <typename T, int N>
constexpr int adj_acc_wpe() {
  return (std::is_same<T, float>::value && N == 48) ? 2 : 1;
}

template <typename T, int N>
__global__ __launch_bounds__(256, (adj_acc_wpe<T, N>())) void k_adj_acc(const C<T> *Y, const C<T> *phase, C<T> *Z,
                                                                      C<T> *Zp, long ib0, long ni, int M, int Nr) {
  constexpr int SPB = slab_spb2<T, N>();
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  __shared__ T sre[SPB][N][N + 1];
  __shared__ T sim[SPB][N][N + 1];
  const int s = int(threadIdx.x) / N, c = int(threadIdx.x) % N;
  const long nz = ni * N;
  const long z = long(blockIdx.x) * SPB + s;   // Z slab (relative to ib0)
  const long zl = z < nz ? z : nz - 1;
  const long bl = zl / N;
  const int k1 = int(zl % N);
  T ar[N], ai[N];
  static_for<0, N>([&](auto k) { ar[decltype(k)::value] = T(0); ai[decltype(k)::value] = T(0); });
  const int ntask = Nr * M;
  const int half = int(blockIdx.y);
  const int t0 = (half * ntask) / 2, t1 = ((half + 1) * ntask) / 2;
  for (int task = t0; task < t1; ++task) {
    const int p = task / M, q = task % M;
    const C<T> *y = Y + ((bl * Nr + p) * M + q) * n3 + long(k1) * n2 + c;
    T xr[N], xi[N];
    static_for<0, N>([&](auto r) {
      const C<T> v = y[decltype(r)::value * N];
      xr[decltype(r)::value] = v.re;
      xi[decltype(r)::value] = v.im;
    });
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
    const C<T> *ph = phase + size_t(p * M + q) * 3 * N;
    const C<T> b1 = ph[k1], b3 = ph[2 * N + c];
    const T x13 = b1.re * b3.re - b1.im * b3.im, y13 = b1.re * b3.im + b1.im * b3.re;
    // c_s = Re(b13 b2) + Im(b13 b2) = b2.re P + b2.im Q
    const T P = x13 + y13, Q = x13 - y13;
    static_for<0, N>([&](auto r) {
      constexpr int rr = decltype(r)::value;
      const C<T> b2 = ph[N + rr];
      const T cm = b2.re * P + b2.im * Q;
      ar[rr] += cm * sre[s][rr][c];
      ai[rr] += cm * sim[s][rr][c];
    });
    __syncthreads();
  }
  if (z < nz) {
    C<T> *zo = (half == 0 ? Z + (ib0 + bl) * n3 : Zp + bl * n3) + long(k1) * n2 + c;
    static_for<0, N>([&](auto r) { zo[decltype(r)::value * N] = C<T>{ar[decltype(r)::value], ai[decltype(r)::value]}; });
  }
}

// Z[ib0 + i] += Zp[i] for the ni items of a sub-chunk (n complex values each)
template <typename T>
__global__ __launch_bounds__(256) void k_adj_acc_add(C<T> *Z, const C<T> *Zp, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const C<T> a = Z[i], b = Zp[i];
  Z[i] = C<T>{a.re + b.re, a.im + b.im};
}

// loss adjoint spectrum, FP64: Lam (H + i FG), slab = item*N + k1
template <int N>
struct SrcLossAdj {
  const C<double> *H, *FG;
  const double *lam;
  __device__ C<double> operator()(long g, int r, int c) const {
    const long o = (g * N + r) * N + c;
    const double l = lam[((g % N) * N + r) * N + c];
    const C<double> h = H[o], x = FG[o];
    return C<double>{(h.re - x.im) * l, (h.im + x.re) * l};
  }
};

// final pencil pass: df = 2 Re ifft(Z)/N^3 - g Re(L) - Im(L)
// Loss part of the adjoint's last pencil: df = gain - g Re(L) - Im(L), with
// gain the pencil's transformed gain part and L = ifft of the loss adjoint
// spectrum along axis 1.  The loads of g for each group of points are issued
// before the group's stores (df may alias g as far as the compiler knows, so a
// load after a store would wait for it).
template <int N>
__device__ __forceinline__ void vjp_assemble_loss(const double (&out)[N], const C<double> *x, const double *gb,
                                                  double *o) {
  constexpr long n2 = long(N) * N;
  double lr[N], li[N];
  static_for<0, N>([&](auto k) {
    const C<double> v = x[decltype(k)::value * n2];
    lr[decltype(k)::value] = v.re;
    li[decltype(k)::value] = v.im;
  });
  fft_reg<N, +1, double>(lr, li);
  constexpr int G = (N % 8 == 0) ? 8 : 4;
  static_for<0, N / G>([&](auto gg) {
    constexpr int j0 = decltype(gg)::value * G;
    double gv[G];
    static_for<0, G>([&](auto i) { gv[decltype(i)::value] = gb[(j0 + decltype(i)::value) * n2]; });
    static_for<0, G>([&](auto i) {
      constexpr int jj = j0 + decltype(i)::value;
      double v = out[jj];
      v -= gv[decltype(i)::value] * lr[jj] + li[jj];
      o[jj * n2] = v;
    });
  });
}

template <typename T, int N>
struct OpVjpAssemble {
  const C<T> *Z;
  const C<double> *Lm;
  const double *g;
  double *df;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    double out[N];
    {
      T zr[N], zi[N];
      const C<T> *x = Z + b * n3 + r;
      static_for<0, N>([&](auto k) {
        const C<T> v = x[decltype(k)::value * n2];
        zr[decltype(k)::value] = v.re;
        zi[decltype(k)::value] = v.im;
      });
      fft_reg<N, +1, T>(zr, zi);
      constexpr double sc = 2.0 / double(n3);
      static_for<0, N>([&](auto j) { out[decltype(j)::value] = sc * double(zr[decltype(j)::value]); });
    }
    vjp_assemble_loss<N>(out, Lm + b * n3 + r, g + b * n3 + r, df + b * n3 + r);
  }
};

// final pencil pass of the fused adjoint: the gain part arrives as the planes
// k1 <= N/2 of the Hermitian spectrum Zh (already transformed along axes 2 and
// 3; the planes k1 > N/2 are the conjugates of planes N - k1 at the same
// (j2, j3)), with 2 Re ifft3[Z] = ifft3[Zh]:
// df = ifft(Zh)/N^3 - g Re(L) - Im(L)
template <typename T, int N>
struct OpVjpAssembleHalf {
  const C<T> *Z;
  const C<double> *Lm;
  const double *g;
  double *df;
  __device__ void operator()(long b, int r) const {
    constexpr long n2 = long(N) * N, n3 = n2 * N;
    constexpr int H1 = N / 2 + 1;
    double out[N];
    {
      T zr[N], zi[N];
      const C<T> *x = Z + b * n3 + r;
      static_for<0, H1>([&](auto k) {
        const C<T> v = x[decltype(k)::value * n2];
        zr[decltype(k)::value] = v.re;
        zi[decltype(k)::value] = v.im;
      });
      static_for<H1, N>([&](auto k) {
        zr[decltype(k)::value] = zr[N - decltype(k)::value];
        zi[decltype(k)::value] = -zi[N - decltype(k)::value];
      });
      fft_reg<N, +1, T>(zr, zi);
      constexpr double sc = 1.0 / double(n3);
      static_for<0, N>([&](auto j) { out[decltype(j)::value] = sc * double(zr[decltype(j)::value]); });
    }
    vjp_assemble_loss<N>(out, Lm + b * n3 + r, g + b * n3 + r, df + b * n3 + r);
  }
};

// loss part of the omega gradient and the final combination:
// domega[b] = sum_p dlog_p ( dwg[b][p] - (1/N^3) sum_k Re(conj(FG) H) Lam_p(k) ).
// The spectrum of an item is split into kDomSeg segments; a block takes one
// segment of IB items, reads each Lam_p(k) of the segment once for all of them,
// forms x(k) = Re(conj(FG) H)(k) once per item and point, and accumulates
// x Lam_p for every node p in registers; then it reduces each sum over the
// block (wave butterflies, then the four waves in order).  Rows p >= N_rho of
// the padded width NRM read row N_rho - 1 (no branch in the load stream) and are
// dropped.  An item's sums do not depend on the other items of its block.
template <int NRM>
constexpr int domega_items() {
  return NRM <= 16 ? 2 : 1;
}

template <int NRM, int IB = domega_items<NRM>()>
__global__ __launch_bounds__(256) void k_domega_part(const C<double> *H, const C<double> *FG, const double *lam_p,
                                                     double *part, long nb, int Nr, long n3) {
  const long b0 = (blockIdx.x / kDomSeg) * IB;
  const int g = blockIdx.x % kDomSeg;
  const long seg = (n3 + kDomSeg - 1) / kDomSeg;
  const long k0 = g * seg, k1 = (k0 + seg < n3) ? k0 + seg : n3;
  const int ni = (nb - b0 < IB) ? int(nb - b0) : IB;
  double acc[IB][NRM];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int q = 0; q < NRM; ++q) acc[i][q] = 0.0;
  for (long k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    double lam[NRM];
#pragma unroll
    for (int q = 0; q < NRM; ++q) lam[q] = lam_p[(q < Nr ? q : Nr - 1) * n3 + k];
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      // items past the batch repeat the last one (valid) and are not written
      const long b = b0 + (i < ni ? i : ni - 1);
      const C<double> h = H[b * n3 + k], x = FG[b * n3 + k];
      const double v = x.re * h.re + x.im * h.im;
#pragma unroll
      for (int q = 0; q < NRM; ++q) acc[i][q] += v * lam[q];
    }
  }
  __shared__ double red[4][IB][NRM];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int q = 0; q < NRM; ++q) {
      double v = acc[i][q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) red[wave][i][q] = v;
    }
  __syncthreads();
  for (int t = threadIdx.x; t < ni * Nr; t += blockDim.x) {
    const int i = t / Nr, q = t % Nr;
    part[((b0 + i) * kDomSeg + g) * long(Nr) + q] = ((red[0][i][q] + red[1][i][q]) + red[2][i][q]) + red[3][i][q];
  }
}

__global__ __launch_bounds__(64) void k_domega_final(const double *part, const double *dlog, const double *dwg,
                                                     double *domega, int Nr, long n3) {
  const long b = blockIdx.x;
  __shared__ double t[64];
  const int q = threadIdx.x;
  if (q < Nr) {
    double s = 0.0;
    for (int g = 0; g < kDomSeg; ++g) s += part[(b * kDomSeg + g) * Nr + q];
    t[q] = dlog[q] * (dwg[b * Nr + q] - s / double(n3));
  }
  __syncthreads();
  if (q == 0) {
    double tot = 0.0;
    for (int r = 0; r < Nr; ++r) tot += t[r];
    domega[b] = tot;
  }
}

static void launch_domega(const C<double> *H, const C<double> *FG, const double *lam_p, const double *dlog,
                          const double *dwg, double *part, double *domega, long nb, int Nr, long n3,
                          hipStream_t st) {
  const dim3 blk(256);
  auto grid = [&](int ib) { return dim3(unsigned((nb + ib - 1) / ib * kDomSeg)); };
  switch (mix_width(Nr)) {
    case 8:
      hipLaunchKernelGGL((k_domega_part<8>), grid(domega_items<8>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
    case 16:
      hipLaunchKernelGGL((k_domega_part<16>), grid(domega_items<16>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
    case 24:
      hipLaunchKernelGGL((k_domega_part<24>), grid(domega_items<24>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
    case 32:
      hipLaunchKernelGGL((k_domega_part<32>), grid(domega_items<32>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
    case 48:
      hipLaunchKernelGGL((k_domega_part<48>), grid(domega_items<48>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
    default:
      hipLaunchKernelGGL((k_domega_part<64>), grid(domega_items<64>()), blk, 0, st, H, FG, lam_p, part, nb, Nr, n3);
      break;
  }
  hipLaunchKernelGGL(k_domega_final, dim3(unsigned(nb)), dim3(64), 0, st, part, dlog, dwg, domega, Nr, n3);
}

// Conservation projection of the cotangent, g -> g - sum_a lam_a phi_a with
// lam = G^-1 <phi, g> (phi = 1, c, |c|^2 on the grid).  An item is split into
// kProjSeg segments of one block each, so that a chunk of a few tens of items
// still fills the GPU: the first kernel writes the segment's five moment sums,
// the second adds the segments' sums in a fixed order and applies the update.

__device__ __forceinline__ void grid_coord(int j, int N, double L, double &c1, double &c2, double &c3) {
  const double dc = 2.0 * L / N;
  const int i1 = j / (N * N), i2 = (j / N) % N, i3 = j % N;
  c1 = -L + (i1 + 0.5) * dc;
  c2 = -L + (i2 + 0.5) * dc;
  c3 = -L + (i3 + 0.5) * dc;
}

__global__ __launch_bounds__(256) void k_project_moments(const double *in, double *part, int N, double L) {
  const int n3 = N * N * N, seg = (n3 + kProjSeg - 1) / kProjSeg;
  const long b = blockIdx.x / kProjSeg;
  const int g = blockIdx.x % kProjSeg;
  const int j0 = g * seg, j1 = (j0 + seg < n3) ? j0 + seg : n3;
  const double *x = in + b * n3;
  double s[5] = {0, 0, 0, 0, 0};
  for (int j = j0 + int(threadIdx.x); j < j1; j += blockDim.x) {
    double c1, c2, c3;
    grid_coord(j, N, L, c1, c2, c3);
    const double v = x[j];
    s[0] += v;
    s[1] += v * c1;
    s[2] += v * c2;
    s[3] += v * c3;
    s[4] += v * (c1 * c1 + c2 * c2 + c3 * c3);
  }
  __shared__ double red[5][256];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_project_apply(const double *in, double *out, const double *part,
                                                       const double *ginv, int N, double L) {
  const int n3 = N * N * N, seg = (n3 + kProjSeg - 1) / kProjSeg;
  const long b = blockIdx.x / kProjSeg;
  const int g = blockIdx.x % kProjSeg;
  const int j0 = g * seg, j1 = (j0 + seg < n3) ? j0 + seg : n3;
  __shared__ double mom[5];
  if (threadIdx.x < 5) {
    double m = 0;
    for (int h = 0; h < kProjSeg; ++h) m += part[(b * kProjSeg + h) * 5 + threadIdx.x];
    mom[threadIdx.x] = m;
  }
  __syncthreads();
  double lam[5];
  for (int a = 0; a < 5; ++a) {
    double acc = 0;
    for (int c = 0; c < 5; ++c) acc += ginv[a * 5 + c] * mom[c];
    lam[a] = acc;
  }
  const double *x = in + b * n3;
  double *y = out + b * n3;
  for (int j = j0 + int(threadIdx.x); j < j1; j += blockDim.x) {
    double c1, c2, c3;
    grid_coord(j, N, L, c1, c2, c3);
    y[j] = x[j] - (lam[0] + lam[1] * c1 + lam[2] * c2 + lam[3] * c3 + lam[4] * (c1 * c1 + c2 * c2 + c3 * c3));
  }
}

template <typename T, int N>
struct Vjp {
  using P = Passes<T, N>;
  using P64 = Passes<double, N>;
  static constexpr long n3 = P::n3;
  static constexpr int SPB = slab_spb2<T, N>();

  static qcoll_status run(const Plan &p, int64_t batch, const double *f, const double *g_in, double *df,
                          double *domega, bool through, void *ws, const Layout &lay, hipStream_t st) {
    char *w = static_cast<char *>(ws);
    C<double> *H64 = reinterpret_cast<C<double> *>(w + lay.off_h64);
    C<double> *G64 = reinterpret_cast<C<double> *>(w + lay.off_g);
    C<double> *FG64 = reinterpret_cast<C<double> *>(w + lay.off_z);
    C<T> *H = reinterpret_cast<C<T> *>(w + lay.off_h);
    C<T> *GT = reinterpret_cast<C<T> *>(w + lay.off_w);          // spectrum of g in T
    C<T> *R = reinterpret_cast<C<T> *>(w + lay.off_b);           // packed pair inverses
    T *Hp = reinterpret_cast<T *>(w + lay.off_hp);
    C<T> *Y = reinterpret_cast<C<T> *>(w + lay.off_y);
    C<T> *Z = reinterpret_cast<C<T> *>(w + lay.off_t);
    C<double> *Lm = reinterpret_cast<C<double> *>(w + lay.off_l);
    double *gproj = reinterpret_cast<double *>(w + lay.off_a);
    double *dwg = reinterpret_cast<double *>(w + lay.off_d);
    double *pm = reinterpret_cast<double *>(w + lay.off_pm);
    double *dpart = reinterpret_cast<double *>(w + lay.off_dp);
    double *pdots = reinterpret_cast<double *>(w + lay.off_pd);
    C<T> *Yh = reinterpret_cast<C<T> *>(w + lay.off_yh);     // VSS: paired h_pq volumes of a sub-chunk
    const bool vss = p.is_vss();
    const int S = p.nv, np = p.npair(), Nr = p.N_rho, M = p.M;
    const bool fused_adjoint = std::is_same<T, float>::value && use_fused_adjoint(p);
    qcoll_status s;
    for (long b0 = 0; b0 < batch; b0 += lay.bc) {
      const long nb = (batch - b0 < lay.bc) ? (batch - b0) : lay.bc;
      const double *fb = f + b0 * n3;
      const double *gb = g_in + b0 * n3;
      if (through) {
        TimedLaunch tl("vjp project", st);
        hipLaunchKernelGGL(k_project_moments, dim3(unsigned(nb * kProjSeg)), dim3(256), 0, st, gb, pm, N, p.L);
        hipLaunchKernelGGL(k_project_apply, dim3(unsigned(nb * kProjSeg)), dim3(256), 0, st, gb, gproj, pm, p.ginv,
                           N, p.L);
        QC_LAUNCH_CHECK("vjp project");
        gb = gproj;
      }
      // FP64 spectra of f, g and f g
      if ((s = P64::template forward_to<T>(fb, H64, H, nb, st))) return s;
      if ((s = P64::template forward_to<T>(gb, G64, GT, nb, st))) return s;
      if ((s = P64::template slab<SrcProd<N>, DstCplx<double, N>, -1>(SrcProd<N>{fb, gb}, DstCplx<double, N>{FG64},
                                                                    nb * N, st, "vjp fg slab")))
        return s;
      if ((s = P64::pencil(OpPencilInPlace<double, N, -1>{FG64}, nb * N * N, st, "vjp fg pencil"))) return s;
      // h_p = C_p g: packed inverse transforms of (V_2s + i V_2s+1) G^, then unpack + mix
      // (the fused adjoint forms h_p on chip; VSS kernels form h_pq per sphere
      // point in the gain loop below)
      if (!vss && !fused_adjoint) {
        if ((s = P::template slab<SrcVPair<T, N>, DstCplx<T, N>, +1>(
                 SrcVPair<T, N>{GT, reinterpret_cast<const T *>(p.V), np}, DstCplx<T, N>{R}, nb * np * N, st,
                 "vjp h slab")))
          return s;
        if ((s = P::pencil(OpPencilInPlace<T, N, +1>{R}, nb * np * N * N, st, "vjp h pencil"))) return s;
        TimedLaunch tl("vjp unpack", st);
        launch_unpack_mix<T>(R, reinterpret_cast<const T *>(p.umix_d), Hp, nb, S, Nr, np, n3, st);
        QC_LAUNCH_CHECK("vjp unpack");
      }
      if (fused_adjoint) {
        // gain adjoint on chip, one workgroup per (item, p) pair, then the sum
        // over p of the pairs' half spectra and the inverse along axes 2, 3
        constexpr int H1 = N / 2 + 1;
        constexpr long nh = long(H1) * N * N;
        if ((s = launch_adjoint_fused(p, H, GT, reinterpret_cast<float *>(Hp), Y, domega ? dwg : nullptr,
                                      nb * Nr, st)))
          return s;
        {
          TimedLaunch tl("vjp sum nodes", st);
          launch_sum_nodes(Y, Z, nb, Nr, nh / 2, n3 / 2, st);
          QC_LAUNCH_CHECK("vjp sum nodes");
        }
        if ((s = P::template slab<SrcCplxHalf<T, N>, DstCplxHalf<T, N>, +1>(
                 SrcCplxHalf<T, N>{Z}, DstCplxHalf<T, N>{Z}, nb * H1, st, "vjp inverse slab")))
          return s;
      } else {
        // gain adjoint, items in sub-chunks of lay.pc items
        const T scale = T(1.0 / double(n3));
        for (long ib0 = 0; ib0 < nb; ib0 += lay.pc) {
          const long ni = (nb - ib0 < lay.pc) ? (nb - ib0) : lay.pc;
          const long bp0 = ib0 * Nr;
          const long cnt = ni * Nr;
          SrcShift<T, N> src{H, reinterpret_cast<const C<T> *>(p.phase), bp0, M, Nr, scale};
          if ((s = P::template slab<SrcShift<T, N>, DstCplx<T, N>, +1>(src, DstCplx<T, N>{Y}, cnt * M * N, st,
                                                                        "vjp gain slab")))
            return s;
          if (vss) {
            const int MH = (M + 1) / 2;
            SrcVssG<T, N> sg{GT, reinterpret_cast<const T *>(p.alpha_pq), bp0, M, Nr};
            if ((s = P::template slab<SrcVssG<T, N>, DstCplx<T, N>, +1>(sg, DstCplx<T, N>{Yh}, cnt * MH * N, st,
                                                                         "vjp h slab")))
              return s;
            OpAdjPencilVss<T, N> op{Y, Yh, domega ? pdots : nullptr, bp0, M};
            if ((s = P::pencil(op, cnt * N * N, st, "vjp gain pencil"))) return s;
          } else {
            OpAdjPencil<T, N> op{Y, Hp, reinterpret_cast<const T *>(p.wq), domega ? pdots : nullptr, bp0, M};
            if ((s = P::pencil(op, cnt * N * N, st, "vjp gain pencil"))) return s;
          }
          TimedLaunch tl("vjp gain acc", st);
          // second half of the tasks into the first ni volumes of GT: the spectrum
          // of g is no longer read for these items (VSS kernels still read it for
          // the items of later sub-chunks, which lie past the first lay.pc)
          hipLaunchKernelGGL((k_adj_acc<T, N>), dim3(nblk(ni * N, SPB), 2), dim3(SPB * N), 0, st, Y,
                             reinterpret_cast<const C<T> *>(p.phase), Z, GT, ib0, ni, M, Nr);
          hipLaunchKernelGGL((k_adj_acc_add<T>), dim3(nblk(ni * n3, 256)), dim3(256), 0, st, Z + ib0 * n3, GT,
                             ni * n3);
          QC_LAUNCH_CHECK("vjp gain acc");
        }
        if (domega) {
          hipLaunchKernelGGL(k_pair_dot_sum, dim3(unsigned(nb * Nr)), dim3(256), 0, st, pdots, dwg, long(N) * N);
          QC_LAUNCH_CHECK("vjp pair dots");
        }
        // gain inverse (slab pass; the pencil pass is in the assembly)
        if ((s = P::template slab<SrcCplx<T, N>, DstCplx<T, N>, +1>(SrcCplx<T, N>{Z}, DstCplx<T, N>{Z}, nb * N, st,
                                                                     "vjp inverse slab")))
          return s;
      }
      // loss adjoint spectrum Lam (H + i FG), inverse slab pass
      if ((s = P64::template slab<SrcLossAdj<N>, DstCplx<double, N>, +1>(
               SrcLossAdj<N>{H64, FG64, reinterpret_cast<const double *>(p.lam)}, DstCplx<double, N>{Lm}, nb * N,
               st, "vjp loss slab")))
        return s;
      if (df && fused_adjoint) {
        if ((s = P::pencil(OpVjpAssembleHalf<T, N>{Z, Lm, gb, df + b0 * n3}, nb * N * N, st, "vjp assemble")))
          return s;
      } else if (df) {
        if ((s = P::pencil(OpVjpAssemble<T, N>{Z, Lm, gb, df + b0 * n3}, nb * N * N, st, "vjp assemble")))
          return s;
      }
      if (domega) {
        TimedLaunch tl("vjp domega", st);
        launch_domega(H64, FG64, p.lam_p, p.dlog, dwg, dpart, domega + b0, nb, Nr, n3, st);
        QC_LAUNCH_CHECK("vjp domega");
      }
    }
    return QCOLL_OK;
  }
};

template <typename T, int N>
static long adj_acc_round(int cus) {
  constexpr int SPB = slab_spb2<T, N>();
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_adj_acc<T, N>), SPB * N,
                                                   0) != hipSuccess)
    return 0;
  // the launch for ni items has 2 * ceil(ni N / SPB) workgroups (two task halves)
  const long slots = long(occ) * cus;
  long ni = 0;
  while (2 * ((long(ni + 1) * N + SPB - 1) / SPB) <= slots) ++ni;
  return ni;
}

template <typename T>
static long adj_acc_round_t(int N, int cus) {
  switch (N) {
    case 8: return adj_acc_round<T, 8>(cus);
    case 12: return adj_acc_round<T, 12>(cus);
    case 16: return adj_acc_round<T, 16>(cus);
    case 24: return adj_acc_round<T, 24>(cus);
    case 32: return adj_acc_round<T, 32>(cus);
    case 48: return adj_acc_round<T, 48>(cus);
    default: return 0;
  }
}

long adj_acc_items_per_round(const Plan &p) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 0;
  return p.precision == QCOLL_FP32 ? adj_acc_round_t<float>(p.N, cus) : adj_acc_round_t<double>(p.N, cus);
}

template <typename T>
static qcoll_status vjp_dispatch(const Plan &p, int64_t batch, const double *f, const double *g, double *df,
                                 double *domega, bool through, void *ws, const Layout &lay, hipStream_t st) {
  switch (p.N) {
    case 8: return Vjp<T, 8>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    case 12: return Vjp<T, 12>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    case 16: return Vjp<T, 16>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    case 24: return Vjp<T, 24>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    case 32: return Vjp<T, 32>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    case 48: return Vjp<T, 48>::run(p, batch, f, g, df, domega, through, ws, lay, st);
    default: set_error("unsupported N"); return QCOLL_ENOTSUP;
  }
}

qcoll_status launch_vjp(const Plan &p, int64_t batch, const double *f, const double *g, double *df,
                        double *domega, bool through, void *ws, const Layout &lay, hipStream_t st) {
  if (p.precision == QCOLL_FP32) return vjp_dispatch<float>(p, batch, f, g, df, domega, through, ws, lay, st);
  return vjp_dispatch<double>(p, batch, f, g, df, domega, through, ws, lay, st);
}

}  // namespace qcoll
