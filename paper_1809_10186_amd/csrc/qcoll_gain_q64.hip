// FP64 gain loop on chip (N = 16): for one (item, radial node) pair
// and one residue class g of the second output index (j2 = 4u + g), a
// workgroup of N^2/4 lanes runs
//   A_p(j) += w_q (Re(u)^2 - Im(u)^2),  u = ifft3[c_s f^]   for every q
// (Appendix: the product of the two shifted copies of f for one quadrature
// term, packed in one complex transform) and writes its quarter of A_p once.
// Four workgroups cover one pair; nothing of the per-term volumes reaches HBM,
// where the two-pass FP64 schedule writes and re-reads M complex volumes per pair.
//
// Per term, lane (k1, t) (t < N/4):
//   stage 1: the inverse transform along axis 2 of its four pencils
//            (k1, k3 = t + m N/4), evaluated only at the outputs j2 = 4u + g:
//            with k2 = (N/4) a + b, X[4u + g] = sum_b w^(g b) w4^(u b) y_b and
//            y_b = sum_a i^(g a) x[(N/4) a + b]  (w = e^(2 pi i/N), w4 = w^4),
//            i.e. a four-term combination, a twiddle and an N/4-point
//            transform, about a third of a full transform.  The shift
//            multiplier c_s (times sqrt(w_q)) is applied as the pencil loads.
//   stage 2: a transpose among the N/4 lanes of one k1 gives lane (k1, u) all
//            k3 of j2 = 4u + g; inverse transform along axis 3.
//   stage 3: a transpose across the workgroup gives lane (u, j3) all k1 of
//            (j2, j3); inverse transform along axis 1, then the product.
// The transposes move one component at a time through an LDS tile of
// N x (N/4)(N+1) doubles.
//
// The kernel is written for any N divisible by 4, but it is launched only at
// N = 16 (1.4x faster than the two-pass schedule there).  From N = 24 a lane's
// pencil, its FFT temporaries and the N-double accumulator exceed 256 VGPRs;
// at one wave per SIMD the per-term reloads of the item spectrum from L2 are
// not hidden and the two-pass schedule is faster (2x at 24^3, 1.3x at 32^3).
#include <hip/hip_runtime.h>

#include "qcoll_fused.hpp"

namespace qcoll {

template <int N>
struct Q64Geom {
  static constexpr int N4 = N / 4;
  static constexpr int NL = N * N4;     // lanes
  static constexpr int R = N + 1;       // tile row stride (doubles)
  static constexpr int S = N4 * R;      // tile stride per k1
  static constexpr size_t lds_bytes = size_t(N) * S * sizeof(double);
  // the stage-2 transpose stays inside a wave when the N/4 lanes of a k1 do
  static constexpr bool WAVE2 = (64 % N4 == 0);
  // rows of stage-1 loads in flight (4 pencils each): the outputs and the
  // accumulator hold most of the register budget
  static constexpr int KG = 2;
};

// stage 1 for residue class G: v[m N/4 + u] = X_m[4u + G], X_m the inverse
// transform along axis 2 of pencil (k1, t + m N/4) of c_s f^
template <int N, int G>
__device__ __forceinline__ void q64_stage1(const cplx<double> *__restrict__ hb, const cplx<double> *__restrict__ ph,
                                           int k1, int t, double sc, double *vr, double *vi) {
  constexpr int N4 = N / 4, KG = Q64Geom<N>::KG;
  const cplx<double> b1 = ph[k1];
  double P[4], Qm[4];
  static_for<0, 4>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    const cplx<double> b3 = ph[2 * N + t + N4 * m];
    const double xr = b1.re * b3.re - b1.im * b3.im;
    const double xi = b1.re * b3.im + b1.im * b3.re;
    // Re(b1 b2 b3) + Im(b1 b2 b3) = b2.re P + b2.im Qm
    P[m] = (xr + xi) * sc;
    Qm[m] = (xr - xi) * sc;
  });
  static_for<0, 4 * N4>([&](auto j) {
    vr[decltype(j)::value] = 0.0;
    vi[decltype(j)::value] = 0.0;
  });
  // k2 outer (each b2 serves the four pencils), KG rows of loads in flight at
  // a time (scheduling barriers): the outputs and the accumulator already hold
  // most of the register budget
  static_for<0, N>([&](auto kk) {
    constexpr int k2 = decltype(kk)::value;
    constexpr int a = k2 / N4, bb = k2 % N4;
    constexpr int e = (G * a) & 3;   // y_b += i^e c x
    if constexpr (k2 % KG == 0) __builtin_amdgcn_sched_barrier(0);
    const cplx<double> b2 = ph[N + k2];
    static_for<0, 4>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      constexpr int o = m * N4 + bb;
      const cplx<double> h = hb[(long(k1) * N + k2) * N + t + N4 * m];
      const double c = b2.re * P[m] + b2.im * Qm[m];
      if constexpr (e == 0) {
        vr[o] += h.re * c;
        vi[o] += h.im * c;
      } else if constexpr (e == 1) {
        vr[o] -= h.im * c;
        vi[o] += h.re * c;
      } else if constexpr (e == 2) {
        vr[o] -= h.re * c;
        vi[o] -= h.im * c;
      } else {
        vr[o] += h.im * c;
        vi[o] -= h.re * c;
      }
    });
  });
  __builtin_amdgcn_sched_barrier(0);
  static_for<0, 4>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    static_for<0, N4>([&](auto bb) {
      constexpr int b = decltype(bb)::value;
      twiddle<N, G * b, +1, double>(vr[m * N4 + b], vi[m * N4 + b]);
    });
    fft_reg<N4, +1, double>(vr + m * N4, vi + m * N4);
  });
}

template <int N>
__global__ __launch_bounds__(Q64Geom<N>::NL, 2) void k_gain_q64(const cplx<double> *__restrict__ H,
                                                                const cplx<double> *__restrict__ phase,
                                                                const double *__restrict__ wq,
                                                                double *__restrict__ A, long nbp, int M, int Nr,
                                                                double scale) {
  using G = Q64Geom<N>;
  constexpr int N4 = G::N4, R = G::R, S = G::S;
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  extern __shared__ double tile[];

  const long lb = xcd_block();
  if (lb >= nbp * 4) return;  // uniform per workgroup
  const long bp = lb / 4;
  const int g = int(lb % 4);
  const long b = bp / Nr;
  const int p = int(bp % Nr);
  const int lane = threadIdx.x;
  const int k1 = lane / N4, t = lane % N4;   // stages 1 and 2
  const int u3 = lane / N, j3 = lane % N;    // stage 3: pencil (j2 = 4 u3 + g, j3)
  auto sync2 = [&]() {
    if constexpr (G::WAVE2) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  };

  double acc[N];
  static_for<0, N>([&](auto j) { acc[decltype(j)::value] = 0.0; });
  const cplx<double> *hb = H + b * n3;
  for (int q = 0; q < M; ++q) {
    const cplx<double> *ph = phase + size_t(p * M + q) * 3 * N;
    const double sc = scale * __builtin_sqrt(wq[q]);
    double vr[N], vi[N];
    switch (g) {
      case 0: q64_stage1<N, 0>(hb, ph, k1, t, sc, vr, vi); break;
      case 1: q64_stage1<N, 1>(hb, ph, k1, t, sc, vr, vi); break;
      case 2: q64_stage1<N, 2>(hb, ph, k1, t, sc, vr, vi); break;
      default: q64_stage1<N, 3>(hb, ph, k1, t, sc, vr, vi); break;
    }
    // stage 2: (k1, t) holds k3 = t + m N/4 for every u; gather all k3 of u = t.
    // The previous term's stage-3 reads cross waves: finish them first.
    __syncthreads();
    auto gather2 = [&](double *v) {
      static_for<0, 4>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        static_for<0, N4>([&](auto uu) {
          constexpr int u = decltype(uu)::value;
          tile[k1 * S + u * R + t + N4 * m] = v[m * N4 + u];
        });
      });
      sync2();
      static_for<0, N>([&](auto kk) { v[decltype(kk)::value] = tile[k1 * S + t * R + decltype(kk)::value]; });
      sync2();
    };
    gather2(vr);
    gather2(vi);
    fft_reg<N, +1, double>(vr, vi);   // axis 3: lane (k1, u = t) now holds j3 = 0..N-1
    // stage 3: gather all k1 of pencil (u3, j3)
    auto gather3 = [&](double *v) {
      static_for<0, N>([&](auto jj) { tile[k1 * S + t * R + decltype(jj)::value] = v[decltype(jj)::value]; });
      __syncthreads();
      static_for<0, N>([&](auto kk) { v[decltype(kk)::value] = tile[decltype(kk)::value * S + u3 * R + j3]; });
      __syncthreads();
    };
    gather3(vr);
    gather3(vi);
    fft_reg<N, +1, double>(vr, vi);   // axis 1: j1 = 0..N-1
    static_for<0, N>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      acc[jj] += vr[jj] * vr[jj];
      acc[jj] -= vi[jj] * vi[jj];
    });
  }
  double *a = A + bp * n3 + long(4 * u3 + g) * N + j3;
  static_for<0, N>([&](auto j) { a[decltype(j)::value * n2] = acc[decltype(j)::value]; });
}

template <int N>
static qcoll_status launch_q64(const Plan &p, const cplx<double> *H, double *A, long nbp, hipStream_t st) {
  using G = Q64Geom<N>;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gain_q64<N>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(G::lds_bytes)) != hipSuccess) {
    set_error("hipFuncSetAttribute failed for the FP64 gain kernel");
    return QCOLL_EDEVICE;
  }
  TimedLaunch tl("gain q64", st);
  const double scale = 1.0 / double(long(N) * N * N);
  hipLaunchKernelGGL((k_gain_q64<N>), dim3(unsigned(nbp * 4)), dim3(G::NL), G::lds_bytes, st, H,
                     reinterpret_cast<const cplx<double> *>(p.phase), reinterpret_cast<const double *>(p.wq), A,
                     nbp, p.M, p.N_rho, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("gain q64: ") + hipGetErrorString(e));
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

bool gain_q64_supported(int N, int precision) { return precision == QCOLL_FP64 && N == 16; }

bool use_gain_q64(const Plan &p) {
  return p.schedule != 1 && !p.is_vss() && !p.literal && gain_q64_supported(p.N, p.precision);
}

qcoll_status launch_gain_q64(const Plan &p, const void *H, double *A, long nbp, hipStream_t st) {
  const auto *h = static_cast<const cplx<double> *>(H);
  switch (p.N) {
    case 16: return launch_q64<16>(p, h, A, nbp, st);
    default: set_error("FP64 on-chip gain kernel: unsupported N"); return QCOLL_ENOTSUP;
  }
}

}  // namespace qcoll
