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
// four pencils, their FFT temporaries and the N-double accumulator exceed 256
// VGPRs; at one wave per SIMD the per-term reloads of the item spectrum from L2
// are not hidden.  At N = 32 the kernel below splits j1 in two classes
// instead: one pencil per lane, two waves per SIMD.
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

// FP64 gain loop on chip at N = 32, two residue classes of the first output
// index (j1 = 2v + g, v < N/2): a workgroup of N^2/2 lanes (two waves per
// SIMD) runs the same sum for one (item, node) pair and one class, whose
// volume (N/2 x N x N complex doubles) is one N-point pencil per lane.  With
// k1 = (N/2) a + b,
//   u(2v + g) = sum_b e^(2 pi i b v / (N/2)) [e^(2 pi i g b / N) (X(b) + (-1)^g X(N/2 + b))].
//   stage A  lane l holds two pencils (k2, k3) = (l / N + (N/2) m, l % N),
//            m < 2, loaded along k1 with the shift multiplier applied
//            (consecutive lanes read consecutive k3), folded and transformed
//            (N/2 points): v = 0..N/2-1 each;
//   stage B  lane (v, k3) after a transpose across the workgroup: axis 2;
//   stage C  lane (v, j2) after a transpose inside the wave (a wave holds
//            whole planes v): axis 3, then the product; the lane owns
//            A_p[2v + g][j2][:] across all q.
// One component at a time through a tile of N/2 x N x (N+1) doubles (135 KiB);
// the odd row stride keeps the strided reads free of bank conflicts.
template <int N>
struct C2Geom {
  static constexpr int NV = N / 2;
  static constexpr int NL = N * N / 2;
  static constexpr int R = N + 1;
  static constexpr int S = N * R;
  static constexpr size_t lds_bytes = size_t(NV) * S * sizeof(double);
  static constexpr bool WAVE_BC = (64 % N == 0);
  // stage-A outputs whose two loads each are issued together: eight loads in
  // flight (four outputs) fit beside the accumulator and the outputs; with
  // the loads of one output at a time (waits after every pair) the kernel ran
  // 12% slower, with eight outputs per group it spills 32 registers
  static constexpr int KG = 4;
};

template <int N, int G>
__device__ __forceinline__ void c2_stage_a(__amdgpu_buffer_rsrc_t hr, const cplx<double> *__restrict__ ph,
                                           int lane, double sc, double *zr, double *zi) {
  constexpr int NV = C2Geom<N>::NV, NL = C2Geom<N>::NL;
  constexpr long n2 = long(N) * N;
  static_for<0, 2>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    const int t = lane + m * NL;   // pencil (k2, k3) = (t / N, t % N)
    const cplx<double> b2 = ph[N + t / N], b3 = ph[2 * N + t % N];
    // c_s(k1) = Re(b1 b2 b3) + Im(b1 b2 b3) = b1.re P + b1.im Qm, times 1/N^3 sqrt(w_q)
    const double xr = b2.re * b3.re - b2.im * b3.im;
    const double yi = b2.re * b3.im + b2.im * b3.re;
    const double P = (xr + yi) * sc, Qm = (xr - yi) * sc;
    // buffer loads with the element offset as a scalar: no per-element
    // address registers to keep across the term loop.  The loads of KG
    // outputs are issued together (2 KG in flight) before their arithmetic.
    const int vo = int(t * sizeof(cplx<double>));
    constexpr int KG = C2Geom<N>::KG;
    static_for<0, NV / KG>([&](auto gg) {
      constexpr int g0 = decltype(gg)::value * KG;
      cplx<double> hl[KG], hh[KG];
      static_for<0, KG>([&](auto ii) {
        constexpr int b = g0 + decltype(ii)::value;
        hl[decltype(ii)::value] = load_c64(hr, vo, int(b * n2 * sizeof(cplx<double>)));
        hh[decltype(ii)::value] = load_c64(hr, vo, int((NV + b) * n2 * sizeof(cplx<double>)));
      });
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, KG>([&](auto ii) {
      constexpr int b = g0 + decltype(ii)::value;
      const cplx<double> h0 = hl[decltype(ii)::value], h1 = hh[decltype(ii)::value];
      const cplx<double> e0 = ph[b], e1 = ph[NV + b];
      const double c0 = e0.re * P + e0.im * Qm, c1 = e1.re * P + e1.im * Qm;
      double yr, yim;
      if constexpr (G == 0) {
        yr = h0.re * c0 + h1.re * c1;
        yim = h0.im * c0 + h1.im * c1;
      } else {
        yr = h0.re * c0 - h1.re * c1;
        yim = h0.im * c0 - h1.im * c1;
      }
      twiddle<N, G * b, +1, double>(yr, yim);   // e^(2 pi i G b / N)
      zr[m * NV + b] = yr;
      zi[m * NV + b] = yim;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    fft_reg<NV, +1, double>(zr + m * NV, zi + m * NV);
  });
}

template <int N>
__global__ __launch_bounds__(C2Geom<N>::NL) void k_gain_c2(const cplx<double> *__restrict__ H,
                                                          const cplx<double> *__restrict__ phase,
                                                          const double *__restrict__ wq, double *__restrict__ A,
                                                          long nbp, int M, int Nr, double scale) {
  using Gm = C2Geom<N>;
  constexpr int NV = Gm::NV, R = Gm::R, S = Gm::S;
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  extern __shared__ double tile[];

  const long lb = xcd_block();
  if (lb >= nbp * 2) return;  // uniform per workgroup
  const long bp = lb / 2;
  const int g = int(lb % 2);
  const long b = bp / Nr;
  const int p = int(bp % Nr);
  const int lane = threadIdx.x;
  const int k2a = lane / N, k3a = lane % N;   // stage A: pencils (k2a + NV m, k3a)
  const int vb = lane / N, cb = lane % N;     // stages B and C: v, and k3 (B) or j2 (C)

  double acc[N];
  static_for<0, N>([&](auto j) { acc[decltype(j)::value] = 0.0; });
  const __amdgpu_buffer_rsrc_t hr = make_rsrc(H + b * n3, unsigned(n3 * sizeof(cplx<double>)));
  for (int q = 0; q < M; ++q) {
    const cplx<double> *ph = phase + size_t(p * M + q) * 3 * N;
    const double sc = scale * __builtin_sqrt(wq[q]);
    double zr[N], zi[N];
    if (g == 0) c2_stage_a<N, 0>(hr, ph, lane, sc, zr, zi);
    else c2_stage_a<N, 1>(hr, ph, lane, sc, zr, zi);
    // A -> B (across waves): element (v, k2, k3) at v*S + k2*R + k3.  The
    // previous term's stage-C reads stay inside each wave's own planes, so one
    // barrier before the writes orders them against other waves' reads.
    __syncthreads();
    auto a_to_b = [&](double *z, bool tail) {
      static_for<0, 2>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        static_for<0, NV>([&](auto vv) {
          constexpr int v = decltype(vv)::value;
          tile[v * S + (k2a + NV * m) * R + k3a] = z[m * NV + v];
        });
      });
      __syncthreads();
      static_for<0, N>([&](auto kk) { z[decltype(kk)::value] = tile[vb * S + decltype(kk)::value * R + cb]; });
      if (tail) __syncthreads();
    };
    a_to_b(zr, true);
    a_to_b(zi, false);
    fft_reg<N, +1, double>(zr, zi);   // axis 2: lane (v, k3) now holds j2 = 0..N-1
    // B -> C: element (v, j2, k3) at v*S + j2*R + k3; plane v belongs to the
    // N lanes of one wave (64 % N == 0), so the wave orders its own accesses.
    // Before the first write every wave must be done reading the A -> B tile.
    __syncthreads();
    auto b_to_c = [&](double *z) {
      static_for<0, N>([&](auto jj) { tile[vb * S + decltype(jj)::value * R + cb] = z[decltype(jj)::value]; });
      if constexpr (Gm::WAVE_BC) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __syncthreads();
      }
      static_for<0, N>([&](auto kk) { z[decltype(kk)::value] = tile[vb * S + cb * R + decltype(kk)::value]; });
      if constexpr (Gm::WAVE_BC) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __syncthreads();
      }
    };
    b_to_c(zr);
    b_to_c(zi);
    fft_reg<N, +1, double>(zr, zi);   // axis 3: lane (v, j2) holds j3 = 0..N-1
    static_for<0, N>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      acc[jj] += zr[jj] * zr[jj];
      acc[jj] -= zi[jj] * zi[jj];
    });
  }
  // A_p[2v + g][j2][j3]: N consecutive doubles per lane
  double2 *a = reinterpret_cast<double2 *>(A + bp * n3 + long(2 * vb + g) * n2 + long(cb) * N);
  static_for<0, N / 2>([&](auto j) {
    constexpr int jj = decltype(j)::value;
    a[jj] = make_double2(acc[2 * jj], acc[2 * jj + 1]);
  });
}

template <int N>
static qcoll_status launch_c2(const Plan &p, const cplx<double> *H, double *A, long nbp, hipStream_t st) {
  using G = C2Geom<N>;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gain_c2<N>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(G::lds_bytes)) != hipSuccess) {
    set_error("hipFuncSetAttribute failed for the FP64 gain kernel");
    return QCOLL_EDEVICE;
  }
  TimedLaunch tl("gain c2", st);
  const double scale = 1.0 / double(long(N) * N * N);
  hipLaunchKernelGGL((k_gain_c2<N>), dim3(unsigned(nbp * 2)), dim3(G::NL), G::lds_bytes, st, H,
                     reinterpret_cast<const cplx<double> *>(p.phase), reinterpret_cast<const double *>(p.wq), A,
                     nbp, p.M, p.N_rho, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("gain c2: ") + hipGetErrorString(e));
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
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

bool gain_q64_supported(int N, int precision) { return precision == QCOLL_FP64 && (N == 16 || N == 32); }

bool use_gain_q64(const Plan &p) {
  return p.schedule != 1 && !p.is_vss() && !p.literal && gain_q64_supported(p.N, p.precision);
}

qcoll_status launch_gain_q64(const Plan &p, const void *H, double *A, long nbp, hipStream_t st) {
  const auto *h = static_cast<const cplx<double> *>(H);
  switch (p.N) {
    case 16: return launch_q64<16>(p, h, A, nbp, st);
    case 32: return launch_c2<32>(p, h, A, nbp, st);
    default: set_error("FP64 on-chip gain kernel: unsupported N"); return QCOLL_ENOTSUP;
  }
}

}  // namespace qcoll
