// Fused gain kernel (FP32, N <= 32): the whole hot loop of one (item, radial
// node) pair in one workgroup, with no intermediate volume in HBM.
//
// For each half-sphere point q the kernel forms u = ifft3[c_s * H] with the
// real shift multiplier c_s = Re beta_s + Im beta_s (s = rho_p sigma_q / 2) and
// accumulates A_p += w_q (Re(u)^2 - Im(u)^2) = w_q t1 t2 (Appendix, the
// product of the two shifted copies of f for one quadrature term).  It then
// applies the low-rank weight on chip: W_p = alpha_p(k) * fft3(A_p), so that
// the gain spectrum is the sum over p of W_p.
//
// Layout: the workgroup has N^2 lanes, one pencil each.
//   stage A  lane (k2, k3): pencil along axis 1, loaded straight from H with
//            the multiplier applied (coalesced: consecutive lanes read
//            consecutive addresses), inverse FFT in registers -> index j1;
//   stage B  lane (j1, k3): pencil along axis 2 after an LDS transpose;
//   stage C  lane (j1, j2): pencil along axis 3 after a second transpose;
//            the lane owns A_p[j1][j2][:] in registers across all q.
// The forward transform of A_p runs the same stages backwards and stores
// W_p[k1][k2][k3] for k1 <= N/2 from lane (k2, k3), coalesced (the other
// planes follow by Hermitian symmetry).
// Each transpose moves the real parts, then the imaginary parts, through one
// LDS tile of N * (N^2 + 32) floats (135 KiB at N = 32).  The padding makes
// both the writes and the reads of each transpose free of bank conflicts at
// N = 32.  Workgroups are renumbered so that consecutive (item, node) pairs
// run on the same XCD and share the item's spectrum in that XCD's L2.
#include <hip/hip_runtime.h>

#include "qcoll_fused.hpp"

namespace qcoll {

// VSS = true: sigma-dependent kernel modes (VSS kernels).  Each term's
// product t = Re(u)^2 - Im(u)^2 is transformed forward on chip (the same
// transposes run backwards), weighted by alpha_pq(k) and accumulated as a
// half spectrum (planes k1 <= N/2) in registers; the weights carry w_p w_q,
// so the multiplier is not scaled by sqrt(w_q).  The epilogue stores that sum.
template <int N, bool VSS>
__global__ __launch_bounds__(FusedGeom<N>::NL, FusedGeom<N>::WPE) void k_gain_fused(const cplx<float> *__restrict__ H,
                                                                 const cplx<float> *__restrict__ phase,
                                                                 const float *__restrict__ wq,
                                                                 const float *__restrict__ alpha_eff,
                                                                 const float *__restrict__ apq,
                                                                 cplx<float> *__restrict__ W, long nbp, int M,
                                                                 int Nr, float scale) {
  using G = FusedGeom<N>;
  constexpr int PPL = G::PPL, NL = G::NL;
  constexpr int H1 = N / 2 + 1;
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  constexpr int S1 = G::S1;
  // accumulator: VHS A_p in the C layout (N real values per pencil); VSS the
  // half spectrum in the A layout (re, im of planes k1 <= N/2)
  constexpr int NACC = VSS ? 2 * H1 : N;
  extern __shared__ float lds[];

  // XCD-aware renumbering: block i runs on XCD i % 8; give each XCD a
  // contiguous range of logical pair indices.
  const long nb = gridDim.x;
  const long full = nb / 8, rem = nb % 8;
  const long x = blockIdx.x % 8;
  const long bp = x * full + (x < rem ? x : rem) + blockIdx.x / 8;
  if (bp >= nbp) return;  // uniform per workgroup
  const long b = bp / Nr;
  const int p = int(bp % Nr);

  // pencil u of this lane is t = lane + u*NL, split as (hi, lo) = (t / N, t % N)
  // VHS: the lane index passes an empty asm statement, which keeps the
  // compiler from folding the transposes' address arithmetic into forms that
  // cost more VALU instructions in the term loop (1351 -> 1330 per term at
  // 32^3); the VSS loop does not gain from it
  int lane = threadIdx.x;
  if constexpr (!VSS) asm volatile("" : "+v"(lane));
  int hi[PPL], lo[PPL];
  static_for<0, PPL>([&](auto u) {
    const int t = lane + decltype(u)::value * NL;
    hi[decltype(u)::value] = t / N;
    lo[decltype(u)::value] = t % N;
  });

  float acc[PPL][NACC];
  static_for<0, PPL>([&](auto u) {
    static_for<0, NACC>([&](auto j) { acc[decltype(u)::value][decltype(j)::value] = 0.f; });
  });
  auto wa1 = [&](int u, int i) { return i * S1 + hi[u] * N + lo[u]; };
  auto ra1 = [&](int u, int i) { return hi[u] * S1 + i * N + lo[u]; };
  auto wa2 = [&](int u, int i) { return hi[u] * S1 + lo[u] * (N + 1) + i; };
  auto ra2 = [&](int u, int i) { return hi[u] * S1 + i * (N + 1) + lo[u]; };

  const __amdgpu_buffer_rsrc_t hr = make_rsrc(H + b * n3, unsigned(n3 * sizeof(cplx<float>)));
  for (int q = 0; q < M; ++q) {
    const cplx<float> *ph = phase + size_t(p * M + q) * 3 * N;
    float zr[PPL][N], zi[PPL][N];
    // stage A: lane (k2, k3) = (hi, lo); c(k1) = Re(b1 b23) + Im(b1 b23),
    // scaled by sqrt(w_q) (the weights are positive), so that the product
    // below accumulates w_q (Re(u)^2 - Im(u)^2) with two FMAs per point
    const float sc = VSS ? scale : scale * __builtin_sqrtf(wq[q]);
    static_for<0, PPL>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      const cplx<float> b2 = ph[N + hi[u]], b3 = ph[2 * N + lo[u]];
      const float xr = b2.re * b3.re - b2.im * b3.im;
      const float yi = b2.re * b3.im + b2.im * b3.re;
      const float P = (xr + yi) * sc, Qm = (xr - yi) * sc;
      if constexpr (VSS && N == 32) {
        // VSS mode holds its half-spectrum sum besides the pencil: the loads
        // go in groups of eight, each group's loads issued before its
        // products (left to itself the compiler waits for the later loads one
        // by one)
        static_for<0, N / 8>([&](auto gg) {
          constexpr int k0 = decltype(gg)::value * 8;
          cplx<float> v[8];
          static_for<0, 8>([&](auto ii) {
            v[decltype(ii)::value] = load_c32(hr, int((lane + u * NL) * sizeof(cplx<float>)),
                                              int((k0 + decltype(ii)::value) * n2 * sizeof(cplx<float>)));
          });
          __builtin_amdgcn_sched_barrier(0);
          static_for<0, 8>([&](auto ii) {
            constexpr int kk = k0 + decltype(ii)::value;
            const cplx<float> b1 = ph[kk];
            const float c = b1.re * P + b1.im * Qm;
            zr[u][kk] = v[decltype(ii)::value].re * c;
            zi[u][kk] = v[decltype(ii)::value].im * c;
          });
        });
      } else {
        static_for<0, N>([&](auto k) {
          constexpr int kk = decltype(k)::value;
          const cplx<float> v = load_c32(hr, int((lane + u * NL) * sizeof(cplx<float>)),
                                         int(kk * n2 * sizeof(cplx<float>)));
          const cplx<float> b1 = ph[kk];
          const float c = b1.re * P + b1.im * Qm;
          zr[u][kk] = v.re * c;
          zi[u][kk] = v.im * c;
        });
      }
      fft_reg<N, +1, float>(zr[u], zi[u]);
    });
    // A -> B: element (j1, k2, k3) at j1*S1 + k2*N + k3.  The previous
    // iteration's last reads (wave-local B -> C, or in VSS mode the cross-wave
    // B -> A without its closing barrier) must finish before these writes
    // reach other waves' rows; stage A above touches no LDS, so the barrier
    // sits here and a wave that is done with the previous term starts the
    // next term's loads and first transform while others finish theirs.
    if constexpr (G::WAVE_BC || VSS) __syncthreads();
    if constexpr (G::WAVE_BC) {
      // A -> B crosses waves: barrier after the writes; the barrier after the
      // imaginary-part reads is not needed (B -> C below stays in own rows)
      lds_transpose<N, PPL>(lds, zr, wa1, ra1);
      static_for<0, PPL>([&](auto u) {
        static_for<0, N>([&](auto i) {
          lds[wa1(decltype(u)::value, decltype(i)::value)] = zi[decltype(u)::value][decltype(i)::value];
        });
      });
      __syncthreads();
      static_for<0, PPL>([&](auto u) {
        static_for<0, N>([&](auto i) {
          zi[decltype(u)::value][decltype(i)::value] = lds[ra1(decltype(u)::value, decltype(i)::value)];
        });
      });
    } else {
      lds_transpose<N, PPL>(lds, zr, wa1, ra1);
      lds_transpose<N, PPL>(lds, zi, wa1, ra1);
    }
    static_for<0, PPL>([&](auto u) { fft_reg<N, +1, float>(zr[decltype(u)::value], zi[decltype(u)::value]); });
    // B -> C: element (j1, j2, k3) at j1*S1 + k3*(N+1) + j2
    if constexpr (G::WAVE_BC) {
      lds_transpose_wave<N, PPL>(lds, zr, wa2, ra2);
      lds_transpose_wave<N, PPL>(lds, zi, wa2, ra2);
    } else {
      lds_transpose<N, PPL>(lds, zr, wa2, ra2);
      lds_transpose<N, PPL>(lds, zi, wa2, ra2);
    }
    if constexpr (!VSS) {
      static_for<0, PPL>([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        fft_reg<N, +1, float>(zr[u], zi[u]);
        static_for<0, N>([&](auto j) {
          constexpr int jj = decltype(j)::value;
          acc[u][jj] += zr[u][jj] * zr[u][jj];
          acc[u][jj] -= zi[u][jj] * zi[u][jj];
        });
      });
    } else {
      // t = t1 t2 of this term, forward along axis 3 (lane (j1, j2))
      static_for<0, PPL>([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        fft_reg<N, +1, float>(zr[u], zi[u]);
        static_for<0, N>([&](auto j) {
          constexpr int jj = decltype(j)::value;
          const float t = zr[u][jj] * zr[u][jj] - zi[u][jj] * zi[u][jj];
          zr[u][jj] = t;
          zi[u][jj] = 0.f;
        });
        fft_reg<N, -1, float>(zr[u], zi[u]);
      });
      // C -> B (own rows), axis 2; B -> A (across waves), axis 1
      if constexpr (G::WAVE_BC) {
        lds_transpose_wave<N, PPL>(lds, zr, ra2, wa2);
        lds_transpose_wave<N, PPL>(lds, zi, ra2, wa2);
      } else {
        lds_transpose<N, PPL>(lds, zr, ra2, wa2);
        lds_transpose<N, PPL>(lds, zi, ra2, wa2);
      }
      static_for<0, PPL>([&](auto u) { fft_reg<N, -1, float>(zr[decltype(u)::value], zi[decltype(u)::value]); });
      lds_transpose<N, PPL>(lds, zr, ra1, wa1);
      lds_transpose<N, PPL, false>(lds, zi, ra1, wa1);   // closing barrier: before the next A -> B
      const float *a = apq + size_t(p * M + q) * (size_t(H1) * n2);
      static_for<0, PPL>([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        // the term's weights are loaded before the transform, which hides
        // their latency (loaded after it, each load was waited for alone)
        float wv[H1];
        static_for<0, H1>([&](auto k) { wv[decltype(k)::value] = a[decltype(k)::value * n2 + lane + u * NL]; });
        fft_reg<N, -1, float>(zr[u], zi[u]);
        static_for<0, H1>([&](auto k) {
          constexpr int kk = decltype(k)::value;
          acc[u][2 * kk] += wv[kk] * zr[u][kk];
          acc[u][2 * kk + 1] += wv[kk] * zi[u][kk];
        });
      });
    }
  }
  if constexpr (VSS) {
    cplx<float> *wout = W + bp * (long(H1) * n2);
    static_for<0, PPL>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      static_for<0, H1>([&](auto k) {
        constexpr int kk = decltype(k)::value;
        typedef float f2v __attribute__((ext_vector_type(2)));   // streaming store, as below
        __builtin_nontemporal_store(f2v{acc[u][2 * kk], acc[u][2 * kk + 1]},
                                    reinterpret_cast<f2v *>(wout + kk * n2 + lane + u * NL));
      });
    });
    return;
  } else {
  // Low-rank stage on chip: forward 3-D transform of the real A_p (the same
  // two transposes, run backwards), times the gain weights alpha_p(k) (or
  // their truncation, already / N^3), stored as the spectrum W[item][p].
  // lane (j1, j2): axis 3; lane (j1, k3): axis 2; lane (k2, k3): axis 1.
  {
    // the lane coordinates again from the thread index, so that none of the
    // term loop's values has to be kept across it for this stage
    lane = threadIdx.x;
    static_for<0, PPL>([&](auto u) {
      const int t = lane + decltype(u)::value * NL;
      hi[decltype(u)::value] = t / N;
      lo[decltype(u)::value] = t % N;
    });
    if constexpr (G::WAVE_BC) __syncthreads();
    float zr[PPL][N], zi[PPL][N];
    static_for<0, PPL>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      static_for<0, N>([&](auto j) {
        zr[u][decltype(j)::value] = acc[u][decltype(j)::value];
        zi[u][decltype(j)::value] = 0.f;
      });
      fft_reg<N, -1, float>(zr[u], zi[u]);
    });
    lds_transpose<N, PPL>(lds, zr, ra2, wa2);
    lds_transpose<N, PPL>(lds, zi, ra2, wa2);
    static_for<0, PPL>([&](auto u) { fft_reg<N, -1, float>(zr[decltype(u)::value], zi[decltype(u)::value]); });
    lds_transpose<N, PPL>(lds, zr, ra1, wa1);
    lds_transpose<N, PPL>(lds, zi, ra1, wa1);
    // W_p is Hermitian (A_p is real, alpha is even in k): only the planes
    // k1 <= N/2 are stored, compactly, (N/2 + 1) N^2 values per pair
    const float *ae = alpha_eff + long(p) * n3;
    cplx<float> *wout = W + bp * (long(N / 2 + 1) * n2);
    static_for<0, PPL>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      fft_reg<N, -1, float>(zr[u], zi[u]);
      static_for<0, N / 2 + 1>([&](auto k) {
        constexpr int kk = decltype(k)::value;
        const long o = kk * n2 + lane + u * NL;
        const float a = ae[o];
        // streaming store: the half spectra are read once, by the node sum,
        // and should not evict the item spectra the other pairs reuse from L2
        typedef float f2v __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(f2v{zr[u][kk] * a, zi[u][kk] * a}, reinterpret_cast<f2v *>(wout + o));
      });
    });
  }
  }
}

template <int N, bool VSS>
static qcoll_status launch_fused(const Plan &p, const cplx<float> *H, cplx<float> *W, long nbp, hipStream_t st) {
  using G = FusedGeom<N>;
  // the LDS tile exceeds the default dynamic limit at N = 32; set per call
  // (cheap) so that every device the process uses gets the attribute
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gain_fused<N, VSS>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(G::lds_bytes)) != hipSuccess) {
    set_error("hipFuncSetAttribute failed for the fused gain kernel");
    return QCOLL_EDEVICE;
  }
  TimedLaunch tl("gain fused", st);
  const float scale = float(1.0 / double(long(N) * N * N));
  hipLaunchKernelGGL((k_gain_fused<N, VSS>), dim3(unsigned(nbp)), dim3(G::NL), G::lds_bytes, st, H,
                     reinterpret_cast<const cplx<float> *>(p.phase), reinterpret_cast<const float *>(p.wq),
                     reinterpret_cast<const float *>(p.alpha_eff), reinterpret_cast<const float *>(p.alpha_pq), W,
                     nbp, p.M, p.N_rho, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("gain fused: ") + hipGetErrorString(e));
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

template <int N>
static qcoll_status launch_fused_any(const Plan &p, const cplx<float> *H, cplx<float> *W, long nbp, hipStream_t st) {
  return p.is_vss() ? launch_fused<N, true>(p, H, W, nbp, st) : launch_fused<N, false>(p, H, W, nbp, st);
}

bool fused_gain_supported(int N, int precision) {
  return precision == QCOLL_FP32 && (N == 8 || N == 12 || N == 16 || N == 24 || N == 32);
}

qcoll_status launch_gain_fused(const Plan &p, const void *H, void *W, long nbp, hipStream_t st) {
  const auto *h = static_cast<const cplx<float> *>(H);
  auto *a = static_cast<cplx<float> *>(W);
  switch (p.N) {
    case 8: return launch_fused_any<8>(p, h, a, nbp, st);
    case 12: return launch_fused_any<12>(p, h, a, nbp, st);
    case 16: return launch_fused_any<16>(p, h, a, nbp, st);
    case 24: return launch_fused_any<24>(p, h, a, nbp, st);
    case 32: return launch_fused_any<32>(p, h, a, nbp, st);
    default: set_error("fused gain kernel: unsupported N"); return QCOLL_ENOTSUP;
  }
}

}  // namespace qcoll
