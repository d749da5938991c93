// Fused gain adjoint (FP32, N <= 32, VHS kernels): the hot loop of the
// vector-Jacobian product for one (item, radial node) pair in one workgroup,
// with no intermediate volume in HBM.
//
// The gain part of J^T g is 2 Re ifft3[Z] with Z = sum_pq c_s fft3(y_pq),
// y_pq = w_q h_p conj(u_pq), u_pq = ifft3[c_s fft3 f] (the transform of the
// forward hot loop) and c_s the real shift multiplier of the pair's (p, q)
// (Appendix; the adjoint of the product of the two shifted copies of f).  Only
// Re ifft3[Z] is used, and it equals ifft3 of the Hermitian part of Z, so the
// kernel accumulates
//   Zh(k) = sum_q [ c_s(k) P_q(k) + conj(c_s(-k) P_q(-k)) ],  P_q = fft3(y_pq),
// on the planes k1 <= N/2 only (2 Re ifft3[Z] = ifft3[Zh] with Zh extended by
// Hermitian symmetry).  The pair's term for the omega gradient,
// <h_p, A_p> = sum_q w_q sum_j h_p (Re(u)^2 - Im(u)^2), is reduced in the same
// pass and written once per pair (no atomics).
//
// Per term the workgroup runs the stages of the forward fused kernel: lane
// (k2, k3) loads the multiplied spectrum and inverts along axis 1, transposes
// to lane (j1, k3) for axis 2 and to lane (j1, j2) for axis 3, forms y there
// (h_p read as the lane's contiguous row), and runs the same stages backwards
// to the forward spectrum in lane (k2, k3).  The partner values P(-k) sit in
// lane (-k2, -k3); every lane puts the N/2 + 1 values its partner needs into
// LDS (the transpose tile is free at that point) and reads its own.
//
// h_p = C_p g = ifft3[alpha_p g^] is formed by the workgroup itself before the
// term loop: the same three inverse stages on alpha_p g^ leave lane (j1, j2)
// with the row h_p(j1, j2, :), which it stores to the pair's scratch volume and
// re-reads (its own row, from L2) in every term.
#include <hip/hip_runtime.h>

#include "qcoll_fused.hpp"

namespace qcoll {

constexpr int pow2_floor(int n) {
  int p = 1;
  while (2 * p <= n) p *= 2;
  return p;
}

template <int N>
struct AdjGeom {
  static constexpr int H1 = N / 2 + 1;
  static constexpr size_t tile = size_t(N) * FusedGeom<N>::S1;
  static constexpr size_t exch = size_t(2) * H1 * N * N;
  static constexpr size_t work = tile > exch ? tile : exch;   // floats
  // after the work area: the axis-1 shift factors b1 of every q of the pair
  static size_t lds_bytes(int M) { return (work + size_t(2) * M * N) * sizeof(float); }
};

// H, Gs: FP32 spectra of the items' f and g [item][N^3]; alpha: the plan's
// effective per-node gain weights [N_rho][N^3] (already / N^3); Hp: scratch
// for h_p, [pair][N^3] real, written and read by the pair's workgroup; Zh:
// per-pair half spectra [pair][N/2 + 1][N^2]; dwg: [pair] <h_p, A_p> (DW).
template <int N, bool DW>
__global__ __launch_bounds__(FusedGeom<N>::NL) void k_adj_fused(const cplx<float> *__restrict__ H,
                                                                const cplx<float> *__restrict__ Gs,
                                                                const cplx<float> *__restrict__ phase,
                                                                const float *__restrict__ wq,
                                                                const float *__restrict__ alpha, float *Hp,
                                                                cplx<float> *__restrict__ Zh, double *dwg, long nbp,
                                                                int M, int Nr, float scale) {
  using G = FusedGeom<N>;
  static_assert(G::PPL == 1, "one pencil per lane");
  constexpr int NL = G::NL;
  constexpr int H1 = N / 2 + 1;
  constexpr long n2 = long(N) * N, n3 = n2 * N;
  constexpr int S1 = G::S1;
  extern __shared__ float lds[];

  const long bp = xcd_block();
  if (bp >= nbp) return;  // uniform per workgroup
  const long b = bp / Nr;
  const int p = int(bp % Nr);
  // b1 of every q in LDS: read where each stage needs it (after a barrier),
  // instead of being held in scalar registers across the whole term
  cplx<float> *b1s = reinterpret_cast<cplx<float> *>(lds + AdjGeom<N>::work);
  for (int t = threadIdx.x; t < M * N; t += NL) b1s[t] = phase[size_t(p * M + t / N) * 3 * N + t % N];
  __syncthreads();

  const int lane = threadIdx.x;
  const int hi = lane / N, lo = lane % N;
  // the lane holding pencil (-k2, -k3) in the spectral layout
  const int partner = ((N - hi) % N) * N + (N - lo) % N;

  auto wa1 = [&](int, int i) { return i * S1 + hi * N + lo; };
  auto ra1 = [&](int, int i) { return hi * S1 + i * N + lo; };
  auto wa2 = [&](int, int i) { return hi * S1 + lo * (N + 1) + i; };
  auto ra2 = [&](int, int i) { return hi * S1 + i * (N + 1) + lo; };
  // B <-> C: within each wave's own rows when a wave owns whole rows
  auto transpose_bc = [&](float(*v)[N], auto wa, auto ra) {
    if constexpr (G::WAVE_BC) lds_transpose_wave<N, 1>(lds, v, wa, ra);
    else lds_transpose<N, 1>(lds, v, wa, ra);
  };

  {
    // h_p: lane (k2, k3) loads alpha_p g^ along k1, inverse along axes 1, 2, 3
    // with the term loop's transposes, then lane (j1, j2) stores its row
    float zr[1][N], zi[1][N];
    const __amdgpu_buffer_rsrc_t gr = make_rsrc(Gs + b * n3, unsigned(n3 * sizeof(cplx<float>)));
    const float *al = alpha + size_t(p) * n3 + lane;
    static_for<0, N>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      const cplx<float> v = load_c32(gr, int(lane * sizeof(cplx<float>)), int(kk * n2 * sizeof(cplx<float>)));
      const float a = al[kk * n2];
      zr[0][kk] = v.re * a;
      zi[0][kk] = v.im * a;
    });
    fft_reg<N, +1, float>(zr[0], zi[0]);
    lds_transpose<N, 1>(lds, zr, wa1, ra1);
    lds_transpose<N, 1>(lds, zi, wa1, ra1);
    fft_reg<N, +1, float>(zr[0], zi[0]);
    transpose_bc(zr, wa2, ra2);
    transpose_bc(zi, wa2, ra2);
    fft_reg<N, +1, float>(zr[0], zi[0]);
    // h_p is real (alpha_p even and real, g real): keep the real part
    float *ho = Hp + bp * n3 + long(lane) * N;
    static_for<0, N / 4>([&](auto v4) {
      constexpr int j0 = 4 * decltype(v4)::value;
      *reinterpret_cast<float4 *>(ho + j0) = float4{zr[0][j0], zr[0][j0 + 1], zr[0][j0 + 2], zr[0][j0 + 3]};
    });
    // the term loop re-reads the row through a buffer descriptor the compiler
    // does not tie to these stores: complete them first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  }

  float acc[2 * H1];
  static_for<0, 2 * H1>([&](auto j) { acc[decltype(j)::value] = 0.f; });
  double dot = 0.0;

  const __amdgpu_buffer_rsrc_t hr = make_rsrc(H + b * n3, unsigned(n3 * sizeof(cplx<float>)));
  // h_p through a buffer descriptor, re-read for every q where it is used
  // (a plain global load is loop-invariant and would be hoisted and spilled)
  const __amdgpu_buffer_rsrc_t hpr = make_rsrc(Hp + bp * n3, unsigned(n3 * sizeof(float)));
  for (int q = 0; q < M; ++q) {
    const cplx<float> *ph = phase + size_t(p * M + q) * 3 * N;
    float zr[1][N], zi[1][N];
    // stage A, lane (k2, k3): c_s(k) = Re(b1 b2 b3) + Im(b1 b2 b3)
    const cplx<float> b2 = ph[N + hi], b3 = ph[2 * N + lo];
    const float xr = b2.re * b3.re - b2.im * b3.im;
    const float yi = b2.re * b3.im + b2.im * b3.re;
    const float Pm = xr + yi, Qm = xr - yi;
    const float Ps = Pm * scale, Qs = Qm * scale;   // the inverse's 1/N^3, once per term
    const cplx<float> *b1q = b1s + q * N;
    if constexpr (N == 32) {
      // the spectrum's loads in groups of eight, each group issued before its
      // products: left to itself the compiler waits for the later loads one
      // by one (the adjoint's register budget is full); at 24^3 the groups
      // made the adjoint slower
      static_for<0, N / 8>([&](auto gg) {
        constexpr int k0 = decltype(gg)::value * 8;
        cplx<float> v[8];
        static_for<0, 8>([&](auto ii) {
          v[decltype(ii)::value] = load_c32(hr, int(lane * sizeof(cplx<float>)),
                                            int((k0 + decltype(ii)::value) * n2 * sizeof(cplx<float>)));
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, 8>([&](auto ii) {
          constexpr int kk = k0 + decltype(ii)::value;
          const cplx<float> b1 = b1q[kk];
          const float c = b1.re * Ps + b1.im * Qs;
          zr[0][kk] = v[decltype(ii)::value].re * c;
          zi[0][kk] = v[decltype(ii)::value].im * c;
        });
      });
    } else
    static_for<0, N>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      const cplx<float> v = load_c32(hr, int(lane * sizeof(cplx<float>)), int(kk * n2 * sizeof(cplx<float>)));
      const cplx<float> b1 = b1q[kk];
      const float c = b1.re * Ps + b1.im * Qs;
      zr[0][kk] = v.re * c;
      zi[0][kk] = v.im * c;
    });
    fft_reg<N, +1, float>(zr[0], zi[0]);
    // the previous term's partner reads cross waves: finish them before the
    // A -> B writes of this term (stage A above reads only the b1 rows, which
    // the loop never writes)
    __syncthreads();
    // A -> B across waves; when the B -> C transpose after it stays in own
    // rows, the barrier after the imaginary-part reads is not needed
    lds_transpose<N, 1>(lds, zr, wa1, ra1);
    if constexpr (G::WAVE_BC) {
      static_for<0, N>([&](auto i) { lds[wa1(0, decltype(i)::value)] = zi[0][decltype(i)::value]; });
      __syncthreads();
      static_for<0, N>([&](auto i) { zi[0][decltype(i)::value] = lds[ra1(0, decltype(i)::value)]; });
    } else {
      lds_transpose<N, 1>(lds, zi, wa1, ra1);
    }
    fft_reg<N, +1, float>(zr[0], zi[0]);
    transpose_bc(zr, wa2, ra2);
    transpose_bc(zi, wa2, ra2);
    fft_reg<N, +1, float>(zr[0], zi[0]);
    // lane (j1, j2) holds u(j1, j2, :): y = w_q h_p conj(u)
    const float w = wq[q];
    float part = 0.f;
    static_for<0, N / 4>([&](auto v4) {
      constexpr int j0 = 4 * decltype(v4)::value;
      const float4 hv = __builtin_bit_cast(
          float4, __builtin_amdgcn_raw_buffer_load_b128(hpr, int(lane * N * sizeof(float)), j0 * int(sizeof(float)), 0));
      const float hs[4] = {hv.x, hv.y, hv.z, hv.w};
      static_for<0, 4>([&](auto e) {
        constexpr int j = j0 + decltype(e)::value;
        const float h = hs[decltype(e)::value];
        if constexpr (DW) part += h * (zr[0][j] * zr[0][j] - zi[0][j] * zi[0][j]);
        const float s = w * h;
        zr[0][j] = s * zr[0][j];
        zi[0][j] = -s * zi[0][j];
      });
    });
    if constexpr (DW) dot += double(w) * double(part);
    // forward transform: axis 3 here, C -> B (own rows), axis 2, B -> A (across waves), axis 1
    fft_reg<N, -1, float>(zr[0], zi[0]);
    transpose_bc(zr, ra2, wa2);
    transpose_bc(zi, ra2, wa2);
    fft_reg<N, -1, float>(zr[0], zi[0]);
    lds_transpose<N, 1>(lds, zr, ra1, wa1);
    lds_transpose<N, 1, false>(lds, zi, ra1, wa1);   // closing barrier: before the exchange writes
    fft_reg<N, -1, float>(zr[0], zi[0]);
    // lane (k2, k3): c_s(k) P(k), then the values at k1 = -s (s = 0..N/2) to the partner
    static_for<0, N>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      const cplx<float> b1 = b1q[kk];
      const float c = b1.re * Pm + b1.im * Qm;
      zr[0][kk] *= c;
      zi[0][kk] *= c;
    });
    __syncthreads();
    static_for<0, H1>([&](auto s) {
      constexpr int ss = decltype(s)::value;
      constexpr int src = (N - ss) % N;
      lds[ss * NL + lane] = zr[0][src];
      lds[(H1 + ss) * NL + lane] = zi[0][src];
    });
    __syncthreads();
    static_for<0, H1>([&](auto s) {
      constexpr int ss = decltype(s)::value;
      acc[2 * ss] += zr[0][ss] + lds[ss * NL + partner];
      acc[2 * ss + 1] += zi[0][ss] - lds[(H1 + ss) * NL + partner];
    });
  }
  cplx<float> *zo = Zh + bp * (long(H1) * n2);
  static_for<0, H1>([&](auto s) {
    constexpr int ss = decltype(s)::value;
    // streaming store: read once, by the node sum; keeps the item spectra in L2
    typedef float f2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(f2v{acc[2 * ss], acc[2 * ss + 1]}, reinterpret_cast<f2v *>(zo + ss * n2 + lane));
  });
  if constexpr (DW) {
    // fixed-order tree reduction of the lanes' dot products (NL = N^2 need
    // not be a power of two: the lanes above the largest power of two P2 <= NL
    // are folded in first)
    constexpr int P2 = pow2_floor(NL);
    double *red = reinterpret_cast<double *>(lds);
    __syncthreads();
    red[lane] = dot;
    __syncthreads();
    if (lane < NL - P2) red[lane] += red[lane + P2];
    __syncthreads();
    for (int s = P2 / 2; s > 0; s >>= 1) {
      if (lane < s) red[lane] += red[lane + s];
      __syncthreads();
    }
    if (lane == 0) dwg[bp] = red[0];
  }
}

template <int N, bool DW>
static qcoll_status launch_adj(const Plan &p, const cplx<float> *H, const cplx<float> *G, float *Hp,
                               cplx<float> *Zh, double *dwg, long nbp, hipStream_t st) {
  using A = AdjGeom<N>;
  const size_t lds = A::lds_bytes(p.M);
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_adj_fused<N, DW>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess) {
    set_error("hipFuncSetAttribute failed for the fused adjoint kernel");
    return QCOLL_EDEVICE;
  }
  TimedLaunch tl("vjp adjoint fused", st);
  const float scale = float(1.0 / double(long(N) * N * N));
  hipLaunchKernelGGL((k_adj_fused<N, DW>), dim3(unsigned(nbp)), dim3(FusedGeom<N>::NL), lds, st, H, G,
                     reinterpret_cast<const cplx<float> *>(p.phase), reinterpret_cast<const float *>(p.wq),
                     reinterpret_cast<const float *>(p.alpha_eff), Hp, Zh, dwg, nbp, p.M, p.N_rho, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("vjp adjoint fused: ") + hipGetErrorString(e));
    return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

template <int N>
static qcoll_status launch_adj_any(const Plan &p, const cplx<float> *H, const cplx<float> *G, float *Hp,
                                   cplx<float> *Zh, double *dwg, long nbp, hipStream_t st) {
  return dwg ? launch_adj<N, true>(p, H, G, Hp, Zh, dwg, nbp, st)
             : launch_adj<N, false>(p, H, G, Hp, Zh, dwg, nbp, st);
}

static size_t adj_lds_bytes(int N, int M) {
  switch (N) {
    case 8: return AdjGeom<8>::lds_bytes(M);
    case 12: return AdjGeom<12>::lds_bytes(M);
    case 16: return AdjGeom<16>::lds_bytes(M);
    case 24: return AdjGeom<24>::lds_bytes(M);
    case 32: return AdjGeom<32>::lds_bytes(M);
    default: return ~size_t(0);
  }
}

// FP32 VHS plans with N <= 32 whose shift table fits next to the LDS work
// area (160 KiB per CU), unless the two-pass schedule was requested
bool use_fused_adjoint(const Plan &p) {
  return p.schedule_user != 1 && !p.is_vss() && fused_gain_supported(p.N, p.precision) &&
         adj_lds_bytes(p.N, p.M) <= size_t(160) * 1024;
}

qcoll_status launch_adjoint_fused(const Plan &p, const void *H, const void *G, float *Hp, void *Zh, double *dwg,
                                  long nbp, hipStream_t st) {
  const auto *h = static_cast<const cplx<float> *>(H);
  const auto *g = static_cast<const cplx<float> *>(G);
  auto *z = static_cast<cplx<float> *>(Zh);
  switch (p.N) {
    case 8: return launch_adj_any<8>(p, h, g, Hp, z, dwg, nbp, st);
    case 12: return launch_adj_any<12>(p, h, g, Hp, z, dwg, nbp, st);
    case 16: return launch_adj_any<16>(p, h, g, Hp, z, dwg, nbp, st);
    case 24: return launch_adj_any<24>(p, h, g, Hp, z, dwg, nbp, st);
    case 32: return launch_adj_any<32>(p, h, g, Hp, z, dwg, nbp, st);
    default: set_error("fused adjoint kernel: unsupported N"); return QCOLL_ENOTSUP;
  }
}

}  // namespace qcoll
