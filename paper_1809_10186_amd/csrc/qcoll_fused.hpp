// Building blocks of the on-chip kernels.  The FP32 fused kernels (N <= 32):
// one workgroup of N^2 lanes owns a whole N^3 complex volume, one pencil per
// lane, and changes the pencil axis by transposes through one LDS tile; the
// FP64 kernel shares the XCD-aware block numbering.
#pragma once
#include <hip/hip_runtime.h>

#include "qcoll_fft.hpp"
#include "qcoll_internal.h"

namespace qcoll {

// Raw buffer descriptor over [base, base + bytes): loads through it take the
// per-element stride as a scalar offset (no per-element address VGPRs) and
// return 0 outside the range instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes), 0x00020000);
}

__device__ __forceinline__ cplx<float> load_c32(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  return cplx<float>{v.x, v.y};
}

__device__ __forceinline__ cplx<double> load_c64(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  return cplx<double>{v.x, v.y};
}

template <int N>
struct FusedGeom {
  // pencils per lane (1: N^2 lanes; the loops below also support 2, which
  // halves the lane count at twice the registers per lane)
  static constexpr int PPL = 1;
  static constexpr int NL = N * N / PPL;
  static constexpr int S1 = N * N + 32;
  // the B <-> C transposes stay inside a wave when a wave owns whole rows
  // (64 lanes = 64/N rows of N lanes, one pencil per lane)
  static constexpr bool WAVE_BC = (PPL == 1) && (64 % N == 0);
  static constexpr size_t lds_bytes = size_t(N) * S1 * sizeof(float);
  // waves per SIMD the register budget must allow: at N = 24 a workgroup is 9
  // waves with a 57 KiB tile, and 5 waves per SIMD let two workgroups share a
  // CU (their barrier phases then overlap); elsewhere no constraint
  static constexpr int WPE = (N == 24) ? 5 : 1;
};

// move one component (re or im) of every pencil of the lane through LDS; with
// TAIL = false the barrier after the reads is left to the caller (the tile
// must not be written again before one)
template <int N, int PPL, bool TAIL = true, class WA, class RA>
__device__ __forceinline__ void lds_transpose(float *lds, float (*v)[N], WA wa, RA ra) {
  static_for<0, PPL>([&](auto u) {
    static_for<0, N>([&](auto i) {
      lds[wa(decltype(u)::value, decltype(i)::value)] = v[decltype(u)::value][decltype(i)::value];
    });
  });
  __syncthreads();
  static_for<0, PPL>([&](auto u) {
    static_for<0, N>([&](auto i) {
      v[decltype(u)::value][decltype(i)::value] = lds[ra(decltype(u)::value, decltype(i)::value)];
    });
  });
  if constexpr (TAIL) __syncthreads();
}

// Same transpose within one wave: every address a lane writes or reads lies in
// rows owned by its own wave, so ordering the wave's LDS writes before its
// reads is enough (LDS requests of one wave are served in order; the fences
// stop the compiler from moving the accesses across each other).
template <int N, int PPL, class WA, class RA>
__device__ __forceinline__ void lds_transpose_wave(float *lds, float (*v)[N], WA wa, RA ra) {
  static_for<0, PPL>([&](auto u) {
    static_for<0, N>([&](auto i) {
      lds[wa(decltype(u)::value, decltype(i)::value)] = v[decltype(u)::value][decltype(i)::value];
    });
  });
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  static_for<0, PPL>([&](auto u) {
    static_for<0, N>([&](auto i) {
      v[decltype(u)::value][decltype(i)::value] = lds[ra(decltype(u)::value, decltype(i)::value)];
    });
  });
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// XCD-aware block numbering: hardware block i runs on XCD i % 8; logical
// indices are handed out so that each XCD gets one contiguous range (the pairs
// of one item then share the item's spectrum in that XCD's L2).
__device__ __forceinline__ long xcd_block() {
  const long nb = gridDim.x;
  const long full = nb / 8, rem = nb % 8;
  const long x = blockIdx.x % 8;
  return x * full + (x < rem ? x : rem) + blockIdx.x / 8;
}

}  // namespace qcoll
