// In-register mixed-radix FFTs for the velocity-grid transforms.
//
// fft_reg<N, SIGN>(re, im) computes X[k] = sum_j x[j] exp(SIGN * 2 pi i j k / N)
// in natural order, unnormalised, on N values held by one lane.  Every index
// and twiddle is a compile-time constant (the loops are template recursions),
// so the arrays live in VGPRs and trivial twiddles cost nothing.  N = 2^a 3^b.
//
// Twiddles: sin/cos of 2 pi n/d are evaluated at compile time by exact
// rational reduction to [0, pi/4] followed by a Taylor series; the result is
// within an ulp of the true value in double precision and is rounded once to
// the working type.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace qcoll {

template <int I>
using ic = std::integral_constant<int, I>;

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

struct SinCos {
  double s, c;
};

// sin and cos of 2 pi n / d.
constexpr SinCos sincos_2pi(long n, long d) {
  n %= d;
  if (n < 0) n += d;
  const long q = (4 * n) / d;       // quadrant 0..3
  const long r = 4 * n - q * d;     // remaining angle (pi/2) r/d, 0 <= r < d
  double s0 = 0.0, c0 = 1.0;
  if (2 * r <= d) {
    const double phi = 0.5 * kPi * double(r) / double(d);
    s0 = taylor_sin(phi);
    c0 = taylor_cos(phi);
  } else {
    const double phi = 0.5 * kPi * double(d - r) / double(d);
    s0 = taylor_cos(phi);
    c0 = taylor_sin(phi);
  }
  if (r == 0) { s0 = 0.0; c0 = 1.0; }
  switch (q) {
    case 0: return {s0, c0};
    case 1: return {c0, -s0};
    case 2: return {-s0, -c0};
    default: return {-c0, s0};
  }
}

template <typename T>
struct cplx {
  T re, im;
};

// small DFTs across r values (in place), SIGN = -1 forward, +1 inverse
template <int R, int SIGN, typename T>
__device__ __forceinline__ void small_dft(T *xr, T *xi) {
  if constexpr (R == 2) {
    T ar = xr[0] + xr[1], ai = xi[0] + xi[1];
    T br = xr[0] - xr[1], bi = xi[0] - xi[1];
    xr[0] = ar; xi[0] = ai; xr[1] = br; xi[1] = bi;
  } else if constexpr (R == 4) {
    T s02r = xr[0] + xr[2], s02i = xi[0] + xi[2];
    T d02r = xr[0] - xr[2], d02i = xi[0] - xi[2];
    T s13r = xr[1] + xr[3], s13i = xi[1] + xi[3];
    T d13r = xr[1] - xr[3], d13i = xi[1] - xi[3];
    // (SIGN i) * d13
    T wr = (SIGN > 0) ? -d13i : d13i;
    T wi = (SIGN > 0) ? d13r : -d13r;
    xr[0] = s02r + s13r; xi[0] = s02i + s13i;
    xr[2] = s02r - s13r; xi[2] = s02i - s13i;
    xr[1] = d02r + wr;   xi[1] = d02i + wi;
    xr[3] = d02r - wr;   xi[3] = d02i - wi;
  } else if constexpr (R == 3) {
    constexpr T h = T(0.5);
    constexpr T s3 = T(SIGN * 0.866025403784438646763723170752936183);
    T tr = xr[1] + xr[2], ti = xi[1] + xi[2];
    T dr = xr[1] - xr[2], di = xi[1] - xi[2];
    T mr = xr[0] - h * tr, mi = xi[0] - h * ti;
    // (i s3) * d = (-s3 di, s3 dr)
    xr[0] = xr[0] + tr; xi[0] = xi[0] + ti;
    xr[1] = mr - s3 * di; xi[1] = mi + s3 * dr;
    xr[2] = mr + s3 * di; xi[2] = mi - s3 * dr;
  }
}

template <int N>
constexpr int pick_radix() {
  return (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 3);
}

// multiply (a + ib) by exp(SIGN 2 pi i E / N)
template <int N, int E, int SIGN, typename T>
__device__ __forceinline__ void twiddle(T &a, T &b) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
  } else if constexpr (4 * e == N) {          // SIGN * i
    T t = a;
    if constexpr (SIGN > 0) { a = -b; b = t; } else { a = b; b = -t; }
  } else if constexpr (2 * e == N) {
    a = -a; b = -b;
  } else if constexpr (4 * e == 3 * N) {      // -SIGN * i
    T t = a;
    if constexpr (SIGN > 0) { a = b; b = -t; } else { a = -b; b = t; }
  } else {
    constexpr SinCos w = sincos_2pi(e, N);
    constexpr T c = T(w.c);
    constexpr T s = T(SIGN * w.s);
    T na = a * c - b * s;
    T nb = a * s + b * c;
    a = na; b = nb;
  }
}

// Twiddle split for the factored radix-4 combine: w = exp(SIGN 2 pi i E / N) =
// f (1 + i tau) with f = cos (|cos| >= |sin|), or w = f (kap + i) with f = sin
// otherwise, so that w x = f x' where x' costs two FMAs and f folds into the
// butterfly's own FMAs.  Trivial twiddles (multiples of pi/2) are exact moves.
template <int N, int E, int SIGN>
struct TwSplit {
  static constexpr int e = ((E % N) + N) % N;
  static constexpr bool trivial = (e == 0) || (4 * e == N) || (2 * e == N) || (4 * e == 3 * N);
  static constexpr SinCos w = sincos_2pi(e, N);
  static constexpr double c = w.c, s = SIGN * w.s;
  static constexpr bool by_cos = (c >= 0 ? c : -c) >= (s >= 0 ? s : -s);
  static constexpr double f = by_cos ? c : s;
  static constexpr double r = by_cos ? s / c : c / s;   // tau or kap
};

// x' with w x = f x': by cosine, x' = (a - tau b, b + tau a); by sine, x' = (kap a - b, a + kap b)
template <int N, int E, int SIGN, typename T>
__device__ __forceinline__ void twiddle_reduced(T &a, T &b) {
  using W = TwSplit<N, E, SIGN>;
  constexpr T r = T(W::r);
  if constexpr (W::by_cos) {
    const T na = a - r * b, nb = b + r * a;
    a = na;
    b = nb;
  } else {
    const T na = r * a - b, nb = a + r * b;
    a = na;
    b = nb;
  }
}

// Radix-4 combine of output column k: inputs x_i (i = 0..3) of the sub-transforms,
// twiddles w_i = exp(SIGN 2 pi i (i k) / N), then the 4-point DFT.  With
// w_i x_i = f_i x_i', the pair x0 +- w2 x2 takes f2 as an FMA multiplier, and the
// pair w1 x1 +- w3 x3 = f3 (g x1' +- x3') with g = f1 / f3 takes g there and f3 in
// the four output FMAs, so no factor costs a multiply of its own; trivial
// twiddles keep the plain moves.
template <int N, int K, int SIGN, typename T>
__device__ __forceinline__ void combine4(T *xr, T *xi) {
  using W1 = TwSplit<N, K, SIGN>;
  using W2 = TwSplit<N, 2 * K, SIGN>;
  using W3 = TwSplit<N, 3 * K, SIGN>;
  constexpr double F1 = W1::trivial ? 1.0 : W1::f;
  constexpr double F2 = W2::trivial ? 1.0 : W2::f;
  constexpr double F3 = W3::trivial ? 1.0 : W3::f;
  constexpr T g = T(F1 / F3), f2 = T(F2), f3 = T(F3);
  if constexpr (W1::trivial) twiddle<N, K, SIGN, T>(xr[1], xi[1]);
  else twiddle_reduced<N, K, SIGN, T>(xr[1], xi[1]);
  if constexpr (W2::trivial) twiddle<N, 2 * K, SIGN, T>(xr[2], xi[2]);
  else twiddle_reduced<N, 2 * K, SIGN, T>(xr[2], xi[2]);
  if constexpr (W3::trivial) twiddle<N, 3 * K, SIGN, T>(xr[3], xi[3]);
  else twiddle_reduced<N, 3 * K, SIGN, T>(xr[3], xi[3]);
  const T s02r = xr[0] + f2 * xr[2], s02i = xi[0] + f2 * xi[2];
  const T d02r = xr[0] - f2 * xr[2], d02i = xi[0] - f2 * xi[2];
  const T s13r = g * xr[1] + xr[3], s13i = g * xi[1] + xi[3];
  const T d13r = g * xr[1] - xr[3], d13i = g * xi[1] - xi[3];
  // (SIGN i) * d13, still to be scaled by f3
  const T wr = (SIGN > 0) ? -d13i : d13i;
  const T wi = (SIGN > 0) ? d13r : -d13r;
  xr[0] = s02r + f3 * s13r; xi[0] = s02i + f3 * s13i;
  xr[2] = s02r - f3 * s13r; xi[2] = s02i - f3 * s13i;
  xr[1] = d02r + f3 * wr;   xi[1] = d02i + f3 * wi;
  xr[3] = d02r - f3 * wr;   xi[3] = d02i - f3 * wi;
}

template <int N, int SIGN, typename T>
__device__ __forceinline__ void fft_reg(T *re, T *im) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2 || N == 3 || N == 4) {
    small_dft<N, SIGN, T>(re, im);
  } else {
    constexpr int R = pick_radix<N>();
    constexpr int M = N / R;
    T sr[R][M], si[R][M];
    static_for<0, R>([&](auto i) {
      static_for<0, M>([&](auto m) {
        sr[decltype(i)::value][decltype(m)::value] = re[R * decltype(m)::value + decltype(i)::value];
        si[decltype(i)::value][decltype(m)::value] = im[R * decltype(m)::value + decltype(i)::value];
      });
    });
    static_for<0, R>([&](auto i) { fft_reg<M, SIGN, T>(sr[decltype(i)::value], si[decltype(i)::value]); });
    static_for<0, M>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      T xr[R], xi[R];
      static_for<0, R>([&](auto i) {
        constexpr int ii = decltype(i)::value;
        xr[ii] = sr[ii][kk];
        xi[ii] = si[ii][kk];
      });
      if constexpr (R == 4) {
        combine4<N, kk, SIGN, T>(xr, xi);
      } else {
        static_for<0, R>([&](auto i) {
          constexpr int ii = decltype(i)::value;
          twiddle<N, ii * kk, SIGN, T>(xr[ii], xi[ii]);
        });
        small_dft<R, SIGN, T>(xr, xi);
      }
      static_for<0, R>([&](auto t) {
        re[kk + M * decltype(t)::value] = xr[decltype(t)::value];
        im[kk + M * decltype(t)::value] = xi[decltype(t)::value];
      });
    });
  }
}

}  // namespace qcoll
