// Register-resident mixed-radix FFT of compile-time length N = 2^a 3^b 5^c.
//
// One thread transforms one line held in its registers: decimation in time,
// X[k1 + M k2] = sum_r w_N^{r k1} Y_r[k1] w_R^{r k2} with Y_r the M-point
// transform of x[r + R m] (N = R M), recursively, fully unrolled, with every
// twiddle a compile-time constant (computed in double by a constexpr series
// and rounded once to the element type).  sign = +1 computes
// sum_n x_n e^{+2 pi i n k / N} (the inverse direction, unnormalised),
// sign = -1 the forward one.  Host and device.
#pragma once

#include <type_traits>
#include <utility>

#include "common.hpp"

namespace sgo {
namespace freg {

// cos and sin of 2 pi num / den in double, by octant reduction and Taylor
// series on |x| <= pi/4 (terms to x^25; error below 1e-17).
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 13; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 13; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
// angle = 2 pi num/den; reduce num/den to an octant with exact integer steps
constexpr void cossin(long num, long den, double& c, double& s) {
  num %= den;
  if (num < 0) num += den;
  // 8 num / den = oct + frac
  const long n8 = 8 * num;
  const long oct = n8 / den;
  const long rem = n8 - oct * den;  // angle within octant = (pi/4) rem/den
  const double x = (kTwoPi / 8.0) * (double)rem / (double)den;
  const double a = taylor_cos(x), b = taylor_sin(x);
  // from the octant's start angle oct * pi/4 via exact rotations
  const double h = 0.70710678118654752440084436210485;
  double cc = 1.0, ss = 0.0;
  switch (oct) {
    case 0: cc = 1.0; ss = 0.0; break;
    case 1: cc = h; ss = h; break;
    case 2: cc = 0.0; ss = 1.0; break;
    case 3: cc = -h; ss = h; break;
    case 4: cc = -1.0; ss = 0.0; break;
    case 5: cc = -h; ss = -h; break;
    case 6: cc = 0.0; ss = -1.0; break;
    default: cc = h; ss = -h; break;
  }
  // cos(A + x) = cA cx - sA sx, sin(A + x) = sA cx + cA sx; octant starts
  // at multiples of pi/4, where rem = 0 returns the exact start values
  if (rem == 0) {
    c = cc;
    s = ss;
  } else {
    c = cc * a - ss * b;
    s = ss * a + cc * b;
  }
}
constexpr double tw_cos(long num, long den) {
  double c = 0, s = 0;
  cossin(num, den, c, s);
  return c;
}
constexpr double tw_sin(long num, long den) {
  double c = 0, s = 0;
  cossin(num, den, c, s);
  return s;
}

template <int V>
using ic = std::integral_constant<int, V>;

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int radix_of(int n) {
  return (n % 4 == 0 && n != 8) ? 4 : (n % 2 == 0 ? 2 : (n % 3 == 0 ? 3 : 5));
}

// multiply a by e^{sign 2 pi i num/den}
template <typename T, int S, long NUM, long DEN>
__host__ __device__ __forceinline__ cplx<T> twiddle(cplx<T> a) {
  constexpr long n = ((NUM % DEN) + DEN) % DEN;
  if constexpr (n == 0) {
    return a;
  } else if constexpr (4 * n == DEN) {  // e^{sign i pi/2}
    return S > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
  } else if constexpr (2 * n == DEN) {
    return cplx<T>{-a.x, -a.y};
  } else if constexpr (4 * n == 3 * DEN) {
    return S > 0 ? cplx<T>{a.y, -a.x} : cplx<T>{-a.y, a.x};
  } else {
    constexpr T c = (T)tw_cos(n, DEN);
    constexpr T s = (T)(S * tw_sin(n, DEN));
    return cplx<T>{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

// In-place R-point DFT of v[i0 + STEP r], r < R.
template <typename T, int S, int R, int STEP, int I0, int L>
__host__ __device__ __forceinline__ void dft_small(cplx<T> (&v)[L]) {
  if constexpr (R == 2) {
    const cplx<T> a = v[I0], b = v[I0 + STEP];
    v[I0] = {a.x + b.x, a.y + b.y};
    v[I0 + STEP] = {a.x - b.x, a.y - b.y};
  } else if constexpr (R == 4) {
    const cplx<T> a = v[I0], b = v[I0 + STEP], c = v[I0 + 2 * STEP], d = v[I0 + 3 * STEP];
    const cplx<T> s0 = {a.x + c.x, a.y + c.y}, d0 = {a.x - c.x, a.y - c.y};
    const cplx<T> s1 = {b.x + d.x, b.y + d.y}, d1 = {b.x - d.x, b.y - d.y};
    // d1 * (sign i)
    const cplx<T> j1 = S > 0 ? cplx<T>{-d1.y, d1.x} : cplx<T>{d1.y, -d1.x};
    v[I0] = {s0.x + s1.x, s0.y + s1.y};
    v[I0 + STEP] = {d0.x + j1.x, d0.y + j1.y};
    v[I0 + 2 * STEP] = {s0.x - s1.x, s0.y - s1.y};
    v[I0 + 3 * STEP] = {d0.x - j1.x, d0.y - j1.y};
  } else if constexpr (R == 3) {
    constexpr T c = (T)-0.5;
    constexpr T s = (T)(S * 0.86602540378443864676372317075294);
    const cplx<T> a = v[I0], b = v[I0 + STEP], d = v[I0 + 2 * STEP];
    const cplx<T> t = {b.x + d.x, b.y + d.y}, u = {b.x - d.x, b.y - d.y};
    const cplx<T> m = {a.x + c * t.x, a.y + c * t.y};
    v[I0] = {a.x + t.x, a.y + t.y};
    v[I0 + STEP] = {m.x - s * u.y, m.y + s * u.x};
    v[I0 + 2 * STEP] = {m.x + s * u.y, m.y - s * u.x};
  } else {  // R == 5
    constexpr T c1 = (T)0.30901699437494742410229341718282;   // cos 2pi/5
    constexpr T c2 = (T)-0.80901699437494742410229341718282;  // cos 4pi/5
    constexpr T s1 = (T)(S * 0.95105651629515357211643933337938);
    constexpr T s2 = (T)(S * 0.58778525229247312916870595463907);
    const cplx<T> a = v[I0], b = v[I0 + STEP], c = v[I0 + 2 * STEP], d = v[I0 + 3 * STEP],
                  e = v[I0 + 4 * STEP];
    const cplx<T> p1 = {b.x + e.x, b.y + e.y}, m1 = {b.x - e.x, b.y - e.y};
    const cplx<T> p2 = {c.x + d.x, c.y + d.y}, m2 = {c.x - d.x, c.y - d.y};
    const cplx<T> q1 = {a.x + c1 * p1.x + c2 * p2.x, a.y + c1 * p1.y + c2 * p2.y};
    const cplx<T> q2 = {a.x + c2 * p1.x + c1 * p2.x, a.y + c2 * p1.y + c1 * p2.y};
    const cplx<T> r1 = {s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y};  // times i below
    const cplx<T> r2 = {s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y};
    v[I0] = {a.x + p1.x + p2.x, a.y + p1.y + p2.y};
    v[I0 + STEP] = {q1.x - r1.y, q1.y + r1.x};
    v[I0 + 4 * STEP] = {q1.x + r1.y, q1.y - r1.x};
    v[I0 + 2 * STEP] = {q2.x - r2.y, q2.y + r2.x};
    v[I0 + 3 * STEP] = {q2.x + r2.y, q2.y - r2.x};
  }
}

// Transform of the N values v[OFF + STRIDE n], n < N, written in natural
// order to w[WOFF + k], k < N (w and v distinct arrays).
template <typename T, int S, int N, int STRIDE, int OFF, int WOFF, int L, int LW>
__host__ __device__ __forceinline__ void dit(const cplx<T> (&v)[L], cplx<T> (&w)[LW]) {
  if constexpr (N == 1) {
    w[WOFF] = v[OFF];
  } else {
    constexpr int R = radix_of(N), M = N / R;
    // sub-transforms of the R decimated sequences into w[WOFF + r M + k1]
    static_for<0, R>([&](auto r) {
      dit<T, S, M, STRIDE * R, OFF + STRIDE * decltype(r)::value, WOFF + M * decltype(r)::value,
          L, LW>(v, w);
    });
    // twiddles and R-point butterflies, in place over {WOFF + k1 + M r}
    static_for<0, M>([&](auto k1) {
      constexpr int K1 = decltype(k1)::value;
      static_for<1, R>([&](auto r) {
        constexpr int RR = decltype(r)::value;
        w[WOFF + K1 + M * RR] = twiddle<T, S, (long)RR * K1, N>(w[WOFF + K1 + M * RR]);
      });
      dft_small<T, S, R, M, WOFF + K1, LW>(w);
    });
  }
}

// Whole-line transform: out[k] = sum_n in[n] e^{sign 2 pi i n k / N}.
template <typename T, int S, int N>
__host__ __device__ __forceinline__ void fft(const cplx<T> (&in)[N], cplx<T> (&out)[N]) {
  dit<T, S, N, 1, 0, 0, N, N>(in, out);
}

}  // namespace freg
}  // namespace sgo
