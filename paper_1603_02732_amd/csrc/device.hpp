// Device helpers: wavefront/block/grid reductions and the LDS-resident
// mixed-radix Stockham FFT used by every transform of the engine.
#pragma once
#include "common.hpp"

namespace sgo {

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum N values over the block; every thread receives the totals.  The order
// of additions is fixed by the thread layout, so results are reproducible.
// sh must hold 16*N doubles.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* sh) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[i * 16 + w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += sh[i * 16 + k];
    v[i] = s;
  }
  __syncthreads();
}

// v[0..5] += w * (G G^T) in Voigt order xx yy zz yz xz xy.
__device__ __forceinline__ void add_voigt(double* v, double w, const double* G) {
  v[0] += w * G[0] * G[0];
  v[1] += w * G[1] * G[1];
  v[2] += w * G[2] * G[2];
  v[3] += w * G[1] * G[2];
  v[4] += w * G[0] * G[2];
  v[5] += w * G[0] * G[1];
}

__device__ __forceinline__ double load_coherent(const double* p) {
  unsigned long long u =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)u);
}

// Grid-wide sum of N values per block.  Each block passes its block totals
// (valid in every thread); the last block to arrive sums the partials in
// block order and returns true with the totals in out (all its threads).
// The ticket is returned to zero by that block, ready for the next launch.
template <int N>
__device__ bool grid_sum_last(const double (&v)[N], double* part, unsigned* ticket, int nblocks,
                              int bid, double (&out)[N], double* sh) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) part[(size_t)bid * N + i] = v[i];
    __threadfence();
    unsigned t = atomicAdd(ticket, 1u);
    is_last = (t == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[(size_t)b * N + i];
    out[i] = s;
  }
  block_sum<N>(out, sh);
  if (threadIdx.x == 0) atomicExch(ticket, 0u);
  return true;
}

// ----------------------------------------------------------------------- FFT
// Twiddle table tw[k] = exp(-2 pi i k / n), k < n, computed in FP64.
template <typename T>
__device__ __forceinline__ void fill_twiddles(cplx<T>* tw, int n, int tid, int nthr) {
  for (int k = tid; k < n; k += nthr) {
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = {(T)c, (T)s};
  }
}

// i * sign * z
template <typename T>
__device__ __forceinline__ cplx<T> imul(cplx<T> z, int sign) {
  return sign > 0 ? cplx<T>{-z.y, z.x} : cplx<T>{z.y, -z.x};
}

template <typename T>
__device__ __forceinline__ void bfly2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <typename T>
__device__ __forceinline__ void bfly4(cplx<T>* v, int sign) {
  cplx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  cplx<T> c = cadd(v[1], v[3]), d = imul(csub(v[1], v[3]), sign);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <typename T>
__device__ __forceinline__ void bfly3(cplx<T>* v, int sign) {
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  cplx<T> t = cadd(v[1], v[2]);
  cplx<T> u = csub(v[1], v[2]);
  cplx<T> m = {v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y};
  cplx<T> iu = imul(cplx<T>{h * u.x, h * u.y}, sign);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, iu);
  v[2] = csub(m, iu);
}
template <typename T>
__device__ __forceinline__ void bfly5(cplx<T>* v, int sign) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
  cplx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  cplx<T> u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
  cplx<T> r1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
  cplx<T> r2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
  cplx<T> q1 = imul(cplx<T>{s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y}, sign);
  cplx<T> q2 = imul(cplx<T>{s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y}, sign);
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(r1, q1);
  v[4] = csub(r1, q1);
  v[2] = cadd(r2, q2);
  v[3] = csub(r2, q2);
}

// One radix-R Stockham stage over nseq sequences of length n stored at
// element stride es and sequence stride ss, from `a` into `b`.
template <typename T, int R>
__device__ __forceinline__ void fft_stage(const cplx<T>* __restrict__ a, cplx<T>* __restrict__ b,
                                          int n, int Ns, int nseq, int es, int ss,
                                          const cplx<T>* __restrict__ tw, int sign, int tid,
                                          int nthr) {
  const int nbf = n / R;
  const int tws = n / (Ns * R);
  const int total = nbf * nseq;
  for (int t = tid; t < total; t += nthr) {
    // consecutive threads take consecutive elements when elements are
    // contiguous (es == 1), else consecutive sequences: either way the LDS
    // addresses of a wavefront are consecutive (no bank conflicts).
    int seq, j;
    if (es == 1) {
      seq = t / nbf;
      j = t - seq * nbf;
    } else {
      j = t / nseq;
      seq = t - j * nseq;
    }
    const cplx<T>* src = a + seq * ss;
    cplx<T>* dst = b + seq * ss;
    const int jm = j % Ns;
    cplx<T> v[R];
    v[0] = src[j * es];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cplx<T> x = src[(j + r * nbf) * es];
      cplx<T> w = tw[jm * r * tws];
      if (sign > 0) w.y = -w.y;
      v[r] = cmul(x, w);
    }
    if (R == 2) bfly2(v);
    if (R == 3) bfly3(v, sign);
    if (R == 4) bfly4(v, sign);
    if (R == 5) bfly5(v, sign);
    const int base = (j - jm) * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * es] = v[r];
  }
}

// Batched in-LDS FFT.  Data starts in `a`; `b` is scratch of the same
// shape.  Returns the buffer holding the result (natural order).
// sign = -1: forward  X_k = sum_j x_j e^{-2 pi i jk/n};  sign = +1: inverse
// (unnormalised).  Ends with a barrier.
template <typename T>
__device__ cplx<T>* lds_fft(cplx<T>* a, cplx<T>* b, const FftPlan& P, int nseq, int es, int ss,
                            const cplx<T>* tw, int sign, int tid, int nthr) {
  int Ns = 1;
  for (int st = 0; st < P.nstage; ++st) {
    const int R = P.radix[st];
    if (R == 4) fft_stage<T, 4>(a, b, P.n, Ns, nseq, es, ss, tw, sign, tid, nthr);
    else if (R == 2) fft_stage<T, 2>(a, b, P.n, Ns, nseq, es, ss, tw, sign, tid, nthr);
    else if (R == 3) fft_stage<T, 3>(a, b, P.n, Ns, nseq, es, ss, tw, sign, tid, nthr);
    else fft_stage<T, 5>(a, b, P.n, Ns, nseq, es, ss, tw, sign, tid, nthr);
    __syncthreads();
    cplx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// Unpack Gamma-point storage of half-sphere coefficient g of a band:
// c_G = (x[2g] + i x[2g+1]) / sqrt2 for G != 0, c_0 = x[0].
template <typename T>
__device__ __forceinline__ cplx<T> unpack_coef(const T* x, int g) {
  const T r = (T)0.70710678118654752440;
  if (g == 0) return {x[0], (T)0};
  return {x[2 * g] * r, x[2 * g + 1] * r};
}

// Perdew-Zunger 1981 LDA (unpolarised): eps_xc and v_xc = d(rho eps)/d rho.
// The r_s >= 1 branch is taken at r_s = 1; rho <= 1e-30 gives zero.
__device__ __forceinline__ void pz81(double rho, double* eps, double* v) {
  if (!(rho > 1e-30)) {
    *eps = 0.0;
    *v = 0.0;
    return;
  }
  const double pi = 3.14159265358979323846;
  const double rs = cbrt(3.0 / (4.0 * pi * rho));
  const double ex = -0.75 * cbrt(3.0 / pi) * cbrt(rho);
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double l = log(rs);
    ec = A * l + B + C * rs * l + D * rs;
    vc = A * l + (B - A / 3.0) + 2.0 / 3.0 * C * rs * l + (2.0 * D - C) / 3.0 * rs;
  }
  *eps = ex + ec;
  *v = 4.0 / 3.0 * ex + vc;
}

}  // namespace sgo
