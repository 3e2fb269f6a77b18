// k-point sampling of the Brillouin zone (the rough k-point grids that
// Section 2.3 allows for the energy evaluations of a search): FP64 kernels
// of the complex-band path.  At a k-point the Bloch periodic parts
// u_nk = sum_G c_G e^{iG.r} live on the shifted sphere |k+G|^2/2 <= Ecut,
// complex with no relation between c(G) and c(-G), so one band is one
// complex FFT (no pairing of two real bands) and every subspace matrix is
// complex Hermitian.  Bands are rows X[band][npw] of complex coefficients.
// The steps are those of Algorithm 1 (H psi, subspace matrix, Cholesky
// orthonormalisation, subspace diagonalisation, residual, preconditioned
// CG direction, projection, line minimisation) for each k, and the density
// of Section 2.4 summed over k with the k-point weights.  The grid side
// (mixing, potentials, energies) is the Gamma path's.
#include "device.hpp"
#include "launch.hpp"

#include <algorithm>

namespace sgo {

using zc = cplx<double>;

__device__ __forceinline__ zc zconj(zc a) { return {a.x, -a.y}; }
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) b
__device__ __forceinline__ zc zcmul(zc a, zc b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
__device__ __forceinline__ zc zscale(zc a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ zc zadd(zc a, zc b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ zc zsub(zc a, zc b) { return {a.x - b.x, a.y - b.y}; }

__device__ __forceinline__ double wave_sum_kp(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ grids
__global__ void k_kpt_zero(zc* __restrict__ a, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    a[e] = {0.0, 0.0};
}

// zk[b][box[g]] = X[b][g]
__global__ void k_kpt_scatter(zc* __restrict__ zk, const zc* __restrict__ X, const int* __restrict__ box,
                              int npw, int nb, long ntot) {
  const long n = (long)nb * npw;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e / npw), g = (int)(e - (long)b * npw);
    zk[(long)b * ntot + box[g]] = X[e];
  }
}

// Batched line transforms along one axis of grids [nb][N3][N2][N1]: line l
// starts at (l / A) * Bs + (l % A) * Cs and its elements are es apart.  L
// lines per workgroup go through the LDS Stockham passes together.
__global__ void __launch_bounds__(256) k_kpt_lines(zc* __restrict__ data, FftPlan P, int A, long Bs,
                                                   long Cs, long es, long nlines, int L, int sign) {
  extern __shared__ __align__(16) char smem[];
  const int n = P.n;
  zc* a = (zc*)smem;
  zc* b = a + (size_t)L * n;
  zc* tw = b + (size_t)L * n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, n, tid, nthr);
  const long l0 = (long)blockIdx.x * L;
  for (int t = tid; t < L * n; t += nthr) {
    int li, j;
    if (es == 1) {
      li = t / n;
      j = t - li * n;
    } else {  // consecutive threads on consecutive lines: consecutive addresses
      j = t / L;
      li = t - j * L;
    }
    const long l = l0 + li;
    a[li * n + j] = l < nlines ? data[(l / A) * Bs + (l % A) * Cs + j * es] : zc{0.0, 0.0};
  }
  __syncthreads();
  zc* r = lds_fft(a, b, P, L, 1, n, tw, sign, tid, nthr);
  for (int t = tid; t < L * n; t += nthr) {
    int li, j;
    if (es == 1) {
      li = t / n;
      j = t - li * n;
    } else {
      j = t / L;
      li = t - j * L;
    }
    const long l = l0 + li;
    if (l < nlines) data[(l / A) * Bs + (l % A) * Cs + j * es] = r[li * n + j];
  }
}

// zk[b][r] *= V(r)
__global__ void k_kpt_vmul(zc* __restrict__ zk, const double* __restrict__ v, int nb, long ntot) {
  const long n = (long)nb * ntot;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    zk[e] = zscale(zk[e], v[e % ntot]);
}

// Y[b][g] = |k+G|^2/2 X[b][g] + zk[b][box[g]] / ntot
__global__ void k_kpt_gather(const zc* __restrict__ zk, const zc* __restrict__ X, zc* __restrict__ Y,
                             const int* __restrict__ box, const double* __restrict__ kin, int npw,
                             int nb, long ntot) {
  const long n = (long)nb * npw;
  const double s = 1.0 / (double)ntot;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e / npw), g = (int)(e - (long)b * npw);
    const zc w = zk[(long)b * ntot + box[g]];
    Y[e] = {kin[g] * X[e].x + w.x * s, kin[g] * X[e].y + w.y * s};
  }
}

// ------------------------------------------------------- band products
// C[i * ldc + j] = sum_g conj(A[i][g]) B[j][g] (times i q_a(g) when q is
// given: the derivative of a projector phase e^{-i(k+G).R}); one wavefront
// per output element.
__global__ void __launch_bounds__(256) k_kpt_zdot(const zc* __restrict__ A, int na,
                                                  const zc* __restrict__ B, int nbb, int npw,
                                                  zc* __restrict__ C, int ldc,
                                                  const double* __restrict__ q, int qa) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w >= na * nbb) return;
  const int i = w / nbb, j = w - i * nbb;
  const zc* a = A + (size_t)i * npw;
  const zc* b = B + (size_t)j * npw;
  double re = 0.0, im = 0.0;
  for (int g = lane; g < npw; g += 64) {
    zc t = zcmul(a[g], b[g]);
    if (q) t = {-q[3 * g + qa] * t.y, q[3 * g + qa] * t.x};  // i q t
    re += t.x;
    im += t.y;
  }
  re = wave_sum_kp(re);
  im = wave_sum_kp(im);
  if (lane == 0) C[(size_t)i * ldc + j] = {re, im};
}

// Y[i][g] = beta Y[i][g] + alpha sum_j s_j X[j][g] M[j * ldm + i]
// (s_j = h[j] when h is given, else 1); one thread per output coefficient.
__global__ void k_kpt_zgemm(const zc* __restrict__ X, int nx, const zc* __restrict__ M, int ldm,
                            zc* __restrict__ Y, int ny, int npw, double alpha, double beta,
                            const double* __restrict__ h) {
  const long n = (long)ny * npw;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / npw), g = (int)(e - (long)i * npw);
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nx; ++j) {
      zc m = M[(size_t)j * ldm + i];
      if (h) m = zscale(m, h[j]);
      const zc t = zmul(X[(size_t)j * npw + g], m);
      re += t.x;
      im += t.y;
    }
    const zc y = beta == 0.0 ? zc{0.0, 0.0} : zscale(Y[e], beta);
    Y[e] = {y.x + alpha * re, y.y + alpha * im};
  }
}

__global__ void k_kpt_copy(zc* __restrict__ dst, const zc* __restrict__ src, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// ------------------------------------------------------------ projectors
// beta_{k,Ilm}(G) = p_l(|k+G|) (-i)^l Y_lm(k+G) e^{-i(k+G).R_I} / sqrt(Omega)
// with the normalised Gaussian radial projectors (l = 0, 1) of the Gamma
// setup, evaluated at q = k + G.
__global__ void k_kpt_beta(zc* __restrict__ beta, const double* __restrict__ q, int npw, int nproj,
                           const int* __restrict__ patom, const int* __restrict__ plm,
                           const double* __restrict__ pr, const double* __restrict__ pos,
                           double omega) {
  const int p = blockIdx.y;
  if (p >= nproj) return;
  const int I = patom[p], l = plm[p] >> 2, m = plm[p] & 3;
  const double rl = pr[p];
  const double pi = 3.14159265358979323846;
  const double inv = 1.0 / sqrt(omega);
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npw; g += gridDim.x * blockDim.x) {
    const double q0 = q[3 * g], q1 = q[3 * g + 1], q2 = q[3 * g + 2];
    const double qq = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
    double val;
    if (l == 0) {
      val = 4.0 * pi * sqrt(pi) * pow(rl, 1.5) * exp(-0.5 * qq * qq * rl * rl) /
            sqrt(0.5 * sqrt(pi)) * (1.0 / sqrt(4.0 * pi));
    } else {
      const double qm = m == 0 ? q0 : (m == 1 ? q1 : q2);
      val = 4.0 * pi * sqrt(pi) * pow(rl, 2.5) * exp(-0.5 * qq * qq * rl * rl) /
            sqrt(0.75 * sqrt(pi)) * sqrt(3.0 / (4.0 * pi)) * qm;
    }
    val *= inv;
    double sn, cs;
    sincos(-(q0 * pos[3 * I] + q1 * pos[3 * I + 1] + q2 * pos[3 * I + 2]), &sn, &cs);
    zc v = {val * cs, val * sn};
    if (l == 1) v = {v.y, -v.x};  // times -i
    beta[(size_t)p * npw + g] = v;
  }
}

// ------------------------------------------------- complex subspace step
// One workgroup, matrices in global memory (n x n complex, row-major):
//   S = L L^H (Cholesky, lower), W = L^-1, H' = W H W^H, cyclic complex
//   Jacobi H' = V diag V^H, M = W^H V with eigenvalues ascending.
// mode 1: M = W^H only (orthonormalisation).  New band i = sum_j old band j
// M[j][i].  fail receives 1 if S is not positive definite.
__device__ __forceinline__ void zjacobi_rot(zc apq, double app, double aqq, double* c, double* s,
                                            zc* ph) {
  const double r = sqrt(apq.x * apq.x + apq.y * apq.y);
  if (r == 0.0) {
    *c = 1.0;
    *s = 0.0;
    *ph = {1.0, 0.0};
    return;
  }
  *ph = {apq.x / r, apq.y / r};  // e^{i phi}
  const double tau = (aqq - app) / (2.0 * r);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * *c;
}

__global__ void __launch_bounds__(256) k_kpt_subspace(zc* __restrict__ S, zc* __restrict__ H,
                                                      zc* __restrict__ W, zc* __restrict__ V,
                                                      zc* __restrict__ M, double* __restrict__ eps,
                                                      int n, int mode, int* __restrict__ fail) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  __shared__ int bad;
  __shared__ double sh[8];
  __shared__ int rank[256];
  if (tid == 0) bad = 0;
  __syncthreads();
  // Cholesky, in place in S (lower triangle)
  for (int k = 0; k < n; ++k) {
    const double d = S[(size_t)k * n + k].x;
    if (!(d > 0.0)) {
      if (tid == 0) bad = 1;
      break;
    }
    const double piv = sqrt(d), ip = 1.0 / piv;
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += nthr) S[(size_t)i * n + k] = zscale(S[(size_t)i * n + k], ip);
    __syncthreads();
    if (tid == 0) S[(size_t)k * n + k] = {piv, 0.0};
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += nthr) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i)
        S[(size_t)i * n + j] = zsub(S[(size_t)i * n + j], zmul(S[(size_t)i * n + k], zconj(S[(size_t)j * n + k])));
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *fail = 1;
    for (int e = tid; e < n * n; e += nthr) M[e] = (e / n == e % n) ? zc{1.0, 0.0} : zc{0.0, 0.0};
    return;
  }
  // W = L^-1 by forward substitution, one column per thread group
  for (int e = tid; e < n * n; e += nthr) W[e] = {0.0, 0.0};
  __syncthreads();
  for (int c = tid; c < n; c += nthr) {
    for (int i = c; i < n; ++i) {
      zc s = i == c ? zc{1.0, 0.0} : zc{0.0, 0.0};
      for (int k = c; k < i; ++k) s = zsub(s, zmul(S[(size_t)i * n + k], W[(size_t)k * n + c]));
      W[(size_t)i * n + c] = zscale(s, 1.0 / S[(size_t)i * n + i].x);
    }
  }
  __syncthreads();
  if (mode == 1) {
    for (int e = tid; e < n * n; e += nthr) {
      const int j = e / n, i = e % n;
      M[e] = zconj(W[(size_t)i * n + j]);  // (W^H)[j][i]
    }
    return;
  }
  // H' = W H W^H: first T = W H into V, then H' = T W^H into S
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e / n, j = e % n;
    zc s = {0.0, 0.0};
    for (int k = 0; k <= i; ++k) s = zadd(s, zmul(W[(size_t)i * n + k], H[(size_t)k * n + j]));
    V[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e / n, j = e % n;
    zc s = {0.0, 0.0};
    for (int k = 0; k <= j; ++k) s = zadd(s, zmul(V[(size_t)i * n + k], zconj(W[(size_t)j * n + k])));
    S[e] = s;
  }
  __syncthreads();
  // Hermitian part, V = I
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e / n, j = e % n;
    if (i < j) {
      const zc a = S[(size_t)i * n + j], b = zconj(S[(size_t)j * n + i]);
      const zc h = {0.5 * (a.x + b.x), 0.5 * (a.y + b.y)};
      S[(size_t)i * n + j] = h;
      S[(size_t)j * n + i] = zconj(h);
    } else if (i == j) {
      S[e].y = 0.0;
    }
    V[e] = i == j ? zc{1.0, 0.0} : zc{0.0, 0.0};
  }
  __syncthreads();
  // cyclic Jacobi: for each pair (p, q), U = D J with D = diag(1, e^{-i phi})
  // and the real rotation J = [[c, s], [-s, c]] that diagonalises the real
  // 2x2 block [[a_pp, |a_pq|], [|a_pq|, a_qq]]; H' <- U^H H' U, V <- V U
  for (int sweep = 0; sweep < 60; ++sweep) {
    double v[2] = {0.0, 0.0};
    for (int e = tid; e < n * n; e += nthr) {
      const zc a = S[e];
      if (e / n == e % n) v[1] += a.x * a.x;
      else v[0] += a.x * a.x + a.y * a.y;
    }
    v[0] = wave_sum_kp(v[0]);
    v[1] = wave_sum_kp(v[1]);
    __syncthreads();
    if ((tid & 63) == 0) {
      sh[2 * (tid >> 6)] = v[0];
      sh[2 * (tid >> 6) + 1] = v[1];
    }
    __syncthreads();
    double off = 0.0, dia = 0.0;
    for (int w = 0; w < (nthr + 63) / 64; ++w) {
      off += sh[2 * w];
      dia += sh[2 * w + 1];
    }
    __syncthreads();
    if (!(off > 1e-26 * dia + 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int qq = p + 1; qq < n; ++qq) {
        double c, s;
        zc ph;
        zjacobi_rot(S[(size_t)p * n + qq], S[(size_t)p * n + p].x, S[(size_t)qq * n + qq].x, &c, &s, &ph);
        __syncthreads();
        if (s == 0.0) continue;
        const zc phc = zconj(ph);  // e^{-i phi}
        // columns p, q of H' and V: col_p <- c col_p - s e^{-i phi} col_q,
        // col_q <- s col_p + c e^{-i phi} col_q
        for (int k = tid; k < 2 * n; k += nthr) {
          zc* A = k < n ? S : V;
          const int r = k < n ? k : k - n;
          const zc ap = A[(size_t)r * n + p], aq = zmul(A[(size_t)r * n + qq], phc);
          A[(size_t)r * n + p] = {c * ap.x - s * aq.x, c * ap.y - s * aq.y};
          A[(size_t)r * n + qq] = {s * ap.x + c * aq.x, s * ap.y + c * aq.y};
        }
        __syncthreads();
        // rows p, q of H': row_p <- c row_p - s e^{i phi} row_q,
        // row_q <- s row_p + c e^{i phi} row_q
        for (int k = tid; k < n; k += nthr) {
          const zc ap = S[(size_t)p * n + k], aq = zmul(S[(size_t)qq * n + k], ph);
          S[(size_t)p * n + k] = {c * ap.x - s * aq.x, c * ap.y - s * aq.y};
          S[(size_t)qq * n + k] = {s * ap.x + c * aq.x, s * ap.y + c * aq.y};
        }
        __syncthreads();
        if (tid == 0) {
          S[(size_t)p * n + qq] = {0.0, 0.0};
          S[(size_t)qq * n + p] = {0.0, 0.0};
          S[(size_t)p * n + p].y = 0.0;
          S[(size_t)qq * n + qq].y = 0.0;
        }
        __syncthreads();
      }
  }
  // ascending order (ties by index); M = W^H V with columns by rank
  for (int i = tid; i < n; i += nthr) {
    const double li = S[(size_t)i * n + i].x;
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = S[(size_t)j * n + j].x;
      if (lj < li || (lj == li && j < i)) ++r;
    }
    rank[i] = r;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += nthr) {
    const int j = e / n, i = e % n;
    zc s = {0.0, 0.0};
    for (int k = j; k < n; ++k) s = zadd(s, zcmul(W[(size_t)k * n + j], V[(size_t)k * n + i]));
    M[(size_t)j * n + rank[i]] = s;
  }
  for (int i = tid; i < n; i += nthr) eps[rank[i]] = S[(size_t)i * n + i].x;
}

// ------------------------------------------------------ CG and line search
__device__ __forceinline__ double tpa_k(double x) {
  const double p = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
  return p / (p + 16.0 * x * x * x * x);
}

template <int N>
__device__ __forceinline__ void block_sum_kp(double (&v)[N], double* sh) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum_kp(v[i]);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) sh[i * 16 + w] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += sh[i * 16 + k];
    v[i] = s;
  }
  __syncthreads();
}

// residual R = H x - eps x, Teter-Payne-Allan preconditioned g = K R,
// D = g + (gamma / gamma_prev) D_prev (Fletcher-Reeves on the
// preconditioned norm); one workgroup per band
__global__ void __launch_bounds__(256) k_kpt_cg_dir(const zc* __restrict__ X, const zc* __restrict__ HX,
                                                    zc* __restrict__ D, const double* __restrict__ kin,
                                                    const double* __restrict__ eps, double* __restrict__ gam,
                                                    int npw, int first) {
  const int i = blockIdx.x;
  __shared__ double sh[16 * 2];
  const zc* x = X + (size_t)i * npw;
  const zc* hx = HX + (size_t)i * npw;
  zc* d = D + (size_t)i * npw;
  double v[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) v[0] += kin[g] * (x[g].x * x[g].x + x[g].y * x[g].y);
  block_sum_kp<1>(v, sh);
  const double ek = fmax(v[0], 1e-8), e = eps[i];
  double w[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const zc r = {hx[g].x - e * x[g].x, hx[g].y - e * x[g].y};
    w[0] += tpa_k(kin[g] / ek) * (r.x * r.x + r.y * r.y);
  }
  block_sum_kp<1>(w, sh);
  const double gm = w[0];
  const double beta = first ? 0.0 : (gam[i] > 0.0 ? gm / gam[i] : 0.0);
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double kk = tpa_k(kin[g] / ek);
    const zc r = {hx[g].x - e * x[g].x, hx[g].y - e * x[g].y};
    const zc dp = first ? zc{0.0, 0.0} : d[g];
    d[g] = {kk * r.x + beta * dp.x, kk * r.y + beta * dp.y};
  }
  if (threadIdx.x == 0) gam[i] = gm;
}

// exact minimiser of the 2x2 Rayleigh quotient in span{x, d / |d|} (d is
// orthogonal to every band): theta = atan2(-2b, c - a) / 2 with
// a = <x|H|x>, b = Re<x|H|d>/|d|, c = <d|H|d>/|d|^2
__global__ void __launch_bounds__(256) k_kpt_linemin(zc* __restrict__ X, zc* __restrict__ HX,
                                                     const zc* __restrict__ D, const zc* __restrict__ HD,
                                                     int npw) {
  const int i = blockIdx.x;
  __shared__ double sh[16 * 4];
  zc* x = X + (size_t)i * npw;
  zc* hx = HX + (size_t)i * npw;
  const zc* d = D + (size_t)i * npw;
  const zc* hd = HD + (size_t)i * npw;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    v[0] += x[g].x * hx[g].x + x[g].y * hx[g].y;
    v[1] += x[g].x * hd[g].x + x[g].y * hd[g].y;
    v[2] += d[g].x * hd[g].x + d[g].y * hd[g].y;
    v[3] += d[g].x * d[g].x + d[g].y * d[g].y;
  }
  block_sum_kp<4>(v, sh);
  if (!(v[3] > 0.0)) return;
  const double inv = 1.0 / sqrt(v[3]);
  const double a = v[0], b = v[1] * inv, c = v[2] * inv * inv;
  const double th = 0.5 * atan2(-2.0 * b, c - a);
  double sn, cs;
  sincos(th, &sn, &cs);
  const double s2 = sn * inv;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    x[g] = {cs * x[g].x + s2 * d[g].x, cs * x[g].y + s2 * d[g].y};
    hx[g] = {cs * hx[g].x + s2 * hd[g].x, cs * hx[g].y + s2 * hd[g].y};
  }
}

// random starting bands, damped by 1/(1 + |k+G|^2/2) (counter-based hash of
// (seed, k, band, coefficient))
__device__ __forceinline__ double hash_unit(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}
__global__ void k_kpt_init(zc* __restrict__ X, const double* __restrict__ kin, int npw, int nb,
                           unsigned seed, int kidx) {
  const long n = (long)nb * npw;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int g = (int)(e % npw);
    const unsigned long long base = ((unsigned long long)seed << 40) ^ ((unsigned long long)kidx << 32) ^
                                    (unsigned long long)e * 2ull;
    const double s = 1.0 / (1.0 + kin[g]);
    X[e] = {hash_unit(base) * s, hash_unit(base + 1) * s};
  }
}

// ------------------------------------------------ occupations, density
// Occupations over every k with one chemical potential (Fermi-Dirac,
// sum_k w_k sum_n f_nk = N_el) or fixed (the lowest N_el/2 states of each k
// doubly occupied); writes occ[k][n] and the band energy, entropy and mu
// into the structure's status block (slots as at Gamma).
__global__ void k_kpt_occupations(const double* __restrict__ eps, const double* __restrict__ wk,
                                  int nk, int nb, double nelec, int kind, double sigma,
                                  double* __restrict__ occ, double* __restrict__ scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = nk * nb;
  double mu;
  if (kind == 0) {
    const int nocc = (int)(nelec / 2.0 + 0.5);
    double hi = -1e300, lo = 1e300;
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < nb; ++i) {
        occ[k * nb + i] = i < nocc ? 2.0 : 0.0;
        if (i == nocc - 1) hi = fmax(hi, eps[k * nb + i]);
        if (i == nocc) lo = fmin(lo, eps[k * nb + i]);
      }
    mu = nocc < nb ? 0.5 * (hi + lo) : hi;
    double eb = 0.0;
    for (int e = 0; e < n; ++e) eb += wk[e / nb] * occ[e] * eps[e];
    scal[S_EBAND] = eb;
    scal[S_ENTROPY] = 0.0;
    scal[S_MU] = mu;
    return;
  }
  double lo = 1e300, hi = -1e300;
  for (int e = 0; e < n; ++e) {
    lo = fmin(lo, eps[e]);
    hi = fmax(hi, eps[e]);
  }
  lo -= 40.0 * sigma;
  hi += 40.0 * sigma;
  for (int it = 0; it < 200; ++it) {
    mu = 0.5 * (lo + hi);
    double s = 0.0;
    for (int e = 0; e < n; ++e) s += wk[e / nb] * 2.0 / (1.0 + exp((eps[e] - mu) / sigma));
    if (s > nelec) hi = mu;
    else lo = mu;
  }
  mu = 0.5 * (lo + hi);
  double eb = 0.0, ent = 0.0;
  for (int e = 0; e < n; ++e) {
    const double f = 2.0 / (1.0 + exp((eps[e] - mu) / sigma));
    occ[e] = f;
    const double g = fmin(fmax(0.5 * f, 1e-300), 1.0), gm = fmin(fmax(1.0 - 0.5 * f, 1e-300), 1.0);
    eb += wk[e / nb] * f * eps[e];
    ent += wk[e / nb] * (g * log(g) + gm * log(gm));
  }
  scal[S_EBAND] = eb;
  scal[S_ENTROPY] = -2.0 * ent;
  scal[S_MU] = mu;
}

// kinetic energy of each band, sum_G |k+G|^2/2 |c|^2
__global__ void __launch_bounds__(256) k_kpt_band_kinetic(const zc* __restrict__ X,
                                                          const double* __restrict__ kin, int npw,
                                                          double* __restrict__ out) {
  const int i = blockIdx.x;
  __shared__ double sh[16];
  const zc* x = X + (size_t)i * npw;
  double v[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) v[0] += kin[g] * (x[g].x * x[g].x + x[g].y * x[g].y);
  block_sum_kp<1>(v, sh);
  if (threadIdx.x == 0) out[i] = v[0];
}

// the structure's band arrays carry the k-weighted kinetic energy for the
// energy bookkeeping of the SCF control: occ[0] = 1, bandw[0] = sum_k w_k
// sum_n f_nk E_kin,nk, the other entries 0
__global__ void k_kpt_kinetic_total(const double* __restrict__ bandw_k, const double* __restrict__ occ_k,
                                    const double* __restrict__ wk, int nk, int nb,
                                    double* __restrict__ occ_s, double* __restrict__ bandw_s, int nb_s) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int e = 0; e < nk * nb; ++e) t += wk[e / nb] * occ_k[e] * bandw_k[e];
  for (int i = 0; i < nb_s; ++i) {
    occ_s[i] = i == 0 ? 1.0 : 0.0;
    bandw_s[i] = i == 0 ? t : 0.0;
  }
}

// dens[r] (+)= w_k sum_n f_n |u_n(r)|^2 (u unnormalised, Omega^-1/2 applied
// by the density finalisation)
__global__ void k_kpt_density(const zc* __restrict__ zk, const double* __restrict__ occ, double wk,
                              int nb, long ntot, double* __restrict__ dens, int first) {
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < ntot; r += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) {
      const zc u = zk[(long)b * ntot + r];
      s += occ[b] * (u.x * u.x + u.y * u.y);
    }
    dens[r] = (first ? 0.0 : dens[r]) + wk * s;
  }
}

// nonlocal forces of one k, accumulated: F_I,a += -2 w_k sum_{p on I} h_p
// sum_n f_n Re[conj(P_pn) dP_pn,a], P = <beta|u>, dP = <-i(k+G) beta|u>
__global__ void k_kpt_force_nl(const zc* __restrict__ P, const zc* __restrict__ dP, int nproj, int nb,
                               const double* __restrict__ h, const int* __restrict__ patom,
                               const double* __restrict__ occ, double wk, int nat,
                               double* __restrict__ fnl, int first) {
  for (int t = threadIdx.x; t < 3 * nat; t += blockDim.x) {
    const int I = t / 3, a = t - 3 * I;
    double f = 0.0;
    for (int p = 0; p < nproj; ++p) {
      if (patom[p] != I) continue;
      double s = 0.0;
      for (int n = 0; n < nb; ++n) {
        const zc pp = P[(size_t)p * nb + n], dd = dP[((size_t)a * nproj + p) * nb + n];
        s += occ[n] * (pp.x * dd.x + pp.y * dd.y);
      }
      f += -2.0 * h[p] * s;
    }
    fnl[t] = (first ? 0.0 : fnl[t]) + wk * f;
  }
}

// total force: local (force_part) + nonlocal + Ewald
__global__ void k_kpt_force_total(const double* __restrict__ floc, const double* __restrict__ fnl,
                                  const double* __restrict__ few, int nat, double* __restrict__ force,
                                  double* __restrict__ fnl_part) {
  for (int t = threadIdx.x; t < 3 * nat; t += blockDim.x) {
    fnl_part[t] = fnl[t];
    force[t] = floc[t] + fnl[t] + few[t];
  }
}

// ---------------------------------------------------------------- launchers
static int nblocks(long n, int per = 256) {
  return (int)std::max(1L, std::min(65536L, (n + per - 1) / per));
}

void kpt_zero(hipStream_t s, zc* a, long n) {
  hipLaunchKernelGGL(k_kpt_zero, dim3(nblocks(n)), dim3(256), 0, s, a, n);
  check_launch("k_kpt_zero");
}

// Inverse (sign +1) or forward (sign -1) 3-D transforms of nb grids
// [nb][N3][N2][N1], axis by axis.
void kpt_fft3(hipStream_t s, zc* zk, int nb, const int N[3], const FftPlan* plans, int sign) {
  const long N1 = N[0], N2 = N[1], N3 = N[2], ntot = N1 * N2 * N3;
  // (lines, A, Bs, Cs, es, plan)
  struct Ax {
    long nlines;
    int A;
    long Bs, Cs, es;
    int ax;
  } axes[3] = {{nb * N3 * N2, 1, N1, 0, 1, 0},
               {nb * N3 * N1, (int)N1, N1 * N2, 1, N1, 1},
               {nb * N2 * N1, (int)(N1 * N2), ntot, 1, N1 * N2, 2}};
  for (const Ax& a : axes) {
    const int n = plans[a.ax].n;
    const int L = std::max(1, 512 / n);
    const size_t lds = (size_t)(2 * L * n + n) * sizeof(zc);
    hipLaunchKernelGGL(k_kpt_lines, dim3((unsigned)((a.nlines + L - 1) / L)), dim3(256), lds, s, zk,
                       plans[a.ax], a.A, a.Bs, a.Cs, a.es, a.nlines, L, sign);
    check_launch("k_kpt_lines");
  }
}

void kpt_hpsi(hipStream_t s, const KptBands& kb, const zc* X, zc* Y, zc* zk, const double* veff,
              const int N[3], const FftPlan* plans, zc* P, const double* h) {
  const long ntot = (long)N[0] * N[1] * N[2];
  kpt_zero(s, zk, (long)kb.nb * ntot);
  hipLaunchKernelGGL(k_kpt_scatter, dim3(nblocks((long)kb.nb * kb.npw)), dim3(256), 0, s, zk, X,
                     kb.box, kb.npw, kb.nb, ntot);
  check_launch("k_kpt_scatter");
  kpt_fft3(s, zk, kb.nb, N, plans, +1);
  hipLaunchKernelGGL(k_kpt_vmul, dim3(nblocks((long)kb.nb * ntot)), dim3(256), 0, s, zk, veff, kb.nb, ntot);
  check_launch("k_kpt_vmul");
  kpt_fft3(s, zk, kb.nb, N, plans, -1);
  hipLaunchKernelGGL(k_kpt_gather, dim3(nblocks((long)kb.nb * kb.npw)), dim3(256), 0, s, zk, X, Y,
                     kb.box, kb.kin, kb.npw, kb.nb, ntot);
  check_launch("k_kpt_gather");
  if (kb.nproj > 0) {
    kpt_zdot(s, kb.beta, kb.nproj, X, kb.nb, kb.npw, P, kb.nb, nullptr, 0);
    kpt_zgemm(s, kb.beta, kb.nproj, P, kb.nb, Y, kb.nb, kb.npw, 1.0, 1.0, h);
  }
}

void kpt_scatter_bands(hipStream_t s, zc* zk, const zc* X, const KptBands& kb, long ntot) {
  hipLaunchKernelGGL(k_kpt_scatter, dim3(nblocks((long)kb.nb * kb.npw)), dim3(256), 0, s, zk, X, kb.box,
                     kb.npw, kb.nb, ntot);
  check_launch("k_kpt_scatter");
}

void kpt_zdot(hipStream_t s, const zc* A, int na, const zc* B, int nbb, int npw, zc* C, int ldc,
              const double* q, int qa) {
  hipLaunchKernelGGL(k_kpt_zdot, dim3((na * nbb + 3) / 4), dim3(256), 0, s, A, na, B, nbb, npw, C, ldc, q, qa);
  check_launch("k_kpt_zdot");
}

void kpt_zgemm(hipStream_t s, const zc* X, int nx, const zc* M, int ldm, zc* Y, int ny, int npw,
               double alpha, double beta, const double* h) {
  hipLaunchKernelGGL(k_kpt_zgemm, dim3(nblocks((long)ny * npw)), dim3(256), 0, s, X, nx, M, ldm, Y, ny,
                     npw, alpha, beta, h);
  check_launch("k_kpt_zgemm");
}

void kpt_copy(hipStream_t s, zc* dst, const zc* src, long n) {
  hipLaunchKernelGGL(k_kpt_copy, dim3(nblocks(n)), dim3(256), 0, s, dst, src, n);
  check_launch("k_kpt_copy");
}

void kpt_beta(hipStream_t s, const KptBands& kb, const int* patom, const int* plm, const double* pr,
              const double* pos, double omega) {
  if (kb.nproj == 0) return;
  hipLaunchKernelGGL(k_kpt_beta, dim3(nblocks(kb.npw), kb.nproj), dim3(256), 0, s, kb.beta, kb.q, kb.npw,
                     kb.nproj, patom, plm, pr, pos, omega);
  check_launch("k_kpt_beta");
}

void kpt_subspace(hipStream_t s, zc* S, zc* H, zc* W, zc* V, zc* M, double* eps, int n, int mode,
                  int* fail) {
  hipLaunchKernelGGL(k_kpt_subspace, dim3(1), dim3(256), 0, s, S, H, W, V, M, eps, n, mode, fail);
  check_launch("k_kpt_subspace");
}

void kpt_cg_dir(hipStream_t s, const KptBands& kb, const zc* X, const zc* HX, zc* D, const double* eps,
                double* gam, int first) {
  hipLaunchKernelGGL(k_kpt_cg_dir, dim3(kb.nb), dim3(256), 0, s, X, HX, D, kb.kin, eps, gam, kb.npw, first);
  check_launch("k_kpt_cg_dir");
}

void kpt_linemin(hipStream_t s, const KptBands& kb, zc* X, zc* HX, const zc* D, const zc* HD) {
  hipLaunchKernelGGL(k_kpt_linemin, dim3(kb.nb), dim3(256), 0, s, X, HX, D, HD, kb.npw);
  check_launch("k_kpt_linemin");
}

void kpt_init(hipStream_t s, const KptBands& kb, zc* X, unsigned seed, int kidx) {
  hipLaunchKernelGGL(k_kpt_init, dim3(nblocks((long)kb.nb * kb.npw)), dim3(256), 0, s, X, kb.kin, kb.npw,
                     kb.nb, seed, kidx);
  check_launch("k_kpt_init");
}

void kpt_occupations(hipStream_t s, const double* eps, const double* wk, int nk, int nb, double nelec,
                     int kind, double sigma, double* occ, double* scal) {
  hipLaunchKernelGGL(k_kpt_occupations, dim3(1), dim3(64), 0, s, eps, wk, nk, nb, nelec, kind, sigma, occ,
                     scal);
  check_launch("k_kpt_occupations");
}

void kpt_band_kinetic(hipStream_t s, const KptBands& kb, const zc* X, double* out) {
  hipLaunchKernelGGL(k_kpt_band_kinetic, dim3(kb.nb), dim3(256), 0, s, X, kb.kin, kb.npw, out);
  check_launch("k_kpt_band_kinetic");
}

void kpt_kinetic_total(hipStream_t s, const double* bandw_k, const double* occ_k, const double* wk, int nk,
                       int nb, double* occ_s, double* bandw_s, int nb_s) {
  hipLaunchKernelGGL(k_kpt_kinetic_total, dim3(1), dim3(64), 0, s, bandw_k, occ_k, wk, nk, nb, occ_s,
                     bandw_s, nb_s);
  check_launch("k_kpt_kinetic_total");
}

void kpt_density(hipStream_t s, const zc* zk, const double* occ, double wk, int nb, long ntot, double* dens,
                 int first) {
  hipLaunchKernelGGL(k_kpt_density, dim3(nblocks(ntot)), dim3(256), 0, s, zk, occ, wk, nb, ntot, dens, first);
  check_launch("k_kpt_density");
}

void kpt_force_nl(hipStream_t s, const zc* P, const zc* dP, int nproj, int nb, const double* h,
                  const int* patom, const double* occ, double wk, int nat, double* fnl, int first) {
  hipLaunchKernelGGL(k_kpt_force_nl, dim3(1), dim3(256), 0, s, P, dP, nproj, nb, h, patom, occ, wk, nat,
                     fnl, first);
  check_launch("k_kpt_force_nl");
}

void kpt_force_total(hipStream_t s, const double* floc, const double* fnl, const double* few, int nat,
                     double* force, double* fnl_part) {
  hipLaunchKernelGGL(k_kpt_force_total, dim3(1), dim3(256), 0, s, floc, fnl, few, nat, force, fnl_part);
  check_launch("k_kpt_force_total");
}

void configure_kpt_kernels() { allow_lds((const void*)k_kpt_lines); }

}  // namespace sgo
