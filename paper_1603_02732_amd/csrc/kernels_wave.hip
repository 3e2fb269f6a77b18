// Wavefunction-side kernels, templated on the bulk precision T.
//
//  * H|psi> (the H psi steps of Algorithm 1): Gamma-point
//    two-bands-per-FFT packing, sphere-pruned z transforms on the occupied
//    stick pairs, a fused per-plane kernel (inverse 2-D FFT, multiply by
//    V_eff(r), forward 2-D FFT) and a gather that unpacks the two bands and
//    adds the kinetic term; projector products for the nonlocal part.
//  * density planes (output charge density of the SCF step, Section 2.4).
//  * split-K Gram products and in-place rotations (the subspace and
//    projection steps of Algorithm 1), FP64 accumulation.
//  * per-band CG kernels: residual + preconditioning + CG direction, and the
//    line minimisation over the angle theta.
//  * the FP64 subspace solver: Cholesky orthonormalisation and Jacobi
//    diagonalisation of the subspace Hamiltonian.
#include "device.hpp"
#include "launch.hpp"

#include <type_traits>

#include <algorithm>

namespace sgo {

template <typename T>
__device__ __forceinline__ T* warr(const CandDesc& c, int w) {
  switch (w) {
    case W_X: return (T*)c.X;
    case W_HX: return (T*)c.HX;
    case W_D: return (T*)c.D;
    case W_HD: return (T*)c.HD;
    default: return (T*)c.beta;
  }
}
__device__ __forceinline__ int wrows(const CandDesc& c, int w) { return w == W_BETA ? c.nproj : c.nb; }
__device__ __forceinline__ double* marr(const CandDesc& c, int m) {
  switch (m) {
    case M_S: return c.S;
    case M_H: return c.Hs;
    case M_M: return c.M;
    default: return c.C;
  }
}

__device__ __forceinline__ int mirror_stick(int s) { return s == 0 ? 0 : ((s & 1) ? s + 1 : s - 1); }

// ------------------------------------------------------------ z transforms
// Scatter band pair (2p, 2p+1) of the half sphere into its stick pairs
// (c_{-G} = conj c_G fills the mirror stick) and inverse-transform along z.
// Output layout: sticks[pair][z][stick] (z-major, so the plane kernel reads
// one contiguous row per plane).
template <typename T>
__global__ void __launch_bounds__(kNT) k_z_inverse(const CandDesc* __restrict__ cds, int src,
                                                   int sp_chunk) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int pair = blockIdx.y;
  const int q0 = blockIdx.x * sp_chunk;
  if (pair >= cd.npair || q0 >= cd.nsp) return;
  const int q1 = min(q0 + sp_chunk, cd.nsp);
  const int s0 = q0 == 0 ? 0 : 2 * q0 - 1;
  const int s1 = 2 * q1 - 1;
  const int nloc = s1 - s0;
  const int N3 = cd.N3;
  const int tid = threadIdx.x, nthr = blockDim.x;
  extern __shared__ __align__(16) char smem[];
  cplx<T>* tw = (cplx<T>*)smem;
  cplx<T>* A = tw + kMaxFftN;
  cplx<T>* Bf = A + nloc * N3;
  fill_twiddles(tw, N3, tid, nthr);
  for (int e = tid; e < nloc * N3; e += nthr) A[e] = {(T)0, (T)0};
  __syncthreads();
  const T* base = warr<T>(cd, src);
  const T* xa = base + (size_t)(2 * pair) * cd.Kp;
  const bool hasb = 2 * pair + 1 < cd.nb;
  const T* xb = base + (size_t)(2 * pair + 1) * cd.Kp;
  const int g0 = cd.sp_off[q0], g1 = cd.sp_off[q1];
  for (int g = g0 + tid; g < g1; g += nthr) {
    const int meta = cd.gmeta[g];
    const int s = meta & 0xFFFFF, z = meta >> 20;
    cplx<T> ca = unpack_coef(xa, g);
    cplx<T> cb = hasb ? unpack_coef(xb, g) : cplx<T>{(T)0, (T)0};
    A[(s - s0) * N3 + z] = {ca.x - cb.y, ca.y + cb.x};  // c_a + i c_b
    if (g != 0) {
      const int sm = mirror_stick(s);
      const int zm = z == 0 ? 0 : N3 - z;
      A[(sm - s0) * N3 + zm] = {ca.x + cb.y, cb.x - ca.y};  // conj c_a + i conj c_b
    }
  }
  __syncthreads();
  cplx<T>* r = lds_fft(A, Bf, cd.plan[2], nloc, 1, N3, tw, +1, tid, nthr);
  cplx<T>* out = (cplx<T>*)cd.sticks + (size_t)pair * N3 * cd.nst;
  for (int t = tid; t < nloc * N3; t += nthr) {
    const int z = t / nloc, s = t - z * nloc;
    out[(size_t)z * cd.nst + s0 + s] = r[s * N3 + z];
  }
}

// Forward z transform of the stick pairs and gather back to the half
// sphere: split the pair by Hermitian symmetry, scale 1/Ntot, add the
// kinetic term |G|^2/2 psi, write H psi in the packed layout.
template <typename T>
__global__ void __launch_bounds__(kNT) k_z_forward(const CandDesc* __restrict__ cds, int src,
                                                   int dst, int sp_chunk) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int pair = blockIdx.y;
  const int q0 = blockIdx.x * sp_chunk;
  if (pair >= cd.npair || q0 >= cd.nsp) return;
  const int q1 = min(q0 + sp_chunk, cd.nsp);
  const int s0 = q0 == 0 ? 0 : 2 * q0 - 1;
  const int s1 = 2 * q1 - 1;
  const int nloc = s1 - s0;
  const int N3 = cd.N3;
  const int tid = threadIdx.x, nthr = blockDim.x;
  extern __shared__ __align__(16) char smem[];
  cplx<T>* tw = (cplx<T>*)smem;
  cplx<T>* A = tw + kMaxFftN;
  cplx<T>* Bf = A + nloc * N3;
  fill_twiddles(tw, N3, tid, nthr);
  const cplx<T>* in = (const cplx<T>*)cd.sticks + (size_t)pair * N3 * cd.nst;
  for (int t = tid; t < nloc * N3; t += nthr) {
    const int z = t / nloc, s = t - z * nloc;
    A[s * N3 + z] = in[(size_t)z * cd.nst + s0 + s];
  }
  __syncthreads();
  cplx<T>* r = lds_fft(A, Bf, cd.plan[2], nloc, 1, N3, tw, -1, tid, nthr);
  const T sc = (T)(1.0 / (double)cd.ntot);
  const T rt2 = (T)1.41421356237309504880;
  const T* xsrc = warr<T>(cd, src);
  T* ydst = warr<T>(cd, dst);
  const int a = 2 * pair, b = 2 * pair + 1;
  const bool hasb = b < cd.nb;
  const T* xa = xsrc + (size_t)a * cd.Kp;
  const T* xb = xsrc + (size_t)b * cd.Kp;
  T* ya = ydst + (size_t)a * cd.Kp;
  T* yb = ydst + (size_t)b * cd.Kp;
  const int g0 = cd.sp_off[q0], g1 = cd.sp_off[q1];
  for (int g = g0 + tid; g < g1; g += nthr) {
    const int meta = cd.gmeta[g];
    const int s = meta & 0xFFFFF, z = meta >> 20;
    const int sm = mirror_stick(s);
    const int zm = z == 0 ? 0 : N3 - z;
    cplx<T> W = r[(s - s0) * N3 + z];
    cplx<T> Wm = r[(sm - s0) * N3 + zm];
    // (V psi_a)_G = (W_G + conj W_-G)/2 ; (V psi_b)_G = (W_G - conj W_-G)/(2i)
    cplx<T> va = {(T)0.5 * (W.x + Wm.x) * sc, (T)0.5 * (W.y - Wm.y) * sc};
    cplx<T> vb = {(T)0.5 * (W.y + Wm.y) * sc, (T)-0.5 * (W.x - Wm.x) * sc};
    const T kin = (T)cd.kin[g];
    if (g == 0) {
      ya[0] = va.x + kin * xa[0];
      ya[1] = (T)0;
      if (hasb) {
        yb[0] = vb.x + kin * xb[0];
        yb[1] = (T)0;
      }
    } else {
      ya[2 * g] = rt2 * va.x + kin * xa[2 * g];
      ya[2 * g + 1] = rt2 * va.y + kin * xa[2 * g + 1];
      if (hasb) {
        yb[2 * g] = rt2 * vb.x + kin * xb[2 * g];
        yb[2 * g + 1] = rt2 * vb.y + kin * xb[2 * g + 1];
      }
    }
  }
}

// ------------------------------------------------------------ plane kernels
// One z-plane of one band pair: gather the stick values, inverse 2-D FFT,
// multiply by V_eff(r), forward 2-D FFT, scatter back to the sticks.
template <typename T>
__global__ void __launch_bounds__(kNT) k_plane_hpsi(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int z = blockIdx.x, pair = blockIdx.y;
  if (z >= cd.N3 || pair >= cd.npair) return;
  const int N1 = cd.N1, N2 = cd.N2, NP = N1 * N2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  extern __shared__ __align__(16) char smem[];
  cplx<T>* tw1 = (cplx<T>*)smem;
  cplx<T>* tw2 = tw1 + kMaxFftN;
  cplx<T>* A = tw2 + kMaxFftN;
  cplx<T>* Bf = A + NP;
  fill_twiddles(tw1, N1, tid, nthr);
  fill_twiddles(tw2, N2, tid, nthr);
  for (int e = tid; e < NP; e += nthr) A[e] = {(T)0, (T)0};
  __syncthreads();
  cplx<T>* st = (cplx<T>*)cd.sticks + ((size_t)pair * cd.N3 + z) * cd.nst;
  for (int s = tid; s < cd.nst; s += nthr) {
    const int xy = cd.stick_xy[s];
    A[(xy >> 16) * N1 + (xy & 0xFFFF)] = st[s];
  }
  __syncthreads();
  cplx<T>* r = lds_fft(A, Bf, cd.plan[1], N1, N1, 1, tw2, +1, tid, nthr);  // along y
  cplx<T>* o = r == A ? Bf : A;
  r = lds_fft(r, o, cd.plan[0], N2, 1, N1, tw1, +1, tid, nthr);            // along x
  const T* V = (const T*)cd.veff_t + (size_t)z * NP;
  for (int e = tid; e < NP; e += nthr) {
    const T v = V[e];
    r[e].x *= v;
    r[e].y *= v;
  }
  __syncthreads();
  o = r == A ? Bf : A;
  r = lds_fft(r, o, cd.plan[0], N2, 1, N1, tw1, -1, tid, nthr);
  o = r == A ? Bf : A;
  r = lds_fft(r, o, cd.plan[1], N1, N1, 1, tw2, -1, tid, nthr);
  for (int s = tid; s < cd.nst; s += nthr) {
    const int xy = cd.stick_xy[s];
    st[s] = r[(xy >> 16) * N1 + (xy & 0xFFFF)];
  }
}

// Density of one z-plane summed over a chunk of band pairs:
// part[chunk][z][y][x] = sum_pairs f_a Re(u)^2 + f_b Im(u)^2, u = psi_a + i psi_b
// (unnormalised transforms; the 1/Omega is applied when chunks are summed).
constexpr int kDensRegs = 48;
template <typename T>
__global__ void __launch_bounds__(kNT) k_plane_density(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int z = blockIdx.x, chunk = blockIdx.y;
  if (z >= cd.N3 || chunk >= cd.ndens_chunk) return;
  const int N1 = cd.N1, N2 = cd.N2, NP = N1 * N2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  extern __shared__ __align__(16) char smem[];
  cplx<T>* tw1 = (cplx<T>*)smem;
  cplx<T>* tw2 = tw1 + kMaxFftN;
  cplx<T>* A = tw2 + kMaxFftN;
  cplx<T>* Bf = A + NP;
  fill_twiddles(tw1, N1, tid, nthr);
  fill_twiddles(tw2, N2, tid, nthr);
  double acc[kDensRegs];
#pragma unroll
  for (int k = 0; k < kDensRegs; ++k) acc[k] = 0.0;
  const int per = (cd.npair + cd.ndens_chunk - 1) / cd.ndens_chunk;
  const int p0 = chunk * per, p1 = min(cd.npair, p0 + per);
  for (int pair = p0; pair < p1; ++pair) {
    for (int e = tid; e < NP; e += nthr) A[e] = {(T)0, (T)0};
    __syncthreads();
    const cplx<T>* st = (const cplx<T>*)cd.sticks + ((size_t)pair * cd.N3 + z) * cd.nst;
    for (int s = tid; s < cd.nst; s += nthr) {
      const int xy = cd.stick_xy[s];
      A[(xy >> 16) * N1 + (xy & 0xFFFF)] = st[s];
    }
    __syncthreads();
    cplx<T>* r = lds_fft(A, Bf, cd.plan[1], N1, N1, 1, tw2, +1, tid, nthr);
    cplx<T>* o = r == A ? Bf : A;
    r = lds_fft(r, o, cd.plan[0], N2, 1, N1, tw1, +1, tid, nthr);
    const double fa = cd.occ[2 * pair];
    const double fb = 2 * pair + 1 < cd.nb ? cd.occ[2 * pair + 1] : 0.0;
#pragma unroll
    for (int k = 0; k < kDensRegs; ++k) {
      const int e = tid + k * nthr;
      if (e < NP) {
        const double ux = (double)r[e].x, uy = (double)r[e].y;
        acc[k] += fa * ux * ux + fb * uy * uy;
      }
    }
    __syncthreads();
  }
  double* out = cd.dens_part + (size_t)chunk * cd.ntot + (size_t)z * NP;
#pragma unroll
  for (int k = 0; k < kDensRegs; ++k) {
    const int e = tid + k * nthr;
    if (e < NP) out[e] = acc[k];
  }
}

// ------------------------------------------------ MFMA subspace products
// FP64 matrix-core products (v_mfma_f64_16x16x4f64): operands are the band
// arrays converted to FP64 (exact for FP32 data), accumulation in FP64.
// Fragment layout of one 16x16x4 step, lane l = 16 g + r16 (g = l / 16):
//   A operand: A[r16][g],  B operand: B[g][r16],  result register r: D[4 r + g][r16].
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load4(const float* p, bool ok, double* v) {
  if (ok) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    v[0] = f.x;
    v[1] = f.y;
    v[2] = f.z;
    v[3] = f.w;
  } else {
    v[0] = v[1] = v[2] = v[3] = 0.0;
  }
}
__device__ __forceinline__ void load4(const double* p, bool ok, double* v) {
  if (ok) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
  } else {
    v[0] = v[1] = v[2] = v[3] = 0.0;
  }
}

__device__ __forceinline__ void load4(const float* p, bool ok, float* v) {
  if (ok) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
  } else {
    v[0] = v[1] = v[2] = v[3] = 0.f;
  }
}
typedef float gfloatx4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;
// Split-K Gram product out[i][j] = sum_k A[i][k] B[j][k] for up to two
// products per launch.  A block covers one (16 TB)^2 output tile over one K
// range; its four wavefronts take interleaved 16-wide K steps (the loads of
// the next step are issued before the MFMAs of the current one), each lane
// loading four consecutive reals of one row (the four MFMAs of a step use
// one element each, the same k permutation for both operands).  Waves are
// summed in LDS; each block writes the valid part of its tile to a partial
// buffer that k_gram_reduce sums in K order.  Rows past the band count are
// zero.  F32 = true (FP32 data only): FP32 MFMA with FP32 accumulation over
// each wavefront's share of the K range (at most kc_len/4 terms); the waves,
// blocks and K ranges are still summed in FP64.
constexpr int kGramDepth = 2;  // 16-wide K steps in flight per wave (FP32 data)

template <typename T, int TB, bool F32 = false>
__global__ void __launch_bounds__(kNT) k_gram(const CandDesc* __restrict__ cds, int kc_len,
                                              int nkc_max, int a0, int b0, int a1, int b1) {
  using AT = typename std::conditional<F32, float, double>::type;
  using ACC = typename std::conditional<F32, gfloatx4, dbl4>::type;
  constexpr int TT = 16 * TB;
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int prod = blockIdx.y;
  const int wa = prod ? a1 : a0, wb = prod ? b1 : b0;
  const int na = wrows(cd, wa), nbb = wrows(cd, wb);
  if (na == 0 || nbb == 0) return;
  const int nti = (na + TT - 1) / TT, ntj = (nbb + TT - 1) / TT;
  const int nkc = (cd.K + kc_len - 1) / kc_len;
  const int kc = blockIdx.x % nkc_max;
  const int tile = blockIdx.x / nkc_max;
  if (kc >= nkc || tile >= nti * ntj) return;
  const int ti = tile / ntj, tj = tile - ti * ntj;
  const T* Am = warr<T>(cd, wa);
  const T* Bm = warr<T>(cd, wb);
  const int Kp = cd.Kp;
  const int k0 = kc * kc_len, k1 = min(cd.K, k0 + kc_len);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int BI = min(TB, (na - ti * TT + 15) / 16), BJ = min(TB, (nbb - tj * TT + 15) / 16);
  __shared__ double tileS[TT * TT];
  for (int e = threadIdx.x; e < TT * TT; e += blockDim.x) tileS[e] = 0.0;
  ACC acc[TB][TB];
#pragma unroll
  for (int u = 0; u < TB; ++u)
#pragma unroll
    for (int v = 0; v < TB; ++v) acc[u][v] = ACC{0, 0, 0, 0};
  const T* pa[TB];
  const T* pb[TB];
  bool oka[TB], okb[TB];
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    const int ra = ti * TT + u * 16 + r16, rb = tj * TT + u * 16 + r16;
    oka[u] = u < BI && ra < na;
    okb[u] = u < BJ && rb < nbb;
    pa[u] = Am + (size_t)(oka[u] ? ra : 0) * Kp + 4 * g;
    pb[u] = Bm + (size_t)(okb[u] ? rb : 0) * Kp + 4 * g;
  }
  // Each wave takes the 16-wide K steps ks, ks + 64, ... of the chunk; kGramDepth
  // of them per iteration, with the loads of the next kGramDepth issued before
  // the MFMAs of the current ones (more loads in flight per wave).
  constexpr int D = sizeof(T) == 4 ? kGramDepth : 1;  // FP64 data: registers bound
  T a[D][TB][4], b[D][TB][4];  // storage type; widened at the MFMA
  int ks = k0 + wave * 16;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int kk = ks + 64 * d;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      load4(pa[u] + kk, oka[u] && kk < k1, a[d][u]);
      load4(pb[u] + kk, okb[u] && kk < k1, b[d][u]);
    }
  }
  while (ks < k1) {
    const int kn = ks + 64 * D;
    T an[D][TB][4], bn[D][TB][4];
    if (kn < k1) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int kk = kn + 64 * d;
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          load4(pa[u] + kk, oka[u] && kk < k1, an[d][u]);
          load4(pb[u] + kk, okb[u] && kk < k1, bn[d][u]);
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (ks + 64 * d >= k1) break;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < TB; ++u)
#pragma unroll
          for (int v = 0; v < TB; ++v)
            if (u < BI && v < BJ) {
              if constexpr (F32)
                acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32((AT)a[d][u][t], (AT)b[d][v][t], acc[u][v], 0, 0, 0);
              else
                acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64((AT)a[d][u][t], (AT)b[d][v][t], acc[u][v], 0, 0, 0);
            }
    }
    if (kn < k1) {
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int u = 0; u < TB; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            a[d][u][t] = an[d][u][t];
            b[d][u][t] = bn[d][u][t];
          }
    }
    ks = kn;
  }
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int u = 0; u < TB; ++u)
#pragma unroll
        for (int v = 0; v < TB; ++v)
          if (u < BI && v < BJ)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              // result register r: row 4r + g (f64 16x16x4), row 4g + r (f32 16x16x4)
              const int row = F32 ? 4 * g + r : 4 * r + g;
              tileS[(u * 16 + row) * TT + v * 16 + r16] += (double)acc[u][v][r];
            }
    }
    __syncthreads();
  }
  // valid part of the tile -> partial buffer [prod][tile][kc][rows][cols]
  const int rows = min(TT, na - ti * TT), cols = min(TT, nbb - tj * TT);
  const size_t tile_sz = (size_t)TT * TT;
  double* part = cd.red_part + (((size_t)prod * nti * ntj + tile) * nkc + kc) * tile_sz;
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
    const int rr = e / cols, cc = e - rr * cols;
    part[e] = tileS[rr * TT + cc];
  }
}

// Sum of the split-K partial tiles in K order: one thread per output entry.
template <int TB>
__global__ void __launch_bounds__(kNT) k_gram_reduce(const CandDesc* __restrict__ cds, int kc_len,
                                                     int a0, int b0, int o0, int a1, int b1,
                                                     int o1) {
  constexpr int TT = 16 * TB;
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int prod = blockIdx.y;
  const int wa = prod ? a1 : a0, wb = prod ? b1 : b0, wo = prod ? o1 : o0;
  const int na = wrows(cd, wa), nbb = wrows(cd, wb);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= na * nbb) return;
  const int i = e / nbb, j = e - i * nbb;
  const int nti = (na + TT - 1) / TT, ntj = (nbb + TT - 1) / TT;
  const int ti = i / TT, tj = j / TT;
  const int tile = ti * ntj + tj;
  const int rows = min(TT, na - ti * TT), cols = min(TT, nbb - tj * TT);
  (void)rows;
  const int nkc = (cd.K + kc_len - 1) / kc_len;
  const size_t tile_sz = (size_t)TT * TT;
  const double* part = cd.red_part + ((size_t)prod * nti * ntj + tile) * nkc * tile_sz +
                       (i - ti * TT) * cols + (j - tj * TT);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = 0;
  for (; c + 3 < nkc; c += 4) {
    s0 += part[(size_t)c * tile_sz];
    s1 += part[(size_t)(c + 1) * tile_sz];
    s2 += part[(size_t)(c + 2) * tile_sz];
    s3 += part[(size_t)(c + 3) * tile_sz];
  }
  for (; c < nkc; ++c) s0 += part[(size_t)c * tile_sz];
  marr(cd, wo)[(size_t)i * nbb + j] = (s0 + s1) + (s2 + s3);
}

// Band-space product on 64-column slices:
//   Y[i][k] = alpha Y[i][k] + beta sum_j w_j M[j][i] A[j][k]   (i < nout, j < nin)
// w_j = h_j (projector energies) when use_h, else 1.  Each block owns all
// rows of its 64 columns, so Y may alias A (in-place rotation): the block
// reads every A row of its slice (through LDS, 32 rows at a time) before it
// writes.  Wave w holds the output rows 16 (w + 4 m) .. +16, m < IBW.
constexpr int kJC = 32;
template <typename T, int IBW>
__global__ void __launch_bounds__(kNT) k_gemm_acc(const CandDesc* __restrict__ cds, int y0, int y1,
                                                  int y2, int a0, int a1, int a2, int mat,
                                                  double alpha, double beta, int use_h) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int arr = blockIdx.y;
  const int wy = arr == 0 ? y0 : (arr == 1 ? y1 : y2);
  const int wa = arr == 0 ? a0 : (arr == 1 ? a1 : a2);
  const int nin = wrows(cd, wa), nout = wrows(cd, wy);
  if (nin == 0) return;
  const int Kp = cd.Kp;
  const int kbase = blockIdx.x * 64;
  if (kbase >= cd.K) return;
  const T* A = warr<T>(cd, wa);
  T* Y = warr<T>(cd, wy);
  const double* M = marr(cd, mat);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int nib = (nout + 15) / 16;
  extern __shared__ __align__(16) char smem[];
  double* As = (double*)smem;            // [kJC][64]
  double* Ms = As + kJC * 64;            // [kJC][nib*16]
  const int ldm = nib * 16;
  dbl4 acc[IBW][4];
#pragma unroll
  for (int m = 0; m < IBW; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[m][v] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < nin; j0 += kJC) {
    __syncthreads();
    for (int e = threadIdx.x; e < kJC * 64; e += blockDim.x) {
      const int jj = e >> 6, kk = e & 63;
      const int j = j0 + jj, k = kbase + kk;
      As[e] = (j < nin && k < Kp) ? (double)A[(size_t)j * Kp + k] : 0.0;
    }
    for (int e = threadIdx.x; e < kJC * ldm; e += blockDim.x) {
      const int jj = e / ldm, i = e - jj * ldm;
      const int j = j0 + jj;
      double m = 0.0;
      if (j < nin && i < nout) {
        m = M[(size_t)j * nout + i];
        if (use_h) m *= cd.hproj[j];
      }
      Ms[e] = m;
    }
    __syncthreads();
#pragma unroll
    for (int j4 = 0; j4 < kJC / 4; ++j4) {
      const int jr = 4 * j4 + g;
      double bop[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) bop[v] = As[jr * 64 + v * 16 + r16];
#pragma unroll
      for (int m = 0; m < IBW; ++m) {
        const int ib = wave + 4 * m;
        if (ib < nib) {
          const double aop = Ms[jr * ldm + ib * 16 + r16];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[m][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[v], acc[m][v], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();  // every read of A in this slice precedes the writes
#pragma unroll
  for (int m = 0; m < IBW; ++m) {
    const int ib = wave + 4 * m;
    if (ib >= nib) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = kbase + v * 16 + r16;
      if (k >= cd.K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ib * 16 + 4 * r + g;
        if (i >= nout) continue;
        const size_t idx = (size_t)i * Kp + k;
        const double yo = alpha != 0.0 ? (double)Y[idx] : 0.0;
        Y[idx] = (T)(alpha * yo + beta * acc[m][v][r]);
      }
    }
  }
}

// FP32 band products on MFMA (FP32 bulk path):
//   Y[i][k] = alpha Y[i][k] + beta sum_j M'[j][i] A[j][k],  M' = M or h_j M,
// with v_mfma_f32_16x16x4f32 and FP32 accumulation.  One wavefront per
// 64-column slice of every output row; the A slice (nin x 64) is staged in
// LDS before any store, so Y may alias A (in-place rotation).  Column n of
// MFMA tile c is k = k0 + 4n + c: a lane's float4 of a band row is then its
// B operand for the four column tiles, and each result row leaves as one
// float4 per lane.
typedef float floatx4 __attribute__((ext_vector_type(4)));
// TT: 16-row output tiles per pass (2 when every output has at most 32 rows:
// half the accumulator registers, more resident waves).  NW wavefronts
// share one staged slice and take turns over the output row tiles: with
// many bands the slice fills most of the LDS a compute unit has, and a
// single wavefront per slice would leave the matrix cores idle.
template <int TT, int NW>
__global__ void __launch_bounds__(64 * NW) k_gemm_f32(const CandDesc* __restrict__ cds, int y0,
                                                      int y1, int y2, int a0, int a1, int a2,
                                                      int mat, float alpha, float beta, int use_h) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int arr = blockIdx.y;
  const int wy = arr == 0 ? y0 : (arr == 1 ? y1 : y2);
  const int wa = arr == 0 ? a0 : (arr == 1 ? a1 : a2);
  const int nin = wrows(cd, wa), nout = wrows(cd, wy);
  if (nin == 0) return;
  const int Kp = cd.Kp;
  const int k0 = blockIdx.x * 64;
  if (k0 >= cd.K) return;
  const float* A = warr<float>(cd, wa);
  float* Y = warr<float>(cd, wy);
  const double* M = marr(cd, mat);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  const int kc = k0 + 4 * n;          // first of this lane's four columns
  const bool kin = kc < Kp;           // Kp is a multiple of 32: all four or none
  extern __shared__ __align__(16) char smem[];
  float4* As = (float4*)smem;         // [nin][16] float4 = [nin][64] floats
  // staged in batches of 8 rows per thread: the loads of a batch are all in
  // flight before the first store (one memory latency per batch)
  const int gs = threadIdx.x >> 4, ng = 4 * NW;  // row group of this thread, groups
  for (int jb = gs; jb < nin; jb += 8 * ng) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + ng * u;
      v[u] = (kin && j < nin) ? *(const float4*)(A + (size_t)j * Kp + kc)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + ng * u;
      if (j < nin) As[j * 16 + n] = v[u];
    }
  }
  __syncthreads();
  for (int i0 = 16 * TT * wave; i0 < nout; i0 += 16 * TT * NW) {
    floatx4 acc[TT][4];
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    // four 4-deep steps per pass: their M loads (global, FP64) and LDS
    // loads are all issued before the first product, so a pass waits for
    // one load latency instead of four
    for (int j00 = 0; j00 < nin; j00 += 16) {
      float4 b[4];
      float a[4][TT];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j00 + 4 * u + g;
        b[u] = j < nin ? As[j * 16 + n] : make_float4(0.f, 0.f, 0.f, 0.f);
        const double hj = (use_h && j < nin) ? cd.hproj[j] : 1.0;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const int i = i0 + 16 * t + n;
          a[u][t] = (j < nin && i < nout) ? (float)(hj * M[(size_t)j * nout + i]) : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          if (i0 + 16 * t >= nout) break;
          acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][t], b[u].x, acc[t][0], 0, 0, 0);
          acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][t], b[u].y, acc[t][1], 0, 0, 0);
          acc[t][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][t], b[u].z, acc[t][2], 0, 0, 0);
          acc[t][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][t], b[u].w, acc[t][3], 0, 0, 0);
        }
    }
    if (!kin) continue;
#pragma unroll
    for (int t = 0; t < TT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * t + 4 * g + r;
        if (i >= nout) continue;
        float4* yp = (float4*)(Y + (size_t)i * Kp + kc);
        float4 o = make_float4(beta * acc[t][0][r], beta * acc[t][1][r], beta * acc[t][2][r],
                               beta * acc[t][3][r]);
        if (alpha != 0.f) {
          const float4 q = *yp;
          o.x += alpha * q.x;
          o.y += alpha * q.y;
          o.z += alpha * q.z;
          o.w += alpha * q.w;
        }
        *yp = o;
      }
    }
  }
}

// ------------------------------------------------------------- band kernels
// Teter-Payne-Allan preconditioner K(x), x = (|G|^2/2) / E_kin(band).
__device__ __forceinline__ double tpa(double x) {
  const double p = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
  return p / (p + 16.0 * x * x * x * x);
}

// Residual R = H psi - eps psi, preconditioned g = K R, CG direction
// D = g + beta D_prev with beta = <g,R>_k / <g,R>_{k-1} (first step: D = g).
template <typename T>
__global__ void __launch_bounds__(kNT) k_cg_direction(const CandDesc* __restrict__ cds, int first) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16 * 2];
  const int K = cd.K;
  const T* x = (const T*)cd.X + (size_t)i * cd.Kp;
  const T* hx = (const T*)cd.HX + (size_t)i * cd.Kp;
  T* d = (T*)cd.D + (size_t)i * cd.Kp;
  double v1[1] = {0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double xv = (double)x[k];
    v1[0] += cd.kin[k >> 1] * xv * xv;
  }
  block_sum<1>(v1, sh);
  const double ek = fmax(v1[0], 1e-8);
  const double e = cd.eps[i];
  double v2[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double r = (double)hx[k] - e * (double)x[k];
    const double g = tpa(cd.kin[k >> 1] / ek) * r;
    v2[0] += g * r;
    v2[1] += r * r;
  }
  block_sum<2>(v2, sh);
  const double gam = v2[0];
  if (threadIdx.x == 0) cd.resn[i] = v2[1];
  double beta = 0.0;
  if (!first) {
    const double gp = cd.gam[i];
    beta = gp > 0.0 ? gam / gp : 0.0;
  }
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double r = (double)hx[k] - e * (double)x[k];
    const double g = tpa(cd.kin[k >> 1] / ek) * r;
    d[k] = (T)(g + (first ? 0.0 : beta * (double)d[k]));
  }
  if (threadIdx.x == 0) cd.gam[i] = gam;
}

// Line minimisation of each band along its (projected) direction d:
// psi(theta) = x cos(theta) + d/|d| sin(theta), exact minimiser of the 2x2
// Rayleigh quotient at fixed H; H psi is updated with H d (no extra H apply).
template <typename T>
__global__ void __launch_bounds__(kNT) k_linemin(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16 * 4];
  const int K = cd.K;
  T* x = (T*)cd.X + (size_t)i * cd.Kp;
  T* hx = (T*)cd.HX + (size_t)i * cd.Kp;
  const T* d = (const T*)cd.D + (size_t)i * cd.Kp;
  const T* hd = (const T*)cd.HD + (size_t)i * cd.Kp;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double xv = x[k], hxv = hx[k], dv = d[k], hdv = hd[k];
    v[0] += xv * hxv;
    v[1] += xv * hdv;
    v[2] += dv * hdv;
    v[3] += dv * dv;
  }
  block_sum<4>(v, sh);
  const double n2 = v[3];
  if (!(n2 > 0.0)) return;
  const double inv = 1.0 / sqrt(n2);
  const double a = v[0], b = v[1] * inv, c = v[2] * inv * inv;
  const double theta = 0.5 * atan2(-2.0 * b, c - a);
  double sn, cs;
  sincos(theta, &sn, &cs);
  const double sd = sn * inv;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    x[k] = (T)(cs * (double)x[k] + sd * (double)d[k]);
    hx[k] = (T)(cs * (double)hx[k] + sd * (double)hd[k]);
  }
}

// FP32 variants of the CG direction and the line minimisation that read each
// band array once: one 512-thread block per band holds the band's values in
// float4 registers (J per thread and array, Kp <= 2048 J) between the
// reductions and the update.
constexpr int kBandNT = 512;
template <int J>
__device__ __forceinline__ void load_band4(const float* __restrict__ a, int Kp, float4 (&r)[J]) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = threadIdx.x + kBandNT * j;
    r[j] = 4 * c < Kp ? reinterpret_cast<const float4*>(a)[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}
template <int J>
__device__ __forceinline__ void store_band4(float* __restrict__ a, int Kp, const float4 (&r)[J]) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = threadIdx.x + kBandNT * j;
    if (4 * c < Kp) reinterpret_cast<float4*>(a)[c] = r[j];
  }
}

template <int J>
__global__ void __launch_bounds__(kBandNT) k_linemin_r(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16 * 4];
  const int Kp = cd.Kp;
  float* x = (float*)cd.X + (size_t)i * Kp;
  float* hx = (float*)cd.HX + (size_t)i * Kp;
  const float* d = (const float*)cd.D + (size_t)i * Kp;
  const float* hd = (const float*)cd.HD + (size_t)i * Kp;
  float4 X[J], HX[J], D[J], HD[J];
  load_band4<J>(x, Kp, X);
  load_band4<J>(hx, Kp, HX);
  load_band4<J>(d, Kp, D);
  load_band4<J>(hd, Kp, HD);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    v[0] += (double)X[j].x * HX[j].x + (double)X[j].y * HX[j].y + (double)X[j].z * HX[j].z +
            (double)X[j].w * HX[j].w;
    v[1] += (double)X[j].x * HD[j].x + (double)X[j].y * HD[j].y + (double)X[j].z * HD[j].z +
            (double)X[j].w * HD[j].w;
    v[2] += (double)D[j].x * HD[j].x + (double)D[j].y * HD[j].y + (double)D[j].z * HD[j].z +
            (double)D[j].w * HD[j].w;
    v[3] += (double)D[j].x * D[j].x + (double)D[j].y * D[j].y + (double)D[j].z * D[j].z +
            (double)D[j].w * D[j].w;
  }
  block_sum<4>(v, sh);
  const double n2 = v[3];
  if (!(n2 > 0.0)) return;
  const double inv = 1.0 / sqrt(n2);
  const double a = v[0], b = v[1] * inv, c = v[2] * inv * inv;
  const double theta = 0.5 * atan2(-2.0 * b, c - a);
  double sn, cs;
  sincos(theta, &sn, &cs);
  const float c32 = (float)cs, s32 = (float)(sn * inv);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    X[j] = make_float4(c32 * X[j].x + s32 * D[j].x, c32 * X[j].y + s32 * D[j].y,
                       c32 * X[j].z + s32 * D[j].z, c32 * X[j].w + s32 * D[j].w);
    HX[j] = make_float4(c32 * HX[j].x + s32 * HD[j].x, c32 * HX[j].y + s32 * HD[j].y,
                        c32 * HX[j].z + s32 * HD[j].z, c32 * HX[j].w + s32 * HD[j].w);
  }
  store_band4<J>(x, Kp, X);
  store_band4<J>(hx, Kp, HX);
}

template <int J>
__global__ void __launch_bounds__(kBandNT) k_cg_direction_r(const CandDesc* __restrict__ cds, int first) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16 * 2];
  const int Kp = cd.Kp, npwh = cd.npwh;
  const float* x = (const float*)cd.X + (size_t)i * Kp;
  const float* hx = (const float*)cd.HX + (size_t)i * Kp;
  float* d = (float*)cd.D + (size_t)i * Kp;
  float4 X[J], R[J];
  float2 KN[J];  // |G|^2/2 of the two coefficients of each float4
  load_band4<J>(x, Kp, X);
  load_band4<J>(hx, Kp, R);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = threadIdx.x + kBandNT * j;
    KN[j].x = 2 * c < npwh ? (float)cd.kin[2 * c] : 0.f;
    KN[j].y = 2 * c + 1 < npwh ? (float)cd.kin[2 * c + 1] : 0.f;
  }
  double v[1] = {0.0};
#pragma unroll
  for (int j = 0; j < J; ++j)
    v[0] += (double)KN[j].x * ((double)X[j].x * X[j].x + (double)X[j].y * X[j].y) +
            (double)KN[j].y * ((double)X[j].z * X[j].z + (double)X[j].w * X[j].w);
  block_sum<1>(v, sh);
  const double ek = fmax(v[0], 1e-8);
  const float e = (float)cd.eps[i];
  const float iek = (float)(1.0 / ek);
  double w[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    // residual r = H x - e x, preconditioned g = K(|G|^2/2 / ek) r
    R[j] = make_float4(R[j].x - e * X[j].x, R[j].y - e * X[j].y, R[j].z - e * X[j].z,
                       R[j].w - e * X[j].w);
    const double ra = (double)R[j].x * R[j].x + (double)R[j].y * R[j].y;
    const double rb = (double)R[j].z * R[j].z + (double)R[j].w * R[j].w;
    const float ka = (float)tpa((double)(KN[j].x * iek)), kb = (float)tpa((double)(KN[j].y * iek));
    w[0] += (double)ka * ra + (double)kb * rb;
    w[1] += ra + rb;
    R[j] = make_float4(ka * R[j].x, ka * R[j].y, kb * R[j].z, kb * R[j].w);
  }
  block_sum<2>(w, sh);
  const double gam = w[0];
  if (threadIdx.x == 0) cd.resn[i] = w[1];
  float beta = 0.f;
  if (!first) {
    const double gp = cd.gam[i];
    beta = gp > 0.0 ? (float)(gam / gp) : 0.f;
    float4 D[J];
    load_band4<J>(d, Kp, D);
#pragma unroll
    for (int j = 0; j < J; ++j)
      R[j] = make_float4(R[j].x + beta * D[j].x, R[j].y + beta * D[j].y, R[j].z + beta * D[j].z,
                         R[j].w + beta * D[j].w);
  }
  store_band4<J>(d, Kp, R);
  if (threadIdx.x == 0) cd.gam[i] = gam;
}

// Kinetic energy of each band: bandw[i] = sum_G |G|^2/2 |c_iG|^2.
template <typename T>
__global__ void __launch_bounds__(kNT) k_band_kinetic(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16];
  const T* x = (const T*)cd.X + (size_t)i * cd.Kp;
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < cd.K; k += blockDim.x) {
    const double xv = x[k];
    v[0] += cd.kin[k >> 1] * xv * xv;
  }
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) cd.bandw[i] = v[0];
}

// Counter-based starting wavefunctions: uniform(-1,1) from a 64-bit mix of
// (seed, candidate, band, index), damped by 1/(1 + |G|^2/2).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
template <typename T>
__global__ void k_init_random(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.y;
  if (i >= cd.nb) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cd.K; k += gridDim.x * blockDim.x) {
    unsigned long long h = mix64(((unsigned long long)cd.seed << 40) ^
                                 ((unsigned long long)cd.ncand_index << 32) ^
                                 ((unsigned long long)i << 20) ^ (unsigned long long)k);
    h = mix64(h);
    const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const double v = k == 1 ? 0.0 : u / (1.0 + cd.kin[k >> 1]);
    ((T*)cd.X)[(size_t)i * cd.Kp + k] = (T)v;
    ((T*)cd.D)[(size_t)i * cd.Kp + k] = (T)0;
  }
}

// Kleinman-Bylander projectors in packed storage:
// beta_{Ilm}(G) = p_l(|G|) (-i)^l Y_lm(G^) e^{-i G.R_I} / sqrt(Omega).
template <typename T>
__global__ void k_setup_beta(const CandDesc* __restrict__ cds, const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int p = blockIdx.y;
  if (p >= cd.nproj) return;
  const int I = cd.proj_atom[p];
  const int l = cd.proj_lm[p] >> 2, m = cd.proj_lm[p] & 3;
  const double rl = cd.proj_r[p];
  const double R0 = cd.pos[3 * I], R1 = cd.pos[3 * I + 1], R2 = cd.pos[3 * I + 2];
  const double inv_sqrt_omega = 1.0 / sqrt(cd.omega);
  const double pi = 3.14159265358979323846;
  T* out = (T*)cd.beta + (size_t)p * cd.Kp;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < cd.npwh; g += gridDim.x * blockDim.x) {
    const double m1 = cd.gmill[3 * g], m2 = cd.gmill[3 * g + 1], m3 = cd.gmill[3 * g + 2];
    const double G0 = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
    const double G1 = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
    const double G2 = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
    const double gg = sqrt(G0 * G0 + G1 * G1 + G2 * G2);
    double val;  // real amplitude before the phase; (-i)^l handled below
    if (l == 0) {
      // 4 pi sqrt(pi) r^{3/2} e^{-G^2 r^2/2} / sqrt(Gamma(3/2)) * Y00
      val = 4.0 * pi * sqrt(pi) * pow(rl, 1.5) * exp(-0.5 * gg * gg * rl * rl) /
            sqrt(0.5 * sqrt(pi)) * (1.0 / sqrt(4.0 * pi));
    } else {
      const double gm = m == 0 ? G0 : (m == 1 ? G1 : G2);
      // p_1(G) Y_1m = 4 pi sqrt(pi) r^{5/2} G e^{..} / sqrt(Gamma(5/2)) * sqrt(3/4pi) G_m/G
      val = 4.0 * pi * sqrt(pi) * pow(rl, 2.5) * exp(-0.5 * gg * gg * rl * rl) /
            sqrt(0.75 * sqrt(pi)) * sqrt(3.0 / (4.0 * pi)) * gm;
    }
    val *= inv_sqrt_omega;
    double sn, cs;
    sincos(-(G0 * R0 + G1 * R1 + G2 * R2), &sn, &cs);
    double re = val * cs, im = val * sn;  // val e^{-iG.R}
    if (l == 1) {  // multiply by -i
      const double t = re;
      re = im;
      im = -t;
    }
    if (g == 0) {
      out[0] = (T)re;
      out[1] = (T)0;
    } else {
      out[2 * g] = (T)(1.41421356237309504880 * re);
      out[2 * g + 1] = (T)(1.41421356237309504880 * im);
    }
  }
}

// Projections needed by the nonlocal forces, for projector p and band i:
// P = <beta_p|psi_i>, dP_a = <-i G_a beta_p|psi_i>  (a = x, y, z).
template <typename T>
__global__ void __launch_bounds__(kNT) k_force_nonlocal(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int p = blockIdx.x, i = blockIdx.y;
  if (p >= cd.nproj || i >= cd.nb) return;
  __shared__ double sh[16 * 4];
  const T* b = (const T*)cd.beta + (size_t)p * cd.Kp;
  const T* x = (const T*)cd.X + (size_t)i * cd.Kp;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < cd.npwh; g += blockDim.x) {
    const double br = b[2 * g], bi = b[2 * g + 1], xr = x[2 * g], xi = x[2 * g + 1];
    v[0] += br * xr + bi * xi;
    const double m1 = cd.gmill[3 * g], m2 = cd.gmill[3 * g + 1], m3 = cd.gmill[3 * g + 2];
    const double t = bi * xr - br * xi;  // packed (-i beta) . x per unit G
    v[1] += (m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6]) * t;
    v[2] += (m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7]) * t;
    v[3] += (m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8]) * t;
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0) {
    double* o = cd.nlwork + ((size_t)p * cd.nb + i) * 4;
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
  }
}

// ------------------------------------------------------------------ stress
// Fixed-basis stress under the strain r -> (1 + eps) r: G.R is invariant and
// d(G^2)/d eps_ab = -2 G_a G_b.  Wavefunction-side sums for band i:
// kinetic K_ab = sum_G G_a G_b |c_G|^2 over the full sphere (a packed pair
// x, y of +-G holds x^2 + y^2 = 2 |c_G|^2).
__device__ __forceinline__ void gvec_of(const CandDesc& cd, int g, double* G) {
  const double m1 = cd.gmill[3 * g], m2 = cd.gmill[3 * g + 1], m3 = cd.gmill[3 * g + 2];
  G[0] = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
  G[1] = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
  G[2] = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_stress_kinetic(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int i = blockIdx.x;
  if (i >= cd.nb) return;
  __shared__ double sh[16 * 6];
  const T* x = (const T*)cd.X + (size_t)i * cd.Kp;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < cd.npwh; g += blockDim.x) {
    double G[3];
    gvec_of(cd, g, G);
    const double a = x[2 * g], b = x[2 * g + 1];
    add_voigt(v, a * a + b * b, G);
  }
  block_sum<6>(v, sh);
  if (threadIdx.x == 0) {
    double* o = cd.stwork + stress_layout(cd.nb, cd.nproj, cd.nat).kin + (size_t)6 * i;
    for (int k = 0; k < 6; ++k) o[k] = v[k];
  }
}

// Nonlocal sums for projector p and band i: P = <beta_p|psi_i> and
// Q_ab = <G_a G_b beta_p|psi_i> (both real at the Gamma point).  The strain
// derivative of beta (volume factor, radial part through G^2, and the
// direction factor G_m of l = 1) is assembled from these in the finalize step.
template <typename T>
__global__ void __launch_bounds__(kNT) k_stress_nonlocal(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int p = blockIdx.x, i = blockIdx.y;
  if (p >= cd.nproj || i >= cd.nb) return;
  __shared__ double sh[16 * 7];
  const T* b = (const T*)cd.beta + (size_t)p * cd.Kp;
  const T* x = (const T*)cd.X + (size_t)i * cd.Kp;
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < cd.npwh; g += blockDim.x) {
    const double d = (double)b[2 * g] * x[2 * g] + (double)b[2 * g + 1] * x[2 * g + 1];
    v[0] += d;
    double G[3];
    gvec_of(cd, g, G);
    add_voigt(v + 1, d, G);
  }
  block_sum<7>(v, sh);
  if (threadIdx.x == 0) {
    double* o = cd.stwork + stress_layout(cd.nb, cd.nproj, cd.nat).nl + ((size_t)p * cd.nb + i) * 7;
    for (int k = 0; k < 7; ++k) o[k] = v[k];
  }
}

// V_eff(r) from the inverse transform of V(G) + i rho_in(G): real part is
// V_loc + V_H, imaginary part the mixed input density.  Adds v_xc.
template <typename T>
__global__ void k_potential_finalize(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += gridDim.x * blockDim.x) {
    const cplx<double> z = cd.zgrid[e];
    const double rho = z.y;
    double ex, vx;
    pz81(fmax(rho, 0.0), &ex, &vx);
    const double v = z.x + vx;
    cd.rho_in_r[e] = rho;
    cd.veff_r[e] = v;
    ((T*)cd.veff_t)[e] = (T)v;
  }
}

// ---------------------------------------------------------- launch helpers
template <typename T>
static size_t z_lds(const BatchGeom& g) {
  const int nloc = 2 * g.sp_chunk;
  return sizeof(cplx<T>) * (kMaxFftN + 2 * (size_t)nloc * g.N3max);
}
template <typename T>
static size_t plane_lds(const BatchGeom& g) {
  return sizeof(cplx<T>) * (2 * kMaxFftN + 2 * (size_t)g.plane_max);
}

template <typename T>
void launch_hpsi(const LaunchCtx& L, int src) {
  const BatchGeom& g = L.g;
  const int dst = src == W_X ? W_HX : W_HD;
  const bool reg = std::is_same<T, float>::value && g.plane_reg;
  dim3 gz((g.nsp_max + g.sp_chunk - 1) / g.sp_chunk, g.npair_max, g.ncand);
  if (reg) {
    launch_z_inverse_reg(L, src);
  } else {
    prof_before("k_z_inverse", L.stream);
    hipLaunchKernelGGL(k_z_inverse<T>, gz, dim3(kNT), z_lds<T>(g), L.stream, L.desc, src,
                       g.sp_chunk);
    check_launch("k_z_inverse");
    prof_after("k_z_inverse", L.stream);
  }
  if (std::is_same<T, float>::value && g.plane_reg) {
    launch_plane_hpsi_reg(L);
  } else {
    dim3 gp(g.N3max, g.npair_max, g.ncand);
    prof_before("k_plane_hpsi", L.stream);
    hipLaunchKernelGGL(k_plane_hpsi<T>, gp, dim3(kNT), plane_lds<T>(g), L.stream, L.desc);
    check_launch("k_plane_hpsi");
    prof_after("k_plane_hpsi", L.stream);
  }
  if (reg) {
    launch_z_forward_reg(L, src, dst);
  } else {
    prof_before("k_z_forward", L.stream);
    hipLaunchKernelGGL(k_z_forward<T>, gz, dim3(kNT), z_lds<T>(g), L.stream, L.desc, src, dst,
                       g.sp_chunk);
    check_launch("k_z_forward");
    prof_after("k_z_forward", L.stream);
  }
  if (g.nproj_max > 0 && std::is_same<T, float>::value && g.bf16proj) {
    launch_proj_bf16(L, src, dst);
  } else if (g.nproj_max > 0) {
    int a[1] = {W_BETA}, b[1] = {src}, o[1] = {M_C};
    launch_gram<T>(L, 1, a, b, o);
    int y[1] = {dst}, aa[1] = {W_BETA};
    launch_gemm_acc<T>(L, 1, y, aa, M_C, 1.0, 1.0, 1);
  }
}

template <typename T>
void launch_density(const LaunchCtx& L) {
  const BatchGeom& g = L.g;
  dim3 gz((g.nsp_max + g.sp_chunk - 1) / g.sp_chunk, g.npair_max, g.ncand);
  if (std::is_same<T, float>::value && g.plane_reg) {
    launch_z_inverse_reg(L, (int)W_X);
  } else {
    prof_before("k_z_inverse", L.stream);
    hipLaunchKernelGGL(k_z_inverse<T>, gz, dim3(kNT), z_lds<T>(g), L.stream, L.desc, (int)W_X,
                       g.sp_chunk);
    check_launch("k_z_inverse");
    prof_after("k_z_inverse", L.stream);
  }
  if (std::is_same<T, float>::value && g.plane_reg) {
    launch_plane_density_reg(L);
  } else {
    dim3 gp(g.N3max, g.dens_chunks, g.ncand);
    prof_before("k_plane_density", L.stream);
    hipLaunchKernelGGL(k_plane_density<T>, gp, dim3(kNT), plane_lds<T>(g), L.stream, L.desc);
    check_launch("k_plane_density");
    prof_after("k_plane_density", L.stream);
  }
}

template <typename T>
void launch_gram(const LaunchCtx& L, int nprod, const int* a, const int* b, const int* out) {
  const BatchGeom& g = L.g;
  const int rows = std::max(g.nb_max, g.nproj_max);
  const int a1 = nprod > 1 ? a[1] : 0, b1 = nprod > 1 ? b[1] : 0, o1 = nprod > 1 ? out[1] : 0;
  // rows read per candidate: each distinct operand array once
  long long rows_read = 0;
  {
    int seen[4], ns = 0;
    const int ops[4] = {a[0], b[0], a1, b1};
    for (int q = 0; q < 2 * nprod; ++q) {
      bool dup = false;
      for (int t = 0; t < ns; ++t) dup = dup || seen[t] == ops[q];
      if (dup) continue;
      seen[ns++] = ops[q];
      rows_read += ops[q] == W_BETA ? g.nproj_max : g.nb_max;
    }
  }
  // 32x32 output tiles (88 registers, 4 waves per SIMD; 64x64 tiles take
  // 351 registers, one wave per SIMD, and were 10% slower on the uneven
  // population's 56-112 bands); the tuning key SGO_GRAM_TILE = 64 selects them
  const int TB = g.gram_tile == 64 ? 4 : 2;
  const int TT = 16 * TB;
  const int nt = (rows + TT - 1) / TT;
  dim3 grid(nt * nt * g.nkc_max, nprod, g.ncand);
  dim3 rgrid((rows * rows + kNT - 1) / kNT, nprod, g.ncand);
  prof_before("k_gram", L.stream);
  if constexpr (std::is_same<T, float>::value) {
    if (g.gram_f32) {
      if (TB == 2)
        hipLaunchKernelGGL((k_gram<float, 2, true>), grid, dim3(kNT), 0, L.stream, L.desc, g.kc_len,
                           g.nkc_max, a[0], b[0], a1, b1);
      else
        hipLaunchKernelGGL((k_gram<float, 4, true>), grid, dim3(kNT), 0, L.stream, L.desc, g.kc_len,
                           g.nkc_max, a[0], b[0], a1, b1);
      check_launch("k_gram");
      prof_after("k_gram", L.stream, rows_read);
      goto reduce;
    }
  }
  if (TB == 2)
    hipLaunchKernelGGL((k_gram<T, 2>), grid, dim3(kNT), 0, L.stream, L.desc, g.kc_len, g.nkc_max,
                       a[0], b[0], a1, b1);
  else
    hipLaunchKernelGGL((k_gram<T, 4>), grid, dim3(kNT), 0, L.stream, L.desc, g.kc_len, g.nkc_max,
                       a[0], b[0], a1, b1);
  check_launch("k_gram");
  prof_after("k_gram", L.stream, rows_read);
reduce:
  prof_before("k_gram_reduce", L.stream);
  if (TB == 2)
    hipLaunchKernelGGL((k_gram_reduce<2>), rgrid, dim3(kNT), 0, L.stream, L.desc, g.kc_len, a[0],
                       b[0], out[0], a1, b1, o1);
  else
    hipLaunchKernelGGL((k_gram_reduce<4>), rgrid, dim3(kNT), 0, L.stream, L.desc, g.kc_len, a[0],
                       b[0], out[0], a1, b1, o1);
  check_launch("k_gram_reduce");
  prof_after("k_gram_reduce", L.stream);
}

// input rows from which several wavefronts share a staged slice
constexpr int kGemmWavesFrom = 64;

template <typename T>
void launch_gemm_acc(const LaunchCtx& L, int narr, const int* y, const int* a, int mat,
                     double alpha, double beta, int use_h) {
  const BatchGeom& g = L.g;
  const int rows = std::max(g.nb_max, g.nproj_max);
  const int nib = (g.nb_max + 15) / 16;  // outputs are always band rows
  dim3 grid((g.K_max + 63) / 64, narr, g.ncand);
  size_t lds = sizeof(double) * ((size_t)kJC * 64 + (size_t)kJC * nib * 16);
  (void)rows;
  const int y1 = narr > 1 ? y[1] : 0, y2 = narr > 2 ? y[2] : 0;
  const int a1 = narr > 1 ? a[1] : 0, a2 = narr > 2 ? a[2] : 0;
  int nin_max = 0;
  long long rows_moved = 0;  // per candidate: A read, Y written, Y read when alpha != 0
  for (int q = 0; q < narr; ++q) {
    const int nin = a[q] == W_BETA ? g.nproj_max : g.nb_max;
    nin_max = std::max(nin_max, nin);
    rows_moved += nin + (alpha != 0.0 ? 2 : 1) * g.nb_max;
  }
  // the MFMA kernel stages all nin input rows of its 64 columns in LDS; from
  // kGemmWavesFrom input rows (16 KB a slice and more: few slices resident
  // per compute unit) several wavefronts share a slice, each taking every
  // NW-th output tile (282 bands: 809 ms per evaluation of the 128-atom cell
  // with 4 wavefronts and 32-row tiles, 745 with 8 and 16-row tiles; the
  // uneven population of 24 to 112 bands: 52.5 evaluations/s from 64 rows
  // against 49.4 from 128)
  const size_t lds32 = (size_t)nin_max * 64 * sizeof(float);
  if (std::is_same<T, float>::value && lds32 <= g.lds_limit && g.gemm_f32) {
    prof_before("k_gemm_acc", L.stream);
    const dim3 grid32((g.K_max + 63) / 64, narr, g.ncand);
    if (nin_max >= kGemmWavesFrom && g.gemm_waves >= 8)
      hipLaunchKernelGGL((k_gemm_f32<1, 8>), grid32, dim3(512), lds32, L.stream, L.desc, y[0], y1,
                         y2, a[0], a1, a2, mat, (float)alpha, (float)beta, use_h);
    else if (nin_max >= kGemmWavesFrom && g.gemm_waves >= 6)
      hipLaunchKernelGGL((k_gemm_f32<1, 6>), grid32, dim3(384), lds32, L.stream, L.desc, y[0], y1,
                         y2, a[0], a1, a2, mat, (float)alpha, (float)beta, use_h);
    else if (nin_max >= kGemmWavesFrom)
      hipLaunchKernelGGL((k_gemm_f32<2, 4>), grid32, dim3(256), lds32, L.stream, L.desc, y[0], y1,
                         y2, a[0], a1, a2, mat, (float)alpha, (float)beta, use_h);
    else if (g.nb_max <= 32)
      hipLaunchKernelGGL((k_gemm_f32<2, 1>), grid32, dim3(64), lds32, L.stream, L.desc, y[0], y1,
                         y2, a[0], a1, a2, mat, (float)alpha, (float)beta, use_h);
    else
      hipLaunchKernelGGL((k_gemm_f32<4, 1>), grid32, dim3(64), lds32, L.stream, L.desc, y[0], y1,
                         y2, a[0], a1, a2, mat, (float)alpha, (float)beta, use_h);
    check_launch("k_gemm_acc");
    prof_after("k_gemm_acc", L.stream, rows_moved);
    return;
  }
  prof_before("k_gemm_acc", L.stream);
  if (nib <= 4)
    hipLaunchKernelGGL((k_gemm_acc<T, 1>), grid, dim3(kNT), lds, L.stream, L.desc, y[0], y1, y2,
                       a[0], a1, a2, mat, alpha, beta, use_h);
  else if (nib <= 8)
    hipLaunchKernelGGL((k_gemm_acc<T, 2>), grid, dim3(kNT), lds, L.stream, L.desc, y[0], y1, y2,
                       a[0], a1, a2, mat, alpha, beta, use_h);
  else if (nib <= 20)
    hipLaunchKernelGGL((k_gemm_acc<T, 5>), grid, dim3(kNT), lds, L.stream, L.desc, y[0], y1, y2,
                       a[0], a1, a2, mat, alpha, beta, use_h);
  else
    throw_unsupported("more than 320 bands in the rotation kernel");
  check_launch("k_gemm_acc");
  prof_after("k_gemm_acc", L.stream, rows_moved);
}

// J = float4 per thread and band array of the one-pass FP32 band kernels
// (0: Kp too large, the multi-pass kernels are used)
static int band_j(const BatchGeom& g) {
  int kp = 0;
  kp = (g.K_max + 31) / 32 * 32;
  if (kp <= 4 * kBandNT * 4) return 4;
  if (kp <= 4 * kBandNT * 8) return 8;
  if (kp <= 4 * kBandNT * 12) return 12;
  return 0;
}

template <typename T>
void launch_cg_direction(const LaunchCtx& L, int first) {
  const int J = std::is_same<T, float>::value ? band_j(L.g) : 0;
  if (J) {
    prof_before("k_cg_direction", L.stream);
    const dim3 gr(L.g.nb_max, 1, L.g.ncand);
    if (J == 4) hipLaunchKernelGGL(k_cg_direction_r<4>, gr, dim3(kBandNT), 0, L.stream, L.desc, first);
    else if (J == 8) hipLaunchKernelGGL(k_cg_direction_r<8>, gr, dim3(kBandNT), 0, L.stream, L.desc, first);
    else hipLaunchKernelGGL(k_cg_direction_r<12>, gr, dim3(kBandNT), 0, L.stream, L.desc, first);
    check_launch("k_cg_direction");
    prof_after("k_cg_direction", L.stream);
    return;
  }
  prof_before("k_cg_direction", L.stream);
  hipLaunchKernelGGL(k_cg_direction<T>, dim3(L.g.nb_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, first);
  check_launch("k_cg_direction");
  prof_after("k_cg_direction", L.stream);
}
template <typename T>
void launch_linemin(const LaunchCtx& L) {
  const int J = std::is_same<T, float>::value ? band_j(L.g) : 0;
  if (J) {
    prof_before("k_linemin", L.stream);
    const dim3 gr(L.g.nb_max, 1, L.g.ncand);
    if (J == 4) hipLaunchKernelGGL(k_linemin_r<4>, gr, dim3(kBandNT), 0, L.stream, L.desc);
    else if (J == 8) hipLaunchKernelGGL(k_linemin_r<8>, gr, dim3(kBandNT), 0, L.stream, L.desc);
    else hipLaunchKernelGGL(k_linemin_r<12>, gr, dim3(kBandNT), 0, L.stream, L.desc);
    check_launch("k_linemin");
    prof_after("k_linemin", L.stream);
    return;
  }
  prof_before("k_linemin", L.stream);
  hipLaunchKernelGGL(k_linemin<T>, dim3(L.g.nb_max, 1, L.g.ncand), dim3(kNT), 0, L.stream, L.desc);
  check_launch("k_linemin");
  prof_after("k_linemin", L.stream);
}
template <typename T>
void launch_band_kinetic(const LaunchCtx& L) {
  prof_before("k_band_kinetic", L.stream);
  hipLaunchKernelGGL(k_band_kinetic<T>, dim3(L.g.nb_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc);
  check_launch("k_band_kinetic");
  prof_after("k_band_kinetic", L.stream);
}
template <typename T>
void launch_init_random(const LaunchCtx& L) {
  prof_before("k_init_random", L.stream);
  hipLaunchKernelGGL(k_init_random<T>, dim3(8, L.g.nb_max, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc);
  check_launch("k_init_random");
  prof_after("k_init_random", L.stream);
}
template <typename T>
void launch_setup_beta(const LaunchCtx& L) {
  if (L.g.nproj_max == 0) return;
  prof_before("k_setup_beta", L.stream);
  hipLaunchKernelGGL(k_setup_beta<T>, dim3(16, L.g.nproj_max, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_setup_beta");
  prof_after("k_setup_beta", L.stream);
  if (std::is_same<T, float>::value && L.g.bf16proj) launch_beta_bf16(L);
}
template <typename T>
void launch_force_nonlocal(const LaunchCtx& L) {
  if (L.g.nproj_max == 0) return;
  prof_before("k_force_nonlocal", L.stream);
  hipLaunchKernelGGL(k_force_nonlocal<T>, dim3(L.g.nproj_max, L.g.nb_max, L.g.ncand), dim3(kNT), 0,
                     L.stream, L.desc);
  check_launch("k_force_nonlocal");
  prof_after("k_force_nonlocal", L.stream);
}
template <typename T>
void launch_stress_waves(const LaunchCtx& L) {
  prof_before("k_stress_kinetic", L.stream);
  hipLaunchKernelGGL(k_stress_kinetic<T>, dim3(L.g.nb_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc);
  check_launch("k_stress_kinetic");
  prof_after("k_stress_kinetic", L.stream);
  if (L.g.nproj_max == 0) return;
  prof_before("k_stress_nonlocal", L.stream);
  hipLaunchKernelGGL(k_stress_nonlocal<T>, dim3(L.g.nproj_max, L.g.nb_max, L.g.ncand), dim3(kNT),
                     0, L.stream, L.desc);
  check_launch("k_stress_nonlocal");
  prof_after("k_stress_nonlocal", L.stream);
}
template <typename T>
void launch_potential_finalize(const LaunchCtx& L) {
  prof_before("k_potential_finalize", L.stream);
  hipLaunchKernelGGL(k_potential_finalize<T>, dim3((L.g.ntot_max + kNT - 1) / kNT, 1, L.g.ncand),
                     dim3(kNT), 0, L.stream, L.desc);
  check_launch("k_potential_finalize");
  prof_after("k_potential_finalize", L.stream);
}

template <typename T>
static void configure_t() {
  allow_lds((const void*)k_z_inverse<T>);
  allow_lds((const void*)k_z_forward<T>);
  allow_lds((const void*)k_plane_hpsi<T>);
  allow_lds((const void*)k_plane_density<T>);
  allow_lds((const void*)k_gemm_acc<T, 1>);
  allow_lds((const void*)k_gemm_acc<T, 2>);
  allow_lds((const void*)k_gemm_acc<T, 5>);
}
void configure_wave() {
  allow_lds((const void*)k_gemm_f32<2, 1>);
  allow_lds((const void*)k_gemm_f32<4, 1>);
  allow_lds((const void*)k_gemm_f32<2, 4>);
  allow_lds((const void*)k_gemm_f32<1, 6>);
  allow_lds((const void*)k_gemm_f32<1, 8>);
  configure_t<float>();
  configure_t<double>();
}

#define SGO_INST(T)                                                                       \
  template void launch_hpsi<T>(const LaunchCtx&, int);                                    \
  template void launch_density<T>(const LaunchCtx&);                                      \
  template void launch_gram<T>(const LaunchCtx&, int, const int*, const int*, const int*); \
  template void launch_gemm_acc<T>(const LaunchCtx&, int, const int*, const int*, int, double, \
                                   double, int);                                         \
  template void launch_cg_direction<T>(const LaunchCtx&, int);                            \
  template void launch_linemin<T>(const LaunchCtx&);                                      \
  template void launch_band_kinetic<T>(const LaunchCtx&);                                 \
  template void launch_init_random<T>(const LaunchCtx&);                                  \
  template void launch_setup_beta<T>(const LaunchCtx&);                                   \
  template void launch_force_nonlocal<T>(const LaunchCtx&);                               \
  template void launch_potential_finalize<T>(const LaunchCtx&);                           \
  template void launch_stress_waves<T>(const LaunchCtx&);
SGO_INST(float)
SGO_INST(double)

}  // namespace sgo
