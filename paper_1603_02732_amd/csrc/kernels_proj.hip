// Kleinman-Bylander projector products with BF16 inputs and FP32
// accumulation on MFMA (the FP32_BF16PROJ precision form; the nonlocal part
// of the H psi step of Algorithm 1):
//   P = beta^T Psi          split-K partials in FP32, summed over the K
//                           chunks in FP64 in a fixed order;
//   H Psi += beta (h P)     FP32 accumulation.
// Every operand x is carried as two BF16 numbers, hi = bf16(x) and
// lo = bf16(x - hi) (16 significant bits), and a product is hi*hi + hi*lo +
// lo*hi: three BF16 MFMAs.  A single BF16 rounding of beta and Psi leaves
// ~2^-9/sqrt(K) relative errors in P, which for the cluster population moves
// the energy by ~5e-5 Ha/atom, outside the 1e-5 gate; the split brings the
// products to ~2^-17 relative.
#include "device.hpp"
#include "launch.hpp"

namespace sgo {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// beta (FP32, [nproj][Kp]) -> beta16 [2][np16][Kp] and betaT16 [2][Kp][np16]
// (hi and lo parts; rows nproj..np16-1 stay zero).
__global__ void __launch_bounds__(kNT) k_beta_bf16(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int p = blockIdx.y;
  if (p >= cd.nproj) return;
  const float* b = (const float*)cd.beta + (size_t)p * cd.Kp;
  const size_t plane_r = (size_t)cd.np16 * cd.Kp;  // hi plane, then lo plane
  unsigned short* r = (unsigned short*)cd.beta16 + (size_t)p * cd.Kp;
  unsigned short* t = (unsigned short*)cd.betaT16;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cd.Kp; k += gridDim.x * blockDim.x) {
    const float x = b[k];
    const unsigned short hi = f2bf(x), lo = f2bf(x - bf2f(hi));
    r[k] = hi;
    r[plane_r + k] = lo;
    t[(size_t)k * cd.np16 + p] = hi;
    t[plane_r + (size_t)k * cd.np16 + p] = lo;
  }
}

// Partial projections of one K chunk and one 16-band tile, every 16-row
// projector tile: D[p][i] += A[p][k] B[k][i] with A = beta16 rows, B = Psi^T.
// Lane l supplies A[l%16][4(l/16)..+3] and B[4(l/16)..+3][l%16] (contiguous in
// k for both); D[4(l/16)+r][l%16] comes back in register r.
constexpr int kProjGroup = 8;  // projector tiles per pass over the chunk
__global__ void __launch_bounds__(64) k_proj_bf16(const CandDesc* __restrict__ cds, int src, int kc) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int chunk = blockIdx.x, it = blockIdx.y;
  const int nb = cd.nb, np16 = cd.np16, ntp = np16 / 16, nb16 = (nb + 15) / 16 * 16;
  const int i0 = 16 * it, k0 = chunk * kc;
  if (i0 >= nb || k0 >= cd.Kp || cd.nproj == 0) return;
  const int k1 = min(k0 + kc, cd.Kp);
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  const int i = i0 + n;
  const float* X = (const float*)(src == W_X ? cd.X : cd.D) + (size_t)i * cd.Kp;
  const unsigned short* B16 = (const unsigned short*)cd.beta16;
  const size_t plane = (size_t)np16 * cd.Kp;
  float* part = (float*)cd.red_part + (size_t)chunk * np16 * nb16;
  for (int pg = 0; pg < ntp; pg += kProjGroup) {
    floatx4 acc[kProjGroup];
#pragma unroll
    for (int t = 0; t < kProjGroup; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k = k0; k < k1; k += 16) {
      const int kk = k + 4 * g;
      short4_t bh = {0, 0, 0, 0}, bl = {0, 0, 0, 0};
      if (i < nb) {
        const float4 x = *(const float4*)(X + kk);
        const unsigned short h0 = f2bf(x.x), h1 = f2bf(x.y), h2 = f2bf(x.z), h3 = f2bf(x.w);
        bh = short4_t{(short)h0, (short)h1, (short)h2, (short)h3};
        bl = short4_t{(short)f2bf(x.x - bf2f(h0)), (short)f2bf(x.y - bf2f(h1)),
                      (short)f2bf(x.z - bf2f(h2)), (short)f2bf(x.w - bf2f(h3))};
      }
#pragma unroll
      for (int t = 0; t < kProjGroup; ++t) {
        if (pg + t >= ntp) break;
        const int p = (pg + t) * 16 + n;
        const short4_t ah = *(const short4_t*)(B16 + (size_t)p * cd.Kp + kk);
        const short4_t al = *(const short4_t*)(B16 + plane + (size_t)p * cd.Kp + kk);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < kProjGroup; ++t) {
      if (pg + t >= ntp) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(size_t)((pg + t) * 16 + 4 * g + r) * nb16 + i] = acc[t][r];
    }
  }
}

// P[p][i] = sum over the K chunks (fixed order, FP64) into the matrix C.
__global__ void __launch_bounds__(kNT) k_proj_reduce(const CandDesc* __restrict__ cds, int kc) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  const int nb = cd.nb, np16 = cd.np16, nb16 = (nb + 15) / 16 * 16;
  const int nchunk = (cd.Kp + kc - 1) / kc;
  const float* part = (const float*)cd.red_part;
  for (int e = threadIdx.x; e < cd.nproj * nb; e += blockDim.x) {
    const int p = e / nb, i = e - p * nb;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += (double)part[((size_t)c * np16 + p) * nb16 + i];
    cd.C[(size_t)p * nb + i] = s;
  }
}

// Y[i][k] += sum_p (h_p P[p][i]) beta[p][k] for one 16-band tile and a range of
// 16-column tiles: A[i][p] = hP (hi and lo parts staged in LDS as [i][p]),
// B[p][k] from betaT16 (contiguous in p), D[4(l/16)+r][l%16] =
// dY[i0 + 4(l/16) + r][k0 + l%16].
constexpr int kApplyCols = 256;
__global__ void __launch_bounds__(64) k_proj_apply_bf16(const CandDesc* __restrict__ cds, int dst) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int it = blockIdx.y;
  const int nb = cd.nb, np16 = cd.np16, ntp = np16 / 16;
  const int i0 = 16 * it, kb = blockIdx.x * kApplyCols;
  if (i0 >= nb || kb >= cd.Kp || cd.nproj == 0) return;
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  extern __shared__ __align__(16) char smem[];
  unsigned short* ahi = (unsigned short*)smem;  // [16][np16]
  unsigned short* alo = ahi + 16 * np16;
  for (int e = lane; e < 16 * np16; e += 64) {
    const int ii = e / np16, p = e - ii * np16;
    const int i = i0 + ii;
    float v = 0.f;
    if (p < cd.nproj && i < nb) v = (float)(cd.hproj[p] * cd.C[(size_t)p * nb + i]);
    const unsigned short h = f2bf(v);
    ahi[e] = h;
    alo[e] = f2bf(v - bf2f(h));
  }
  __syncthreads();
  float* Y = (float*)(dst == W_HX ? cd.HX : cd.HD);
  const unsigned short* T16 = (const unsigned short*)cd.betaT16;
  const size_t tplane = (size_t)np16 * cd.Kp;
  const int kend = min(kb + kApplyCols, cd.Kp);
  for (int k0 = kb; k0 < kend; k0 += 16) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const int k = k0 + n;
    for (int pt = 0; pt < ntp; ++pt) {
      const int p = pt * 16 + 4 * g;
      const short4_t bh = *(const short4_t*)(T16 + (size_t)k * np16 + p);
      const short4_t bl = *(const short4_t*)(T16 + tplane + (size_t)k * np16 + p);
      const short4_t ah = *(const short4_t*)(ahi + n * np16 + p);
      const short4_t al = *(const short4_t*)(alo + n * np16 + p);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * g + r;
      if (i < nb) Y[(size_t)i * cd.Kp + k] += acc[r];
    }
  }
}

void launch_beta_bf16(const LaunchCtx& L) {
  if (L.g.nproj_max == 0) return;
  hipLaunchKernelGGL(k_beta_bf16, dim3(16, L.g.nproj_max, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc);
  check_launch("k_beta_bf16");
}

void launch_proj_bf16(const LaunchCtx& L, int src, int dst) {
  const BatchGeom& g = L.g;
  if (g.nproj_max == 0) return;
  const int kpmax = (g.K_max + 31) / 32 * 32;
  const int np16 = (g.nproj_max + 15) / 16 * 16, nb16 = (g.nb_max + 15) / 16 * 16;
  // K chunk: partials [nchunk][np16][nb16] floats must fit the reduction scratch
  int kc = 1024;
  while ((size_t)((kpmax + kc - 1) / kc) * np16 * nb16 * 4 > g.red_min_bytes && kc < kpmax) kc *= 2;
  prof_before("k_proj_bf16", L.stream);
  hipLaunchKernelGGL(k_proj_bf16, dim3((kpmax + kc - 1) / kc, nb16 / 16, g.ncand), dim3(64), 0,
                     L.stream, L.desc, src, kc);
  check_launch("k_proj_bf16");
  prof_after("k_proj_bf16", L.stream);
  hipLaunchKernelGGL(k_proj_reduce, dim3(g.ncand), dim3(kNT), 0, L.stream, L.desc, kc);
  check_launch("k_proj_reduce");
  prof_before("k_proj_apply_bf16", L.stream);
  hipLaunchKernelGGL(k_proj_apply_bf16, dim3((kpmax + kApplyCols - 1) / kApplyCols, nb16 / 16, g.ncand),
                     dim3(64), (size_t)2 * 16 * np16 * sizeof(unsigned short), L.stream, L.desc, dst);
  check_launch("k_proj_apply_bf16");
  prof_after("k_proj_apply_bf16", L.stream);
}

}  // namespace sgo
