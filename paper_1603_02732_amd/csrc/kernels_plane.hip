// FP32 plane kernels of the band FFTs with register-resident line transforms
// (the H psi step of Algorithm 1: the local-potential product in real
// space; Section 2.4: the output density).  One wavefront takes one z-plane
// of one band pair.  The plane lives in LDS only over its active x columns
// (the projection of the wavefunction sphere, |m1| <= m1max, stored
// compactly with an odd row stride so that both the column-wise and the
// row-wise accesses are free of bank conflicts).  Each lane transforms a
// whole line in registers (fft_reg.hpp):
//   y pass   one lane per active column (the other columns are zero),
//   x pass   one lane per row: inverse transform, times V_eff, forward
//            transform, keeping only the active columns,
//   y pass   forward, then the stick values are gathered.
// The y and x phases are dispatched on N2 and N1 separately, so the kernel
// carries one instantiation per supported length and axis, not per pair.
#include "device.hpp"
#include "fft_reg.hpp"
#include "launch.hpp"

#include <algorithm>

namespace sgo {

#define SGO_LINE_SIZES(X) \
  X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) \
  X(48) X(50) X(54) X(60) X(64)

bool plane_reg_length_ok(int n) {
  switch (n) {
#define SGO_CASE(N) \
  case N:           \
    return true;
    SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
    default:
      return false;
  }
}

struct PlaneLds {
  cplx<float>* Q;  // [N2][sx], active columns only
  int sx;          // row stride (odd, >= nx)
  int nx, nxl;     // active columns: x < nxl and x >= N1 - (nx - nxl)
};

__device__ __forceinline__ int col_of_x(const PlaneLds& p, int N1, int x) {
  return x < p.nxl ? x : x - (N1 - p.nx);
}

template <int N2, int S>
__device__ __forceinline__ void column_pass(const PlaneLds& p, int lane) {
  if (lane >= p.nx) return;
  cplx<float> v[N2], w[N2];
#pragma unroll
  for (int k = 0; k < N2; ++k) v[k] = p.Q[k * p.sx + lane];
  freg::fft<float, S, N2>(v, w);
#pragma unroll
  for (int k = 0; k < N2; ++k) p.Q[k * p.sx + lane] = w[k];
}

template <int S, int NMAX>
__device__ __forceinline__ void column_pass_rt(const PlaneLds& p, int N2, int lane) {
  switch (N2) {
#define SGO_CASE(N)              \
  case N:                        \
    if constexpr (N <= NMAX) column_pass<N, S>(p, lane); \
    break;
    SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
    default:
      break;
  }
}

// Row y of the plane into registers (zeros outside the active columns).
template <int N1>
__device__ __forceinline__ void load_row(const PlaneLds& p, int y, cplx<float> (&v)[N1]) {
  const int hi0 = N1 - (p.nx - p.nxl);
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const bool act = k < p.nxl || k >= hi0;
    const int c = act ? (k < p.nxl ? k : k - hi0 + p.nxl) : 0;
    const cplx<float> q = p.Q[y * p.sx + c];
    v[k] = act ? q : cplx<float>{0.f, 0.f};
  }
}

template <int N1>
__device__ __forceinline__ void load_vrow(const float* __restrict__ V, float (&r)[N1]) {
  if constexpr (N1 % 4 == 0) {
#pragma unroll
    for (int k = 0; k < N1 / 4; ++k) {
      const float4 q = reinterpret_cast<const float4*>(V)[k];
      r[4 * k] = q.x;
      r[4 * k + 1] = q.y;
      r[4 * k + 2] = q.z;
      r[4 * k + 3] = q.w;
    }
  } else if constexpr (N1 % 2 == 0) {
#pragma unroll
    for (int k = 0; k < N1 / 2; ++k) {
      const float2 q = reinterpret_cast<const float2*>(V)[k];
      r[2 * k] = q.x;
      r[2 * k + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = V[k];
  }
}

// x pass of H psi for row y: inverse transform, V_eff product, forward
// transform; the active columns are written back.
template <int N1>
__device__ __forceinline__ void row_pass_hpsi(const PlaneLds& p, int y, const float* __restrict__ V) {
  cplx<float> v[N1], w[N1];
  load_row<N1>(p, y, v);
  freg::fft<float, +1, N1>(v, w);
  float vr[N1];
  load_vrow<N1>(V, vr);
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    w[k].x *= vr[k];
    w[k].y *= vr[k];
  }
  freg::fft<float, -1, N1>(w, v);
  const int hi0 = N1 - (p.nx - p.nxl);
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    if (k < p.nxl) p.Q[y * p.sx + k] = v[k];
    else if (k >= hi0) p.Q[y * p.sx + k - hi0 + p.nxl] = v[k];
  }
}

__device__ __forceinline__ PlaneLds plane_of(const CandDesc& cd, cplx<float>* base) {
  PlaneLds p;
  p.Q = base;
  p.nx = cd.pl_nx;
  p.nxl = cd.pl_nxl;
  p.sx = cd.pl_sx;
  return p;
}

// Sticks of plane (pair, z) into the compact plane (zeros elsewhere).
__device__ __forceinline__ void scatter_sticks(const CandDesc& cd, const PlaneLds& p,
                                               const cplx<float>* __restrict__ st, int lane) {
  const int n = cd.N2 * p.sx;
  for (int e = lane; e < n; e += 64) p.Q[e] = {0.f, 0.f};
  __syncthreads();
  // batches of 4 sticks per lane: loads first, then the LDS stores
  for (int s0 = lane; s0 < cd.nst; s0 += 256) {
    int xy[4];
    cplx<float> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + 64 * u;
      xy[u] = s < cd.nst ? cd.stick_xy[s] : 0;
      v[u] = s < cd.nst ? st[s] : cplx<float>{0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (s0 + 64 * u < cd.nst) p.Q[(xy[u] >> 16) * p.sx + col_of_x(p, cd.N1, xy[u] & 0xFFFF)] = v[u];
  }
  __syncthreads();
}

// H psi, local part, of one plane of one band pair: sticks are read, and
// overwritten by the forward transform of V_eff times the inverse transform.
template <int NMAX>
__global__ void __launch_bounds__(64, 2) k_plane_hpsi_reg(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int z = blockIdx.x, pair = blockIdx.y;
  if (z >= cd.N3 || pair >= cd.npair) return;
  extern __shared__ __align__(16) char smem[];
  PlaneLds p = plane_of(cd, (cplx<float>*)smem);
  const int lane = threadIdx.x;
  cplx<float>* st = (cplx<float>*)cd.sticks + ((size_t)pair * cd.N3 + z) * cd.nst;
  scatter_sticks(cd, p, st, lane);
  column_pass_rt<+1, NMAX>(p, cd.N2, lane);
  __syncthreads();
  // strides re-declared opaque between phases: per-line offsets are then
  // recomputed in each phase instead of being held across all of them
  asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl));
  if (lane < cd.N2) {
    const float* V = (const float*)cd.veff_t + ((size_t)z * cd.N2 + lane) * cd.N1;
    switch (cd.N1) {
#define SGO_CASE(N)                       \
  case N:                                 \
    if constexpr (N <= NMAX) row_pass_hpsi<N>(p, lane, V);         \
    break;
      SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
      default:
        break;
    }
  }
  __syncthreads();
  asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl));
  column_pass_rt<-1, NMAX>(p, cd.N2, lane);
  __syncthreads();
  for (int s0 = lane; s0 < cd.nst; s0 += 256) {
    int xy[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xy[u] = s0 + 64 * u < cd.nst ? cd.stick_xy[s0 + 64 * u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (s0 + 64 * u < cd.nst)
        st[s0 + 64 * u] = p.Q[(xy[u] >> 16) * p.sx + col_of_x(p, cd.N1, xy[u] & 0xFFFF)];
  }
}

// H psi, local part, of a group of consecutive z-planes of one band pair
// per workgroup of four wavefronts.  The line transforms of all the planes
// of the group are spread over the 256 lanes, so that planes whose line
// counts leave part of a wavefront idle (say 35 active columns and 48 rows
// on 64 lanes) share the lanes.  Each line is transformed exactly as in
// k_plane_hpsi_reg; the planes lie one after another in LDS, each compact
// (N2 rows of stride sx).
constexpr int kPlaneGroupThreads = 256;
constexpr int kPlaneGroupMax = 8;  // largest group (SGO_PLANE_GROUP)

template <int N2, int S>
__device__ __forceinline__ void column_lines(cplx<float>* Q0, int pstride, int sx, int nx, int nlines,
                                             int tid) {
  for (int l = tid; l < nlines; l += kPlaneGroupThreads) {
    // strides re-declared opaque per line: the per-element offsets are
    // recomputed in each pass of the loop instead of all being hoisted
    int sxl = sx, psl = pstride;
    asm volatile("" : "+s"(sxl), "+s"(psl));
    const int j = l / nx, c = l - j * nx;
    cplx<float>* q = Q0 + j * psl + c;
    cplx<float> v[N2], w[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) v[k] = q[k * sxl];
    freg::fft<float, S, N2>(v, w);
#pragma unroll
    for (int k = 0; k < N2; ++k) q[k * sxl] = w[k];
  }
}

template <int S, int NMAX>
__device__ __forceinline__ void column_lines_rt(cplx<float>* Q0, int pstride, int sx, int nx, int N2,
                                                int nlines, int tid) {
  switch (N2) {
#define SGO_CASE(N)                                                 \
  case N:                                                           \
    if constexpr (N <= NMAX) column_lines<N, S>(Q0, pstride, sx, nx, nlines, tid);           \
    break;
    SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
    default:
      break;
  }
}

template <int N1>
__device__ __forceinline__ void row_lines_hpsi(const PlaneLds& p0, int pstride, int N2, int nlines,
                                               const float* __restrict__ V0, int tid) {
  for (int l = tid; l < nlines; l += kPlaneGroupThreads) {
    const int j = l / N2, y = l - j * N2;
    PlaneLds p = p0;
    int psl = pstride;
    asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl), "+s"(psl));
    p.Q = p0.Q + j * psl;
    row_pass_hpsi<N1>(p, y, V0 + ((size_t)j * N2 + y) * N1);
  }
}

template <int NMAX>
__global__ void __launch_bounds__(kPlaneGroupThreads, 2) k_plane_hpsi_group(
    const CandDesc* __restrict__ cds, int group) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int z0 = blockIdx.x * group, pair = blockIdx.y;
  if (z0 >= cd.N3 || pair >= cd.npair) return;
  const int np = min(group, cd.N3 - z0);
  extern __shared__ __align__(16) char smem[];
  PlaneLds p = plane_of(cd, (cplx<float>*)smem);
  const int tid = threadIdx.x;
  const int N1 = cd.N1, N2 = cd.N2, nst = cd.nst;
  const int pstride = N2 * p.sx;
  cplx<float>* st = (cplx<float>*)cd.sticks + ((size_t)pair * cd.N3 + z0) * nst;
  // sticks of the np planes into the compact planes (zeros elsewhere); the
  // stick positions are read once per batch and serve every plane
  for (int e = tid; e < np * pstride; e += kPlaneGroupThreads) p.Q[e] = {0.f, 0.f};
  __syncthreads();
  // every plane's stick values of a batch are loaded before any is stored,
  // so the group waits for one memory latency per batch, not one per plane
  for (int s0 = tid; s0 < nst; s0 += 4 * kPlaneGroupThreads) {
    int off[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + kPlaneGroupThreads * u;
      const int xy = s < nst ? cd.stick_xy[s] : 0;
      off[u] = (xy >> 16) * p.sx + col_of_x(p, N1, xy & 0xFFFF);
    }
    cplx<float> v[kPlaneGroupMax][4];
#pragma unroll
    for (int j = 0; j < kPlaneGroupMax; ++j)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = s0 + kPlaneGroupThreads * u;
        v[j][u] = (j < np && s < nst) ? st[(size_t)j * nst + s] : cplx<float>{0.f, 0.f};
      }
#pragma unroll
    for (int j = 0; j < kPlaneGroupMax; ++j)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j < np && s0 + kPlaneGroupThreads * u < nst) p.Q[j * pstride + off[u]] = v[j][u];
  }
  __syncthreads();
  column_lines_rt<+1, NMAX>(p.Q, pstride, p.sx, p.nx, N2, np * p.nx, tid);
  __syncthreads();
  asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl));
  {
    const float* V0 = (const float*)cd.veff_t + (size_t)z0 * N2 * N1;
    switch (N1) {
#define SGO_CASE(N)                                              \
  case N:                                                        \
    if constexpr (N <= NMAX) row_lines_hpsi<N>(p, pstride, N2, np * N2, V0, tid);         \
    break;
      SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
      default:
        break;
    }
  }
  __syncthreads();
  asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl));
  column_lines_rt<-1, NMAX>(p.Q, pstride, p.sx, p.nx, N2, np * p.nx, tid);
  __syncthreads();
  for (int s0 = tid; s0 < nst; s0 += 4 * kPlaneGroupThreads) {
    int off[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + kPlaneGroupThreads * u;
      const int xy = s < nst ? cd.stick_xy[s] : 0;
      off[u] = (xy >> 16) * p.sx + col_of_x(p, N1, xy & 0xFFFF);
    }
    for (int j = 0; j < np; ++j) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = s0 + kPlaneGroupThreads * u;
        if (s < nst) st[(size_t)j * nst + s] = p.Q[j * pstride + off[u]];
      }
    }
  }
}

// Density of one plane summed over a chunk of band pairs,
// part[chunk][z][y][x] = sum_pairs f_a Re(u)^2 + f_b Im(u)^2 (u = psi_a + i psi_b,
// unnormalised), accumulated in FP32 in LDS over the chunk's band pairs (row
// stride N1 | 1); the chunks are summed in FP64 by k_density_finalize.
template <int N1>
__device__ __forceinline__ void row_pass_density(const PlaneLds& p, int y, float* acc, double fa,
                                                 double fb) {
  cplx<float> v[N1], w[N1];
  load_row<N1>(p, y, v);
  freg::fft<float, +1, N1>(v, w);
  // this pair's contribution, accumulated in FP32 over the chunk's band
  // pairs (a few per chunk; the chunks are summed in FP64 afterwards) in
  // groups of 8 (a scheduling fence per group keeps the accumulator loads
  // from all being hoisted at once)
  const float fa32 = (float)fa, fb32 = (float)fb;
  float* a = acc + y * (N1 | 1);
  freg::static_for<0, (N1 + 7) / 8>([&](auto q) {
    constexpr int K0 = 8 * decltype(q)::value;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = K0; k < (K0 + 8 < N1 ? K0 + 8 : N1); ++k)
      a[k] += fa32 * w[k].x * w[k].x + fb32 * w[k].y * w[k].y;
  });
}

template <int NMAX>
__global__ void __launch_bounds__(64, 2) k_plane_density_reg(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int z = blockIdx.x, chunk = blockIdx.y;
  if (z >= cd.N3 || chunk >= cd.ndens_chunk) return;
  extern __shared__ __align__(16) char smem[];
  const PlaneLds p_outer = plane_of(cd, (cplx<float>*)smem);
  float* acc = (float*)(smem + (size_t)cd.N2 * p_outer.sx * sizeof(cplx<float>));
  const int lane = threadIdx.x;
  const int N1 = cd.N1, N2 = cd.N2, ar = N1 | 1;
  for (int e = lane; e < N2 * ar; e += 64) acc[e] = 0.f;
  const int per = (cd.npair + cd.ndens_chunk - 1) / cd.ndens_chunk;
  const int p0 = chunk * per, p1 = min(cd.npair, p0 + per);
  for (int pair = p0; pair < p1; ++pair) {
    // the plane strides are re-declared opaque in every iteration, so the
    // per-line offsets of all line lengths are not hoisted out of the loop
    // (they would exhaust the scalar registers)
    PlaneLds p = p_outer;
    asm volatile("" : "+s"(p.sx), "+s"(p.nx), "+s"(p.nxl));
    const cplx<float>* st = (const cplx<float>*)cd.sticks + ((size_t)pair * cd.N3 + z) * cd.nst;
    scatter_sticks(cd, p, st, lane);
    column_pass_rt<+1, NMAX>(p, N2, lane);
    __syncthreads();
    const double fa = cd.occ[2 * pair];
    const double fb = 2 * pair + 1 < cd.nb ? cd.occ[2 * pair + 1] : 0.0;
    if (lane < N2) {
      switch (N1) {
#define SGO_CASE(N)                                   \
  case N:                                             \
    if constexpr (N <= NMAX) row_pass_density<N>(p, lane, acc, fa, fb);        \
    break;
        SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
        default:
          break;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  double* out = cd.dens_part + (size_t)chunk * cd.ntot + (size_t)z * N1 * N2;
  for (int e = lane; e < N1 * N2; e += 64) out[e] = (double)acc[(e / N1) * ar + e % N1];
}

// ------------------------------------------------------------ z transforms
// Register-FFT z passes (FP32): one wavefront per chunk of up to 32 stick
// pairs (at most 64 sticks) of one band pair.  The band coefficients are
// scattered into an LDS tile [stick][z] (row stride N3 | 1) with coalesced
// reads of the half sphere, each lane transforms one stick along z in
// registers, and the sticks buffer [pair][z][stick] is written (or read) one
// 64-stick row per z.
constexpr int kZPairs = 16;
__device__ __forceinline__ int mirror_stick_r(int s) { return s == 0 ? 0 : ((s & 1) ? s + 1 : s - 1); }

template <int N3>
__device__ __forceinline__ void zline_inv(const cplx<float>* __restrict__ row, cplx<float>* out, int nst) {
  cplx<float> v[N3], w[N3];
#pragma unroll
  for (int k = 0; k < N3; ++k) v[k] = row[k];
  freg::fft<float, +1, N3>(v, w);
#pragma unroll
  for (int k = 0; k < N3; ++k) out[(size_t)k * nst] = w[k];
}
template <int N3>
__device__ __forceinline__ void zline_fwd(const cplx<float>* __restrict__ in, int nst, cplx<float>* row) {
  cplx<float> v[N3], w[N3];
#pragma unroll
  for (int k = 0; k < N3; ++k) v[k] = in[(size_t)k * nst];
  freg::fft<float, -1, N3>(v, w);
#pragma unroll
  for (int k = 0; k < N3; ++k) row[k] = w[k];
}

struct ZChunk {
  int q0, q1, s0, nloc;
};
__device__ __forceinline__ ZChunk zchunk(const CandDesc& cd, int c) {
  ZChunk z;
  z.q0 = c * kZPairs;
  z.q1 = min(z.q0 + kZPairs, cd.nsp);
  z.s0 = z.q0 == 0 ? 0 : 2 * z.q0 - 1;
  z.nloc = 2 * z.q1 - 1 - z.s0;
  return z;
}

template <int NMAX>
__global__ void __launch_bounds__(64, 2) k_z_inverse_reg(const CandDesc* __restrict__ cds, int src) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int pair = blockIdx.y;
  if (pair >= cd.npair || (int)blockIdx.x * kZPairs >= cd.nsp) return;
  const ZChunk ch = zchunk(cd, blockIdx.x);
  const int N3 = cd.N3, S = N3 | 1, lane = threadIdx.x;
  extern __shared__ __align__(16) char smem[];
  cplx<float>* A = (cplx<float>*)smem;
  for (int e = lane; e < ch.nloc * S; e += 64) A[e] = {0.f, 0.f};
  __syncthreads();
  const float* base = (const float*)(src == W_X ? cd.X : (src == W_D ? cd.D : cd.HX));
  const float* xa = base + (size_t)(2 * pair) * cd.Kp;
  const bool hasb = 2 * pair + 1 < cd.nb;
  const float* xb = base + (size_t)(2 * pair + 1) * cd.Kp;
  const int g0 = cd.sp_off[ch.q0], g1 = cd.sp_off[ch.q1];
  // batches of 4 coefficients per lane: loads first, then the LDS stores
  for (int gb = g0 + lane; gb < g1; gb += 256) {
    int meta[4];
    cplx<float> ca[4], cb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int g = gb + 64 * u;
      const bool ok = g < g1;
      meta[u] = ok ? cd.gmeta[g] : 0;
      ca[u] = ok ? unpack_coef(xa, g) : cplx<float>{0.f, 0.f};
      cb[u] = (ok && hasb) ? unpack_coef(xb, g) : cplx<float>{0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int g = gb + 64 * u;
      if (g >= g1) continue;
      const int st = meta[u] & 0xFFFFF, z = meta[u] >> 20;
      A[(st - ch.s0) * S + z] = {ca[u].x - cb[u].y, ca[u].y + cb[u].x};  // c_a + i c_b
      if (g != 0) {
        const int sm = mirror_stick_r(st);
        const int zm = z == 0 ? 0 : N3 - z;
        A[(sm - ch.s0) * S + zm] = {ca[u].x + cb[u].y, cb[u].x - ca[u].y};  // conj c_a + i conj c_b
      }
    }
  }
  __syncthreads();
  if (lane < ch.nloc) {
    cplx<float>* out = (cplx<float>*)cd.sticks + (size_t)pair * N3 * cd.nst + ch.s0 + lane;
    switch (N3) {
#define SGO_CASE(N)                                  \
  case N:                                            \
    if constexpr (N <= NMAX) zline_inv<N>(A + lane * S, out, cd.nst);         \
    break;
      SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
      default:
        break;
    }
  }
}

template <int NMAX>
__global__ void __launch_bounds__(64, 2) k_z_forward_reg(const CandDesc* __restrict__ cds, int src,
                                                         int dst) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int pair = blockIdx.y;
  if (pair >= cd.npair || (int)blockIdx.x * kZPairs >= cd.nsp) return;
  const ZChunk ch = zchunk(cd, blockIdx.x);
  const int N3 = cd.N3, S = N3 | 1, lane = threadIdx.x;
  extern __shared__ __align__(16) char smem[];
  cplx<float>* A = (cplx<float>*)smem;
  if (lane < ch.nloc) {
    const cplx<float>* in = (const cplx<float>*)cd.sticks + (size_t)pair * N3 * cd.nst + ch.s0 + lane;
    switch (N3) {
#define SGO_CASE(N)                                  \
  case N:                                            \
    if constexpr (N <= NMAX) zline_fwd<N>(in, cd.nst, A + lane * S);          \
    break;
      SGO_LINE_SIZES(SGO_CASE)
#undef SGO_CASE
      default:
        break;
    }
  }
  __syncthreads();
  const float sc = (float)(1.0 / (double)cd.ntot);
  const float rt2 = 1.41421356237309504880f;
  const float* xsrc = (const float*)(src == W_X ? cd.X : (src == W_D ? cd.D : cd.HX));
  float* ydst = (float*)(dst == W_HX ? cd.HX : cd.HD);
  const int a = 2 * pair, b = 2 * pair + 1;
  const bool hasb = b < cd.nb;
  const float* xa = xsrc + (size_t)a * cd.Kp;
  const float* xb = xsrc + (size_t)b * cd.Kp;
  float* ya = ydst + (size_t)a * cd.Kp;
  float* yb = ydst + (size_t)b * cd.Kp;
  const int g0 = cd.sp_off[ch.q0], g1 = cd.sp_off[ch.q1];
  // batches of 4 coefficients per lane: all loads of a batch before its stores
  for (int gb = g0 + lane; gb < g1; gb += 256) {
    int meta[4];
    float kin[4];
    float2 xav[4], xbv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int g = gb + 64 * u;
      const bool ok = g < g1;
      meta[u] = ok ? cd.gmeta[g] : 0;
      kin[u] = ok ? (float)cd.kin[g] : 0.f;
      xav[u] = ok ? *(const float2*)(xa + 2 * g) : make_float2(0.f, 0.f);
      xbv[u] = (ok && hasb) ? *(const float2*)(xb + 2 * g) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int g = gb + 64 * u;
      if (g >= g1) continue;
      const int st = meta[u] & 0xFFFFF, z = meta[u] >> 20;
      const int sm = mirror_stick_r(st);
      const int zm = z == 0 ? 0 : N3 - z;
      const cplx<float> W = A[(st - ch.s0) * S + z];
      const cplx<float> Wm = A[(sm - ch.s0) * S + zm];
      // (V psi_a)_G = (W_G + conj W_-G)/2 ; (V psi_b)_G = (W_G - conj W_-G)/(2i)
      const cplx<float> va = {0.5f * (W.x + Wm.x) * sc, 0.5f * (W.y - Wm.y) * sc};
      const cplx<float> vb = {0.5f * (W.y + Wm.y) * sc, -0.5f * (W.x - Wm.x) * sc};
      if (g == 0) {
        *(float2*)ya = make_float2(va.x + kin[u] * xav[u].x, 0.f);
        if (hasb) *(float2*)yb = make_float2(vb.x + kin[u] * xbv[u].x, 0.f);
      } else {
        *(float2*)(ya + 2 * g) = make_float2(rt2 * va.x + kin[u] * xav[u].x, rt2 * va.y + kin[u] * xav[u].y);
        if (hasb)
          *(float2*)(yb + 2 * g) = make_float2(rt2 * vb.x + kin[u] * xbv[u].x, rt2 * vb.y + kin[u] * xbv[u].y);
      }
    }
  }
}

size_t z_reg_lds(const BatchGeom& g) {
  return (size_t)2 * kZPairs * (g.N3max | 1) * sizeof(cplx<float>);
}
// Largest line length a launch must handle: 48 or 64.  The kernels carry
// the line transforms of every length up to it; the 64 class holds the
// longest register-resident lines (and the registers they need), so a
// population whose lines all fit 48 runs the lighter instantiation.
static bool small_lines(const BatchGeom& g) {
  return std::max(g.N1max, std::max(g.N2max, g.N3max)) <= 48;
}

void launch_z_inverse_reg(const LaunchCtx& L, int src) {
  const BatchGeom& g = L.g;
  dim3 gz((g.nsp_max + kZPairs - 1) / kZPairs, g.npair_max, g.ncand);
  prof_before("k_z_inverse", L.stream);
  if (small_lines(g))
    hipLaunchKernelGGL(k_z_inverse_reg<48>, gz, dim3(64), z_reg_lds(g), L.stream, L.desc, src);
  else
    hipLaunchKernelGGL(k_z_inverse_reg<64>, gz, dim3(64), z_reg_lds(g), L.stream, L.desc, src);
  check_launch("k_z_inverse");
  prof_after("k_z_inverse", L.stream);
}
void launch_z_forward_reg(const LaunchCtx& L, int src, int dst) {
  const BatchGeom& g = L.g;
  dim3 gz((g.nsp_max + kZPairs - 1) / kZPairs, g.npair_max, g.ncand);
  prof_before("k_z_forward", L.stream);
  if (small_lines(g))
    hipLaunchKernelGGL(k_z_forward_reg<48>, gz, dim3(64), z_reg_lds(g), L.stream, L.desc, src, dst);
  else
    hipLaunchKernelGGL(k_z_forward_reg<64>, gz, dim3(64), z_reg_lds(g), L.stream, L.desc, src, dst);
  check_launch("k_z_forward");
  prof_after("k_z_forward", L.stream);
}

size_t plane_reg_lds(const BatchGeom& g, bool density) {
  size_t b = (size_t)g.N2max * g.pl_sx_max * sizeof(cplx<float>);
  if (density) b += (size_t)g.N2max * (g.N1max | 1) * sizeof(float);
  return b;
}

size_t plane_group_lds(const BatchGeom& g, int group) {
  return (size_t)group * g.N2max * g.pl_sx_max * sizeof(cplx<float>);
}

int plane_group_size(const BatchGeom& g, size_t lds_per_cu, int forced) {
  // wavefront time per plane, in line-transform rounds of one wavefront:
  // one plane per wavefront takes 2 column rounds and 2 row rounds
  // (ceil(lines / 64) each); a group of P planes on four wavefronts takes
  // 4 x the rounds over 256 lanes, shared by P planes.  Two groups must fit
  // one compute unit's LDS, as two one-plane wavefronts per SIMD do.
  auto rounds = [](int lines, int lanes) { return (lines + lanes - 1) / lanes; };
  const int nx = std::max(1, g.pl_sx_max), N2 = std::max(1, g.N2max);
  const double single = 2.0 * rounds(nx, 64) + 2.0 * rounds(N2, 64);
  int best = 1;
  double best_t = single;
  for (int P = 2; P <= kPlaneGroupMax; ++P) {
    if (2 * plane_group_lds(g, P) > lds_per_cu) break;
    const double t = 4.0 * (2 * rounds(P * nx, kPlaneGroupThreads) +
                            2 * rounds(P * N2, kPlaneGroupThreads)) / P;
    if (forced == P) return P;
    if (t < 0.9 * best_t) {
      best = P;
      best_t = t;
    }
  }
  return forced == 1 ? 1 : best;
}

void launch_plane_hpsi_reg(const LaunchCtx& L) {
  const BatchGeom& g = L.g;
  prof_before("k_plane_hpsi", L.stream);
  if (g.plane_group > 1) {
    dim3 gp((g.N3max + g.plane_group - 1) / g.plane_group, g.npair_max, g.ncand);
    if (small_lines(g))
      hipLaunchKernelGGL(k_plane_hpsi_group<48>, gp, dim3(kPlaneGroupThreads),
                         plane_group_lds(g, g.plane_group), L.stream, L.desc, g.plane_group);
    else
      hipLaunchKernelGGL(k_plane_hpsi_group<64>, gp, dim3(kPlaneGroupThreads),
                         plane_group_lds(g, g.plane_group), L.stream, L.desc, g.plane_group);
  } else {
    dim3 gp(g.N3max, g.npair_max, g.ncand);
    if (small_lines(g))
      hipLaunchKernelGGL(k_plane_hpsi_reg<48>, gp, dim3(64), plane_reg_lds(g, false), L.stream, L.desc);
    else
      hipLaunchKernelGGL(k_plane_hpsi_reg<64>, gp, dim3(64), plane_reg_lds(g, false), L.stream, L.desc);
  }
  check_launch("k_plane_hpsi");
  prof_after("k_plane_hpsi", L.stream);
}

void launch_plane_density_reg(const LaunchCtx& L) {
  const BatchGeom& g = L.g;
  dim3 gp(g.N3max, g.dens_chunks, g.ncand);
  prof_before("k_plane_density", L.stream);
  if (small_lines(g))
    hipLaunchKernelGGL(k_plane_density_reg<48>, gp, dim3(64), plane_reg_lds(g, true), L.stream, L.desc);
  else
    hipLaunchKernelGGL(k_plane_density_reg<64>, gp, dim3(64), plane_reg_lds(g, true), L.stream, L.desc);
  check_launch("k_plane_density");
  prof_after("k_plane_density", L.stream);
}

void configure_plane_kernels() {
  allow_lds((const void*)k_plane_hpsi_reg<48>);
  allow_lds((const void*)k_plane_hpsi_group<48>);
  allow_lds((const void*)k_plane_density_reg<48>);
  allow_lds((const void*)k_z_inverse_reg<48>);
  allow_lds((const void*)k_z_forward_reg<48>);
  allow_lds((const void*)k_plane_hpsi_reg<64>);
  allow_lds((const void*)k_plane_hpsi_group<64>);
  allow_lds((const void*)k_plane_density_reg<64>);
  allow_lds((const void*)k_z_inverse_reg<64>);
  allow_lds((const void*)k_z_forward_reg<64>);
}

}  // namespace sgo
