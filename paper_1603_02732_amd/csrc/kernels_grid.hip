// FP64 grid-side kernels: full-grid FFT passes, output density and energy
// sums, density residual and Pulay/Kerker mixing (the step of the SCF loop of
// Section 2.4 that combines the output density with the input one),
// potentials, per-geometry setup (local potential and starting density from
// structure factors, Ewald sum), Hellmann-Feynman force sums, occupations,
// and the FP64 subspace solver (Cholesky orthonormalisation + Jacobi
// diagonalisation: the orthogonalisation and subspace-diagonalisation steps
// of Algorithm 1).
#include "device.hpp"
#include "launch.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace sgo {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ int gfreq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// G vector, |G|^2 and membership of the density set D for grid index e of
// the [z][y][x] layout.
struct GPoint {
  double G[3];
  double g2;
  bool inD;
};
__device__ __forceinline__ GPoint gpoint(const CandDesc& cd, int e) {
  const int x = e % cd.N1;
  const int yz = e / cd.N1;
  const int y = yz % cd.N2;
  const int z = yz / cd.N2;
  const int m1 = gfreq(x, cd.N1), m2 = gfreq(y, cd.N2), m3 = gfreq(z, cd.N3);
  GPoint p;
  p.G[0] = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
  p.G[1] = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
  p.G[2] = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
  p.g2 = p.G[0] * p.G[0] + p.G[1] * p.G[1] + p.G[2] * p.G[2];
  p.inD = 2 * abs(m1) < cd.N1 && 2 * abs(m2) < cd.N2 && 2 * abs(m3) < cd.N3;
  return p;
}

// Local pseudopotential transform v_s(G), G != 0 (Coulomb tail included).
__device__ __forceinline__ double vloc_ft(const SpeciesDev& s, double g2) {
  if (s.local_kind == 0) {  // Appelbaum-Hamann form
    const double a = s.p[0], v1 = s.p[1], v2 = s.p[2];
    const double e = exp(-g2 / (4.0 * a));
    return -4.0 * kPi * s.Z / g2 * e +
           pow(kPi / a, 1.5) * e * (v1 + v2 * (1.5 / a - g2 / (4.0 * a * a)));
  }
  const double rl = s.p[0], c1 = s.p[1], c2 = s.p[2];
  const double e = exp(-0.5 * g2 * rl * rl);
  return -4.0 * kPi * s.Z / g2 * e +
         pow(2.0 * kPi, 1.5) * rl * rl * rl * e * (c1 + c2 * (3.0 - g2 * rl * rl));
}
// lim_{G->0} [v_s(G) + 4 pi Z / G^2]
__device__ __forceinline__ double vloc_g0(const SpeciesDev& s) {
  if (s.local_kind == 0) {
    const double a = s.p[0];
    return kPi * s.Z / a + pow(kPi / a, 1.5) * (s.p[1] + 1.5 * s.p[2] / a);
  }
  const double rl = s.p[0];
  return 2.0 * kPi * s.Z * rl * rl + pow(2.0 * kPi, 1.5) * rl * rl * rl * (s.p[1] + 3.0 * s.p[2]);
}

// History slots of SCF iteration `it` (the batch iterates in lockstep; the
// counter lives in device memory so a captured iteration can be replayed).
struct IterSlots {
  int it, cur, nvalid, next;
};
__device__ __forceinline__ IterSlots slots_of(int it, int H) {
  IterSlots s;
  s.it = it;
  s.cur = it % H;
  s.nvalid = min(it + 1, H - 1);
  s.next = (it + 1) % H;
  return s;
}

__device__ __forceinline__ int nblk(const CandDesc& cd) {
  return min(1024, (cd.ntot + kNT - 1) / kNT);
}
// partial-sum regions of the per-iteration grid kernels in red_part
constexpr int kPartDens = 0;      // [nblk][3]  density_finalize
constexpr int kPartRes = 4096;    // [nblk][10] gspace_residual

// ------------------------------------------------------------ full-grid FFT
// Rows along x (contiguous).
__global__ void __launch_bounds__(kNT) k_grid_fft_x(const CandDesc* __restrict__ cds, int sign,
                                                    int rows_per_block) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int N1 = cd.N1, nrows = cd.N2 * cd.N3;
  const int r0 = blockIdx.x * rows_per_block;
  if (r0 >= nrows) return;
  const int nr = min(rows_per_block, nrows - r0);
  extern __shared__ __align__(16) char smem[];
  cplx<double>* tw = (cplx<double>*)smem;
  cplx<double>* A = tw + kMaxFftN;
  cplx<double>* Bf = A + rows_per_block * N1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, N1, tid, nthr);
  cplx<double>* g = cd.zgrid + (size_t)r0 * N1;
  for (int e = tid; e < nr * N1; e += nthr) A[e] = g[e];
  __syncthreads();
  cplx<double>* r = lds_fft(A, Bf, cd.plan[0], nr, 1, N1, tw, sign, tid, nthr);
  for (int e = tid; e < nr * N1; e += nthr) g[e] = r[e];
}

// Columns along y (axis 1) or z (axis 2): each block takes a tile of TX
// consecutive x values, so global accesses stay contiguous in x.
constexpr int kTX = 16;
__global__ void __launch_bounds__(kNT) k_grid_fft_yz(const CandDesc* __restrict__ cds, int axis,
                                                     int sign) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int N1 = cd.N1, N2 = cd.N2, N3 = cd.N3;
  const int ntx = (N1 + kTX - 1) / kTX;
  const int other_n = axis == 1 ? N3 : N2;
  const int tile = blockIdx.x % ntx, other = blockIdx.x / ntx;
  if (other >= other_n) return;
  const int x0 = tile * kTX, tx = min(kTX, N1 - x0);
  const int n = axis == 1 ? N2 : N3;
  const size_t es = axis == 1 ? (size_t)N1 : (size_t)N1 * N2;
  const size_t base = axis == 1 ? (size_t)other * N1 * N2 + x0 : (size_t)other * N1 + x0;
  extern __shared__ __align__(16) char smem[];
  cplx<double>* tw = (cplx<double>*)smem;
  cplx<double>* A = tw + kMaxFftN;
  cplx<double>* Bf = A + kTX * n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, n, tid, nthr);
  const FftPlan& P = cd.plan[axis];
  for (int t = tid; t < tx * n; t += nthr) {
    const int e = t / tx, c = t - e * tx;
    A[c * n + e] = cd.zgrid[base + e * es + c];
  }
  __syncthreads();
  cplx<double>* r = lds_fft(A, Bf, P, tx, 1, n, tw, sign, tid, nthr);
  for (int t = tid; t < tx * n; t += nthr) {
    const int e = t / tx, c = t - e * tx;
    cd.zgrid[base + e * es + c] = r[c * n + e];
  }
}

// --------------------------------------------------------- density / energy
// rho_out(r) = sum of the band-pair chunks / Omega; accumulates
// sum|rho_out - rho_in|, E_xc[rho_out] and int V_eff,in rho_out.
__global__ void __launch_bounds__(kNT) k_density_finalize(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  if ((int)blockIdx.x >= nblk(cd)) return;
  __shared__ double sh[16 * 3];
  double v[3] = {0.0, 0.0, 0.0};
  const double inv_omega = 1.0 / cd.omega;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += nblk(cd) * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < cd.ndens_chunk; ++c) s += cd.dens_part[(size_t)c * cd.ntot + e];
    const double rho = s * inv_omega;
    cd.rho_out_r[e] = rho;
    cd.zgrid[e] = {rho, 0.0};
    v[0] += fabs(rho - cd.rho_in_r[e]);
    const double rc = fmax(rho, 0.0);
    double ex, vx;
    pz81(rc, &ex, &vx);
    v[1] += rc * ex;
    v[2] += cd.veff_r[e] * rho;
  }
  block_sum<3>(v, sh);
  // per-block partial sums; k_scf_control adds them up in a fixed order
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) cd.red_part[kPartDens + 3 * blockIdx.x + k] = v[k];
}

// Pulay history element access (complex FP64, or complex FP32 when
// hist_f32; arithmetic in FP64 either way)
__device__ __forceinline__ cplx<double> hist_ld(const CandDesc& cd, const void* h, size_t i) {
  if (cd.hist_f32) {
    const float2 v = ((const float2*)h)[i];
    return {(double)v.x, (double)v.y};
  }
  return ((const cplx<double>*)h)[i];
}
__device__ __forceinline__ void hist_st(const CandDesc& cd, void* h, size_t i, cplx<double> v) {
  if (cd.hist_f32)
    ((float2*)h)[i] = make_float2((float)v.x, (float)v.y);
  else
    ((cplx<double>*)h)[i] = v;
}

// After the forward FFT of rho_out: rho_out(G), density residual into the
// history, Hartree and local energies, and the residual dot products of the
// Pulay matrix row of this iteration.
__global__ void __launch_bounds__(kNT) k_gspace_residual(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  if ((int)blockIdx.x >= nblk(cd)) return;
  const IterSlots sl = slots_of(*cd.iter_state, cd.hist_len);
  const int cur = sl.cur, nvalid = sl.nvalid;
  __shared__ double sh[16 * 10];
  const int H = cd.hist_len;
  double v[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) v[k] = 0.0;
  const double inv_n = 1.0 / cd.ntot;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += nblk(cd) * blockDim.x) {
    const cplx<double> z = cd.zgrid[e];
    const cplx<double> rg = {z.x * inv_n, z.y * inv_n};
    cd.rho_out_G[e] = rg;
    const cplx<double> rin = hist_ld(cd, cd.hist_in, (size_t)cur * cd.ntot + e);
    const cplx<double> R = {rg.x - rin.x, rg.y - rin.y};
    hist_st(cd, cd.hist_res, (size_t)cur * cd.ntot + e, R);
    const GPoint p = gpoint(cd, e);
    if (p.inD) {
      if (p.g2 > 0.0) v[0] += 4.0 * kPi * (rg.x * rg.x + rg.y * rg.y) / p.g2;
      const cplx<double> vl = cd.vloc_G[e];
      v[1] += vl.x * rg.x + vl.y * rg.y;
    }
#pragma unroll
    for (int l = 0; l < kMaxHist; ++l) {
      if (l < nvalid) {
        const int slot = (cur - l + H) % H;
        const cplx<double> Rl = hist_ld(cd, cd.hist_res, (size_t)slot * cd.ntot + e);
        v[2 + l] += Rl.x * R.x + Rl.y * R.y;
      }
    }
  }
  block_sum<10>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 10; ++k) cd.red_part[kPartRes + 10 * blockIdx.x + k] = v[k];
}

// Pulay coefficients, total free energy, convergence flags (one block per
// candidate; the work is a few dozen scalars).
__global__ void k_scf_control(const CandDesc* __restrict__ cds, double tol_e_atom, double tol_rho,
                              double res_tol) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  const IterSlots sl = slots_of(*cd.iter_state, cd.hist_len);
  const int cur = sl.cur, nvalid = sl.nvalid, iter = sl.it;
  const int H = cd.hist_len;
  double* sc = cd.scal;
  // the Pulay system lives in LDS (dynamically indexed: in registers it would
  // go to scratch memory); only lane 0 touches it
  __shared__ double A[kMaxHist + 1][kMaxHist + 2];
  __shared__ double x[kMaxHist + 1];
  double ekin_w = 0.0;
  double res_worst = 0.0;
  {
    // block partials of k_density_finalize and k_gspace_residual, summed in
    // a fixed order (one wavefront: lane-strided, then the cross-lane tree)
    const int nbk = nblk(cd);
    double v[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nbk; b += 64) {
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] += cd.red_part[kPartDens + 3 * b + k];
#pragma unroll
      for (int k = 0; k < 10; ++k) v[3 + k] += cd.red_part[kPartRes + 10 * b + k];
    }
#pragma unroll
    for (int k = 0; k < 13; ++k) v[k] = wave_sum(v[k]);
    // band kinetic energy (lane-strided, then the cross-lane tree)
    double ek = 0.0;
    for (int i = threadIdx.x; i < cd.nb; i += 64) ek += cd.occ[i] * cd.bandw[i];
    ekin_w = wave_sum(ek);
    // largest squared occupation-weighted residual (last CG direction) of
    // the bands holding charge, over all 64 lanes before lane 0 goes on alone
    double rw = 0.0;
    if (res_tol > 0.0)
      for (int i = threadIdx.x; i < cd.nb; i += 64)
        if (cd.occ[i] > 1e-6) rw = fmax(rw, 0.25 * cd.occ[i] * cd.occ[i] * cd.resn[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rw = fmax(rw, __shfl_xor(rw, o, 64));
    res_worst = rw;
    if (threadIdx.x != 0) return;
    const double w = cd.omega / cd.ntot;
    sc[S_DRHO] = w * v[0] / fmax(cd.nelec, 1e-30);
    sc[S_EXC] = w * v[1];
    sc[S_VRHO] = w * v[2];
    sc[S_EH] = 0.5 * cd.omega * v[3];
    sc[S_ELOC] = cd.omega * v[4];
    for (int l = 0; l < nvalid; ++l) {
      const int slot = (cur - l + H) % H;
      cd.pulay[cur * kMaxHist + slot] = v[5 + l];
      cd.pulay[slot * kMaxHist + cur] = v[5 + l];
    }
  }
  // Pulay: minimise |sum c_l R_l| with sum c_l = 1
  const int n = nvalid;
  double scale = 0.0;
  for (int l = 0; l < n; ++l) {
    const int sl = (cur - l + H) % H;
    scale = fmax(scale, fabs(cd.pulay[sl * kMaxHist + sl]));
  }
  if (!(scale > 0.0)) scale = 1.0;
  for (int l = 0; l < n; ++l) {
    const int sl = (cur - l + H) % H;
    for (int m = 0; m < n; ++m) {
      const int sm = (cur - m + H) % H;
      A[l][m] = cd.pulay[sl * kMaxHist + sm] / scale;
    }
    A[l][l] += 1e-13;
    A[l][n] = 1.0;
    A[l][n + 1] = 0.0;
  }
  for (int m = 0; m < n; ++m) A[n][m] = 1.0;
  A[n][n] = 0.0;
  A[n][n + 1] = 1.0;
  const int N = n + 1;
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int r = k + 1; r < N; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (piv != k)
      for (int c = 0; c <= N; ++c) {
        const double t = A[k][c];
        A[k][c] = A[piv][c];
        A[piv][c] = t;
      }
    const double d = A[k][k];
    for (int r = k + 1; r < N; ++r) {
      const double f = A[r][k] / d;
      for (int c = k; c <= N; ++c) A[r][c] -= f * A[k][c];
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    double s = A[k][N];
    for (int c = k + 1; c < N; ++c) s -= A[k][c] * x[c];
    x[k] = s / A[k][k];
  }
  bool ok = true;
  for (int l = 0; l < n; ++l) ok = ok && isfinite(x[l]);
  for (int l = 0; l < n; ++l) cd.coef[(cur - l + H) % H] = ok ? x[l] : (l == 0 ? 1.0 : 0.0);
  // energies
  const double ekin = ekin_w;
  const double ekn = sc[S_EBAND] - sc[S_VRHO];
  const double ent = -cd.sigma * sc[S_ENTROPY];
  const double etot = ekn + sc[S_ELOC] + sc[S_EH] + sc[S_EXC] + sc[S_EEW] + ent;
  sc[S_EKIN] = ekin;
  sc[S_ENL] = ekn - ekin;
  sc[S_ENTROPY_TERM] = ent;
  const double de = iter > 0 ? fabs(etot - sc[S_EPREV]) : 1e300;
  sc[S_DE] = de;
  sc[S_EPREV] = etot;
  sc[S_ETOT] = etot;
  sc[S_ITER] = iter + 1;
  // with a residual gate, self-consistency also asks the bands holding
  // charge to be eigenvectors of the last V_eff: occupation-weighted
  // residual (as of the last CG direction) <= max(res_tol, 0.1 sqrt(tol_e
  // per atom))
  bool bands_ok = true;
  if (res_tol > 0.0) {
    const double tau = fmax(res_tol, 0.1 * sqrt(tol_e_atom));
    bands_ok = res_worst <= tau * tau;
  }
  sc[S_CONV] = (iter > 0 && de < tol_e_atom * cd.nat && sc[S_DRHO] < tol_rho && bands_ok) ? 1.0 : 0.0;
  if (!isfinite(etot) || !isfinite(sc[S_DRHO])) sc[S_ERR] = 1.0;
}

// Mixed input density in G space and the potential V(G) = V_loc + V_H on D,
// packed as V(G) + i rho_in(G) for one inverse transform of both.
__global__ void __launch_bounds__(kNT) k_mix(const CandDesc* __restrict__ cds, int initial,
                                             double alpha, double q0) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int H = cd.hist_len;
  // mixes the output of the previous iteration (the counter was advanced
  // after it) into the input of the current one; the first input is rho_0
  const IterSlots sl = slots_of(*cd.iter_state - 1, H);
  const int cur = sl.cur, nvalid = sl.nvalid, next = initial ? 0 : sl.next;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += gridDim.x * blockDim.x) {
    const GPoint p = gpoint(cd, e);
    cplx<double> rho;
    if (initial) {
      rho = cd.rho0_G[e];
    } else {
      const double kk = p.g2 > 0.0 ? p.g2 / (p.g2 + q0 * q0) : 0.0;
      rho = {0.0, 0.0};
      for (int l = 0; l < nvalid; ++l) {
        const int sl = (cur - l + H) % H;
        const double c = cd.coef[sl];
        const cplx<double> ri = hist_ld(cd, cd.hist_in, (size_t)sl * cd.ntot + e);
        const cplx<double> rr = hist_ld(cd, cd.hist_res, (size_t)sl * cd.ntot + e);
        rho.x += c * (ri.x + alpha * kk * rr.x);
        rho.y += c * (ri.y + alpha * kk * rr.y);
      }
    }
    hist_st(cd, cd.hist_in, (size_t)next * cd.ntot + e, rho);
    cplx<double> V = {0.0, 0.0};
    if (p.inD) {
      V = cd.vloc_G[e];
      if (p.g2 > 0.0) {
        V.x += 4.0 * kPi * rho.x / p.g2;
        V.y += 4.0 * kPi * rho.y / p.g2;
      }
    }
    cd.zgrid[e] = {V.x - rho.y, V.y + rho.x};
  }
}

// --------------------------------------------------------------- setup
// V_loc(G) = (1/Omega) sum_I v_s(|G|) e^{-iG.R_I} and the starting density
// rho_0(G) = (1/Omega) sum_I Z_I e^{-G^2 w^2/2} e^{-iG.R_I} on D.
__global__ void __launch_bounds__(kNT) k_setup_grid(const CandDesc* __restrict__ cds,
                                                    const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const double io = 1.0 / cd.omega;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += gridDim.x * blockDim.x) {
    const GPoint p = gpoint(cd, e);
    cplx<double> vl = {0.0, 0.0}, r0 = {0.0, 0.0};
    if (p.inD) {
      double ztot = 0.0;
      for (int I = 0; I < cd.nat; ++I) {
        const SpeciesDev& s = sp[cd.spec[I]];
        double sn, cs;
        sincos(-(p.G[0] * cd.pos[3 * I] + p.G[1] * cd.pos[3 * I + 1] + p.G[2] * cd.pos[3 * I + 2]),
               &sn, &cs);
        const double v = p.g2 > 0.0 ? vloc_ft(s, p.g2) : vloc_g0(s);
        vl.x += v * cs;
        vl.y += v * sn;
        const double a = s.Z * exp(-0.5 * p.g2 * s.rho0_width * s.rho0_width);
        r0.x += a * cs;
        r0.y += a * sn;
        ztot += s.Z;
      }
      if (p.g2 == 0.0) r0.x += cd.nelec - ztot;
    }
    cd.vloc_G[e] = {vl.x * io, vl.y * io};
    cd.rho0_G[e] = {r0.x * io, r0.y * io};
  }
}

// Ewald, reciprocal part: S(G) = sum_J Z_J e^{iG.R_J} on the enumerated box
// and E_recip = (2 pi/Omega) sum_{0<|G|<=gcut} e^{-G^2/4eta^2}/G^2 |S|^2.
__global__ void __launch_bounds__(kNT) k_ewald_recip(const CandDesc* __restrict__ cds,
                                                     const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int nb = min(1024, (cd.ew_ng + kNT - 1) / kNT);
  if ((int)blockIdx.x >= nb) return;
  __shared__ double sh[16];
  const int w1 = 2 * cd.ew_m[0] + 1, w2 = 2 * cd.ew_m[1] + 1;
  const double eta = cd.ew_eta;
  double v[1] = {0.0};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cd.ew_ng; t += nb * blockDim.x) {
    const int m1 = t % w1 - cd.ew_m[0];
    const int m2 = (t / w1) % w2 - cd.ew_m[1];
    const int m3 = t / (w1 * w2) - cd.ew_m[2];
    const double G0 = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
    const double G1 = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
    const double G2 = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
    const double g2 = G0 * G0 + G1 * G1 + G2 * G2;
    cplx<double> S = {0.0, 0.0};
    if (g2 > 0.0 && g2 <= cd.ew_gcut * cd.ew_gcut) {
      for (int J = 0; J < cd.nat; ++J) {
        double sn, cs;
        sincos(G0 * cd.pos[3 * J] + G1 * cd.pos[3 * J + 1] + G2 * cd.pos[3 * J + 2], &sn, &cs);
        const double Z = sp[cd.spec[J]].Z;
        S.x += Z * cs;
        S.y += Z * sn;
      }
      v[0] += exp(-g2 / (4.0 * eta * eta)) / g2 * (S.x * S.x + S.y * S.y);
    }
    cd.ewS[t] = S;
  }
  block_sum<1>(v, sh);
  double out[1];
  if (grid_sum_last<1>(v, cd.red_part, &cd.tickets[kTicketGrid + 2], nb, blockIdx.x, out, sh)) {
    if (threadIdx.x == 0) cd.scal[S_EWRECIP] = 2.0 * kPi / cd.omega * out[0];
  }
}

// Ewald, per atom I: real-space pair sum over images, reciprocal force from
// S(G); the last block adds self and background terms to the total.
__global__ void __launch_bounds__(kNT) k_ewald_atom(const CandDesc* __restrict__ cds,
                                                    const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int I = blockIdx.x;
  if (I >= cd.nat) return;
  __shared__ double sh[16 * 4];
  const double eta = cd.ew_eta;
  const double ZI = sp[cd.spec[I]].Z;
  const double RI0 = cd.pos[3 * I], RI1 = cd.pos[3 * I + 1], RI2 = cd.pos[3 * I + 2];
  const int n1 = 2 * cd.ew_n[0] + 1, n2 = 2 * cd.ew_n[1] + 1;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // energy, Fx, Fy, Fz
  const double rc2 = cd.ew_rcut * cd.ew_rcut;
  const long total = (long)cd.nat * cd.ew_nimg;
  for (long t = threadIdx.x; t < total; t += blockDim.x) {
    const int J = (int)(t / cd.ew_nimg);
    const int im = (int)(t - (long)J * cd.ew_nimg);
    const int a = im % n1 - cd.ew_n[0];
    const int b = (im / n1) % n2 - cd.ew_n[1];
    const int c = im / (n1 * n2) - cd.ew_n[2];
    const double d0 = RI0 - cd.pos[3 * J] + a * cd.A[0] + b * cd.A[3] + c * cd.A[6];
    const double d1 = RI1 - cd.pos[3 * J + 1] + a * cd.A[1] + b * cd.A[4] + c * cd.A[7];
    const double d2 = RI2 - cd.pos[3 * J + 2] + a * cd.A[2] + b * cd.A[5] + c * cd.A[8];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 < 1e-24 || r2 > rc2) continue;
    const double r = sqrt(r2);
    const double ZZ = ZI * sp[cd.spec[J]].Z;
    const double ec = erfc(eta * r);
    v[0] += 0.5 * ZZ * ec / r;
    const double dphi = ec / r2 + 2.0 * eta / sqrt(kPi) * exp(-eta * eta * r2) / r;
    const double f = ZZ * dphi / r;
    v[1] += f * d0;
    v[2] += f * d1;
    v[3] += f * d2;
  }
  const int w1 = 2 * cd.ew_m[0] + 1, w2 = 2 * cd.ew_m[1] + 1;
  for (int t = threadIdx.x; t < cd.ew_ng; t += blockDim.x) {
    const int m1 = t % w1 - cd.ew_m[0];
    const int m2 = (t / w1) % w2 - cd.ew_m[1];
    const int m3 = t / (w1 * w2) - cd.ew_m[2];
    const double G0 = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
    const double G1 = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
    const double G2 = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
    const double g2 = G0 * G0 + G1 * G1 + G2 * G2;
    if (!(g2 > 0.0) || g2 > cd.ew_gcut * cd.ew_gcut) continue;
    const cplx<double> S = cd.ewS[t];
    double sn, cs;
    sincos(G0 * RI0 + G1 * RI1 + G2 * RI2, &sn, &cs);
    // Im[conj(S) e^{iG.R_I}]
    const double im = S.x * sn - S.y * cs;
    const double w = 4.0 * kPi / cd.omega * ZI * exp(-g2 / (4.0 * eta * eta)) / g2 * im;
    v[1] += w * G0;
    v[2] += w * G1;
    v[3] += w * G2;
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0) {
    cd.force_ew[3 * I] = v[1];
    cd.force_ew[3 * I + 1] = v[2];
    cd.force_ew[3 * I + 2] = v[3];
  }
  double e1[1] = {v[0]};
  double out[1];
  if (grid_sum_last<1>(e1, cd.red_part + 64, &cd.tickets[kTicketGrid + 3], cd.nat, I, out, sh)) {
    if (threadIdx.x == 0) {
      double z2 = 0.0, zs = 0.0;
      for (int J = 0; J < cd.nat; ++J) {
        const double Z = sp[cd.spec[J]].Z;
        z2 += Z * Z;
        zs += Z;
      }
      const double eself = -eta / sqrt(kPi) * z2;
      const double ebg = -kPi * zs * zs / (2.0 * cd.omega * eta * eta);
      cd.scal[S_EEW] = out[0] + cd.scal[S_EWRECIP] + eself + ebg;
    }
  }
}

// ------------------------------------------------------------------ forces
// F_loc,I = sum_{G in D, G != 0} G v_s(|G|) Im[e^{iG.R_I} rho(G)].
__global__ void __launch_bounds__(kNT) k_force_local(const CandDesc* __restrict__ cds,
                                                     const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int I = blockIdx.x;
  if (I >= cd.nat) return;
  __shared__ double sh[16 * 3];
  const SpeciesDev& s = sp[cd.spec[I]];
  const double R0 = cd.pos[3 * I], R1 = cd.pos[3 * I + 1], R2 = cd.pos[3 * I + 2];
  double v[3] = {0.0, 0.0, 0.0};
  for (int e = threadIdx.x; e < cd.ntot; e += blockDim.x) {
    const GPoint p = gpoint(cd, e);
    if (!p.inD || !(p.g2 > 0.0)) continue;
    const double vs = vloc_ft(s, p.g2);
    double sn, cs;
    sincos(p.G[0] * R0 + p.G[1] * R1 + p.G[2] * R2, &sn, &cs);
    const cplx<double> r = cd.rho_out_G[e];
    const double im = vs * (cs * r.y + sn * r.x);
    v[0] += p.G[0] * im;
    v[1] += p.G[1] * im;
    v[2] += p.G[2] * im;
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    cd.force_part[3 * I] = v[0];
    cd.force_part[3 * I + 1] = v[1];
    cd.force_part[3 * I + 2] = v[2];
  }
}

// Total force: local + nonlocal (-2 sum_i f_i sum_{p on I} h_p P dP) + Ewald.
__global__ void k_force_finalize(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  for (int t = threadIdx.x; t < 3 * cd.nat; t += blockDim.x) {
    const int I = t / 3, a = t - 3 * I;
    double fnl = 0.0;
    for (int p = 0; p < cd.nproj; ++p) {
      if (cd.proj_atom[p] != I) continue;
      double s = 0.0;
      for (int i = 0; i < cd.nb; ++i) {
        const double* w = cd.nlwork + ((size_t)p * cd.nb + i) * 4;
        s += cd.occ[i] * w[0] * w[1 + a];
      }
      fnl += -2.0 * cd.hproj[p] * s;
    }
    cd.force_part[3 * cd.nat + t] = fnl;
    cd.force[t] = cd.force_part[t] + fnl + cd.force_ew[t];
  }
}

// ------------------------------------------------------------------ stress
// d v_s / d(G^2) for G != 0, from the transforms in vloc_ft.
__device__ __forceinline__ double vloc_dq(const SpeciesDev& s, double q) {
  if (s.local_kind == 0) {
    const double a = s.p[0], v1 = s.p[1], v2 = s.p[2];
    const double e = exp(-q / (4.0 * a)), de = -e / (4.0 * a);
    const double coul = -4.0 * kPi * s.Z * (de / q - e / (q * q));
    const double A = pow(kPi / a, 1.5);
    return coul + A * (de * (v1 + v2 * (1.5 / a - q / (4.0 * a * a))) - e * v2 / (4.0 * a * a));
  }
  const double rl = s.p[0], c1 = s.p[1], c2 = s.p[2];
  const double e = exp(-0.5 * q * rl * rl), de = -0.5 * rl * rl * e;
  const double coul = -4.0 * kPi * s.Z * (de / q - e / (q * q));
  const double A = pow(2.0 * kPi, 1.5) * rl * rl * rl;
  return coul + A * (de * (c1 + c2 * (3.0 - q * rl * rl)) - e * c2 * rl * rl);
}

// Density-side stress sums per block (fixed basis; Omega rho(G) and G.R are
// strain invariant):
//   v[0..5]  sum_{D, G!=0} 4 pi |rho(G)|^2 G_a G_b / G^4         (Hartree)
//   v[6..11] -2 sum_{D, G!=0} sum_I v_I'(G^2) G_a G_b Re(e^{iG.R_I} rho(G))  (local)
//   v[12]    sum_{D, G!=0} 4 pi |rho(G)|^2 / G^2,  v[13] sum_D Re(conj V_loc(G) rho(G))
//   v[14]    sum_r (e_xc - v_xc) rho  (LDA volume term)
__global__ void __launch_bounds__(kNT) k_stress_grid(const CandDesc* __restrict__ cds,
                                                     const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  __shared__ double sh[16 * 16];
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < cd.ntot; e += stride) {
    const GPoint p = gpoint(cd, e);
    if (p.inD) {
      const cplx<double> r = cd.rho_out_G[e];
      const cplx<double> vl = cd.vloc_G[e];
      v[13] += vl.x * r.x + vl.y * r.y;
      if (p.g2 > 0.0) {
        const double h = 4.0 * kPi * (r.x * r.x + r.y * r.y) / p.g2;
        v[12] += h;
        add_voigt(v, h / p.g2, p.G);
        double loc = 0.0;
        for (int I = 0; I < cd.nat; ++I) {
          double sn, cs;
          sincos(p.G[0] * cd.pos[3 * I] + p.G[1] * cd.pos[3 * I + 1] + p.G[2] * cd.pos[3 * I + 2],
                 &sn, &cs);
          loc += vloc_dq(sp[cd.spec[I]], p.g2) * (cs * r.x - sn * r.y);
        }
        add_voigt(v + 6, -2.0 * loc, p.G);
      }
    }
    const double rc = fmax(cd.rho_out_r[e], 0.0);
    double ex, vx;
    pz81(rc, &ex, &vx);
    v[14] += rc * (ex - vx);
  }
  block_sum<16>(v, sh);
  if (threadIdx.x == 0) {
    double* o = cd.stwork + stress_layout(cd.nb, cd.nproj, cd.nat).grid + (size_t)16 * blockIdx.x;
    for (int k = 0; k < 16; ++k) o[k] = v[k];
  }
}

// Ewald stress sums for atom I: real-space pairs
//   v[0..5]  (1/2) sum_{J,n} Z_I Z_J phi'(r) d_a d_b / r,  phi = erfc(eta r)/r,
// and the reciprocal points t = I (mod nat) of the enumerated box
//   v[6..11] sum_G |S|^2 w(G) 2 G_a G_b (1/(4 eta^2) + 1/G^2),  v[12] sum_G |S|^2 w(G)
// with w = e^{-G^2/4eta^2}/G^2.
__global__ void __launch_bounds__(kNT) k_stress_ewald(const CandDesc* __restrict__ cds,
                                                      const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.z];
  if (!cd.active) return;
  const int I = blockIdx.x;
  if (I >= cd.nat) return;
  __shared__ double sh[16 * 13];
  double v[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) v[k] = 0.0;
  const double eta = cd.ew_eta;
  const double ZI = sp[cd.spec[I]].Z;
  const int n1 = 2 * cd.ew_n[0] + 1, n2 = 2 * cd.ew_n[1] + 1;
  const double rc2 = cd.ew_rcut * cd.ew_rcut;
  const long total = (long)cd.nat * cd.ew_nimg;
  for (long t = threadIdx.x; t < total; t += blockDim.x) {
    const int J = (int)(t / cd.ew_nimg);
    const int im = (int)(t - (long)J * cd.ew_nimg);
    const int a = im % n1 - cd.ew_n[0];
    const int b = (im / n1) % n2 - cd.ew_n[1];
    const int c = im / (n1 * n2) - cd.ew_n[2];
    double d[3];
    d[0] = cd.pos[3 * I] - cd.pos[3 * J] + a * cd.A[0] + b * cd.A[3] + c * cd.A[6];
    d[1] = cd.pos[3 * I + 1] - cd.pos[3 * J + 1] + a * cd.A[1] + b * cd.A[4] + c * cd.A[7];
    d[2] = cd.pos[3 * I + 2] - cd.pos[3 * J + 2] + a * cd.A[2] + b * cd.A[5] + c * cd.A[8];
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < 1e-24 || r2 > rc2) continue;
    const double r = sqrt(r2);
    const double dphi = -(erfc(eta * r) / r2 + 2.0 * eta / sqrt(kPi) * exp(-eta * eta * r2) / r);
    add_voigt(v, 0.5 * ZI * sp[cd.spec[J]].Z * dphi / r, d);
  }
  const int w1 = 2 * cd.ew_m[0] + 1, w2 = 2 * cd.ew_m[1] + 1;
  const double q4 = 1.0 / (4.0 * eta * eta);
  for (long t = (long)threadIdx.x * cd.nat + I; t < cd.ew_ng; t += (long)blockDim.x * cd.nat) {
    const int m1 = (int)(t % w1) - cd.ew_m[0];
    const int m2 = (int)((t / w1) % w2) - cd.ew_m[1];
    const int m3 = (int)(t / ((long)w1 * w2)) - cd.ew_m[2];
    double G[3];
    G[0] = m1 * cd.B[0] + m2 * cd.B[3] + m3 * cd.B[6];
    G[1] = m1 * cd.B[1] + m2 * cd.B[4] + m3 * cd.B[7];
    G[2] = m1 * cd.B[2] + m2 * cd.B[5] + m3 * cd.B[8];
    const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    if (!(g2 > 0.0) || g2 > cd.ew_gcut * cd.ew_gcut) continue;
    const cplx<double> S = cd.ewS[t];
    const double w = exp(-g2 * q4) / g2 * (S.x * S.x + S.y * S.y);
    v[12] += w;
    add_voigt(v + 6, 2.0 * w * (q4 + 1.0 / g2), G);
  }
  block_sum<13>(v, sh);
  if (threadIdx.x == 0) {
    double* o = cd.stwork + stress_layout(cd.nb, cd.nproj, cd.nat).ew + (size_t)13 * I;
    for (int k = 0; k < 13; ++k) o[k] = v[k];
  }
}

// Assemble sigma = (1/Omega) dE/d eps from the partial sums (fixed order, so
// the result is deterministic).  Writes the symmetric 3x3 total and the
// kinetic, nonlocal, Hartree, local, xc and Ewald parts.  Nonlocal: with
// P = <beta|psi> and Q_ab = <G_a G_b beta|psi>, the strain derivative of the
// projection is dP_ab = -delta_ab P/2 + r_l^2 Q_ab (volume factor and
// Gaussian radial part), and for l = 1, m: -(delta_mb P_a + delta_ma P_b)/2
// from G_m (P_a = projection of the same channel's m = a projector);
// sigma_nl = (2/Omega) sum_i f_i sum_p h_p P dP.
__global__ void __launch_bounds__(kNT) k_stress_finalize(const CandDesc* __restrict__ cds,
                                                         const SpeciesDev* __restrict__ sp) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  __shared__ double sh[16 * 16];
  const StressLayout SL = stress_layout(cd.nb, cd.nproj, cd.nat);
  const double* w = cd.stwork;
  const int nb = cd.nb;
  double a[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    for (int k = 0; k < 6; ++k) a[k] += cd.occ[i] * w[SL.kin + 6 * (size_t)i + k];
  const int va[6] = {0, 1, 2, 1, 0, 0}, vb[6] = {0, 1, 2, 2, 2, 1};
  for (int t = threadIdx.x; t < cd.nproj * nb; t += blockDim.x) {
    const int p = t / nb, i = t - p * nb;
    const double f = cd.occ[i];
    const double* q = w + SL.nl + (size_t)t * 7;
    const double P = q[0];
    const int l = cd.proj_lm[p] >> 2, m = cd.proj_lm[p] & 3;
    const double rl2 = cd.proj_r[p] * cd.proj_r[p];
    double d[6];
    for (int k = 0; k < 6; ++k) d[k] = rl2 * q[1 + k] - (k < 3 ? 0.5 * P : 0.0);
    if (l == 1) {
      const double* q0 = w + SL.nl + ((size_t)(p - m) * nb + i) * 7;
      const double Pm[3] = {q0[0], q0[(size_t)7 * nb], q0[(size_t)14 * nb]};
      for (int k = 0; k < 6; ++k)
        d[k] -= 0.5 * ((m == vb[k] ? Pm[va[k]] : 0.0) + (m == va[k] ? Pm[vb[k]] : 0.0));
    }
    const double c = 2.0 * cd.hproj[p] * f * P;
    for (int k = 0; k < 6; ++k) a[6 + k] += c * d[k];
  }
  block_sum<12>(a, sh);
  double g[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) g[k] = 0.0;
  for (int b = threadIdx.x; b < kStressBlocks; b += blockDim.x)
    for (int k = 0; k < 15; ++k) g[k] += w[SL.grid + 16 * (size_t)b + k];
  block_sum<15>(g, sh);
  double e[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) e[k] = 0.0;
  for (int I = threadIdx.x; I < cd.nat; I += blockDim.x)
    for (int k = 0; k < 13; ++k) e[k] += w[SL.ew + 13 * (size_t)I + k];
  block_sum<13>(e, sh);
  if (threadIdx.x != 0) return;
  const double om = cd.omega, eta = cd.ew_eta;
  double zs = 0.0;
  for (int J = 0; J < cd.nat; ++J) zs += sp[cd.spec[J]].Z;
  const double e_recip = 2.0 * kPi / om * e[12];
  const double e_bg = -kPi * zs * zs / (2.0 * om * eta * eta);
  double part[6][6];
  for (int k = 0; k < 6; ++k) {
    const double dl = k < 3 ? 1.0 : 0.0;
    part[0][k] = -a[k] / om;
    part[1][k] = a[6 + k] / om;
    part[2][k] = g[k] - 0.5 * g[12] * dl;
    part[3][k] = g[6 + k] / om - g[13] * dl;
    part[4][k] = g[14] / cd.ntot * dl;
    part[5][k] = (e[k] + 2.0 * kPi / om * e[6 + k] - (e_recip + e_bg) * dl) / om;
  }
  auto put = [&](double* o, const double* s6) {
    for (int k = 0; k < 6; ++k) {
      o[3 * va[k] + vb[k]] = s6[k];
      o[3 * vb[k] + va[k]] = s6[k];
    }
  };
  double tot[6];
  for (int k = 0; k < 6; ++k) {
    tot[k] = 0.0;
    for (int j = 0; j < 6; ++j) tot[k] += part[j][k];
  }
  put(cd.stress, tot);
  for (int j = 0; j < 6; ++j) put(cd.stress + 9 + 9 * j, part[j]);
}

// ------------------------------------------------------------ occupations
// Fixed: f = 2 on the lowest nocc bands.  Fermi-Dirac: f = 2/(1+e^{(e-mu)/s})
// with mu from 200 bisection steps so that sum f = N_el; entropy
// S = -2 sum [g ln g + (1-g) ln(1-g)], g = f/2.
__global__ void __launch_bounds__(64) k_occupations(const CandDesc* __restrict__ cds) {
  // one wavefront per candidate: all reductions are cross-lane sums
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  const int n = cd.nb, lane = threadIdx.x;
  if (cd.occ_kind == 0) {
    double v = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double f = i < cd.nocc ? 2.0 : 0.0;
      cd.occ[i] = f;
      v += f * cd.eps[i];
    }
    v = wave_sum(v);
    if (lane == 0) {
      cd.scal[S_EBAND] = v;
      cd.scal[S_ENTROPY] = 0.0;
      cd.scal[S_MU] = cd.nocc < n ? 0.5 * (cd.eps[cd.nocc - 1] + cd.eps[cd.nocc]) : cd.eps[n - 1];
    }
    return;
  }
  const double sg = cd.sigma;
  double lo = 1e300, hi = -1e300;
  for (int i = lane; i < n; i += 64) {
    lo = fmin(lo, cd.eps[i]);
    hi = fmax(hi, cd.eps[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  lo -= 40.0 * sg;
  hi += 40.0 * sg;
  for (int it = 0; it < 200; ++it) {
    const double mu = 0.5 * (lo + hi);
    if (mu <= lo || mu >= hi) break;  // interval exhausted in FP64
    double v = 0.0;
    for (int i = lane; i < n; i += 64) v += 2.0 / (1.0 + exp((cd.eps[i] - mu) / sg));
    v = wave_sum(v);
    if (v > cd.nelec) hi = mu;
    else lo = mu;
  }
  const double mu = 0.5 * (lo + hi);
  double v0 = 0.0, v1 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double f = 2.0 / (1.0 + exp((cd.eps[i] - mu) / sg));
    cd.occ[i] = f;
    v0 += f * cd.eps[i];
    const double g = fmax(0.5 * f, 1e-300), gm = fmax(1.0 - 0.5 * f, 1e-300);
    v1 += g * log(g) + gm * log(gm);
  }
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  if (lane == 0) {
    cd.scal[S_EBAND] = v0;
    cd.scal[S_ENTROPY] = -2.0 * v1;
    cd.scal[S_MU] = mu;
  }
}

// ------------------------------------------------- FP64 subspace solver
// mode 1: orthonormalise only:  S = L L^T, M = L^-T.
// mode 3: orthonormalise + Rayleigh-Ritz:  H' = L^-1 H L^-T = V diag(e) V^T,
//         M = L^-T V (columns sorted by ascending e), eps = e.
// New bands are X_new[:, i] = sum_j X[:, j] M[j][i] (Cholesky-QR, i.e.
// Gram-Schmidt in band order, followed by the subspace diagonalisation).
// max_sweeps bounds the Jacobi sweeps (1 gives an approximate rotation for
// intermediate CG steps; the last step of an SCF iteration converges).
constexpr int kSubNT = 512;

// Pair k of round r of the round-robin (circle) schedule on n2 indices:
// index 0 stays fixed, indices 1..n2-1 rotate.  Returns p < q.
// For rounds r < n2 - 1 and pairs k < n2 / 2 both r + k - 1 and
// r + (n2 - 1 - k) - 1 stay below 2 (n2 - 1), so each remainder modulo
// n2 - 1 is one conditional subtraction.
__device__ __forceinline__ void jacobi_pair(int r, int k, int n2, int* p, int* q) {
  const int m = n2 - 1;
  int a = 0, b = 0;
  if (k != 0) {
    a = r + k - 1;
    a = (a >= m ? a - m : a) + 1;
  }
  const int kb = m - k;
  if (kb != 0) {
    b = r + kb - 1;
    b = (b >= m ? b - m : b) + 1;
  }
  *p = min(a, b);
  *q = max(a, b);
}
// Rotation (c, s) that zeroes A[p][q] of the symmetric matrix A:
// theta = (a_qq - a_pp) / (2 a_pq), t = sgn(theta) / (|theta| + sqrt(theta^2 + 1)).
// Entries at rounding level (|a_pq| <= 1e-17 sqrt|a_pp a_qq|) are left alone.
// 1/x and 1/sqrt(x) from the hardware approximations refined by one Newton
// step (about 1 ulp; the rotation only has to be orthogonal to rounding, and
// c^2 + s^2 = 1 holds by construction below).
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x * r, r, 1.5);
}
__device__ __forceinline__ void jacobi_rot(const double* A, int n, int ld, int p, int q, double* c,
                                           double* s) {
  *c = 1.0;
  *s = 0.0;
  if (q >= n) return;
  const double apq = A[p * ld + q];
  const double app = A[p * ld + p], aqq = A[q * ld + q];
  // skip entries at rounding level: |a_pq|^2 <= 1e-34 |a_pp a_qq|
  if (!(apq * apq > 1e-34 * fabs(app * aqq) + 1e-300)) return;
  const double th = 0.5 * (aqq - app) * rcp_nr(apq);
  double t;
  if (fabs(th) > 1e150) {
    t = 0.5 * rcp_nr(th);
  } else {
    const double h = fma(th, th, 1.0);
    const double r = h * rsq_nr(h);  // sqrt(th^2 + 1)
    t = (th >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(th) + r);
  }
  const double cc = rsq_nr(fma(t, t, 1.0));
  *c = cc;
  *s = t * cc;
}

// One work item of a fast Jacobi round: block (P, Q) of H' and columns 2Q,
// 2Q + 1 of V^T's rows of pair P, loaded into registers, then rotated and
// stored.  Every lane of the wavefront calls load and update (the pair
// indices and rotations come from other lanes' registers).
struct JacItem {
  int P, Q, p1, p2, q1, q2;
  bool ok;
  double a11, a12, a21, a22, vp0, vq0, vp1, vq1;
  __device__ __forceinline__ void load(const double* H, int ldh, const double* Vt, int ldv, int n,
                                       int npair, unsigned inv, int nitem, int t, int pk, int qk) {
    ok = t < nitem;
    const int tc = ok ? t : 0;
    P = (int)(((unsigned)tc * inv) >> 20);
    Q = tc - P * npair;
    p1 = __shfl(pk, P);
    p2 = __shfl(qk, P);
    q1 = __shfl(pk, Q);
    q2 = __shfl(qk, Q);
    const bool p2v = p2 < n, q2v = q2 < n;
    const int p2c = p2v ? p2 : p1, q2c = q2v ? q2 : q1;
    a11 = H[p1 * ldh + q1];
    a12 = q2v ? H[p1 * ldh + q2c] : 0.0;
    a21 = p2v ? H[p2c * ldh + q1] : 0.0;
    a22 = (p2v && q2v) ? H[p2c * ldh + q2c] : 0.0;
    const int i0 = min(2 * Q, n - 1), i1 = min(2 * Q + 1, n - 1);
    vp0 = Vt[p1 * ldv + i0];
    vq0 = Vt[p2c * ldv + i0];
    vp1 = Vt[p1 * ldv + i1];
    vq1 = Vt[p2c * ldv + i1];
  }
  __device__ __forceinline__ void update(double* H, int ldh, double* Vt, int ldv, int n, double ck,
                                         double sk) const {
    const double cP = __shfl(ck, P), sP = __shfl(sk, P);
    const double cQ = __shfl(ck, Q), sQ = __shfl(sk, Q);
    if (!ok) return;
    const bool p2v = p2 < n, q2v = q2 < n;
    const double b11 = fma(cP, a11, -(sP * a21)), b21 = fma(sP, a11, cP * a21);
    const double b12 = fma(cP, a12, -(sP * a22)), b22 = fma(sP, a12, cP * a22);
    H[p1 * ldh + q1] = fma(cQ, b11, -(sQ * b12));
    if (q2v) H[p1 * ldh + q2] = fma(sQ, b11, cQ * b12);
    if (p2v) H[p2 * ldh + q1] = fma(cQ, b21, -(sQ * b22));
    if (p2v && q2v) H[p2 * ldh + q2] = fma(sQ, b21, cQ * b22);
    if (p2v && sP != 0.0) {
      const int i = 2 * Q;
      if (i < n) {
        Vt[p1 * ldv + i] = fma(cP, vp0, -(sP * vq0));
        Vt[p2 * ldv + i] = fma(sP, vp0, cP * vq0);
      }
      if (i + 1 < n) {
        Vt[p1 * ldv + i + 1] = fma(cP, vp1, -(sP * vq1));
        Vt[p2 * ldv + i + 1] = fma(sP, vp1, cP * vq1);
      }
    }
  }
};
// Cyclic Jacobi sweeps, in place, for up to 128 indices (64 pairs).  A round
// is a chain of dependent steps (pair indices, loads, rotation, update), and
// one wavefront issues a vector instruction every few cycles, so the round's
// time is that chain's instruction count and memory latency, not its FP64
// work:
//  - a work item is the 2x2 block (row pair P, column pair Q) of H' together
//    with columns 2Q and 2Q + 1 of V^T's rows of pair P: items own disjoint
//    entries, so they update in place; wavefronts without items skip the
//    round;
//  - each wavefront computes the round's rotations itself (lane k: pair
//    k mod npair) and the items read them, and the pair indices, from those
//    lanes' registers; the first items' loads are issued beside the
//    rotations, and one barrier then separates every read of the round's
//    rotation inputs from the first write.
// The updates are written as fma(x, y, -/+ z w) for x y -/+ z w, the rounding
// the compiler gives the two-barrier rounds in k_subspace (used above 128
// bands), so both give the same bits.
// Stops when the off-diagonal norm is below 1e-13 of the diagonal norm;
// returns the sweeps done.
constexpr int kJacFastPairs = 64;
// nthr_norm: the thread stride of the off-diagonal norm's partial sums (the
// block's thread count, or a smaller one whose sums another launch shape
// must reproduce bit for bit)
__device__ int jacobi_sweeps_fast(double* H, int ldh, double* Vt, int ldv, int n, int max_sweeps,
                                  double* sh, int tid, int nthr, int nthr_norm) {
  const int n2 = n + (n & 1), npair = n2 / 2, m = n2 - 1;
  const int lane = tid & 63;
  // item t = P npair + Q; t / npair as a multiply-shift (exact for t < 4096,
  // npair <= 64)
  const int nitem = npair * npair;
  const unsigned inv = (1u << 20) / (unsigned)npair + 1u;
  const int kl = lane % npair;
  const bool has_items = (tid & ~63) < nitem;
  int nsweep = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // the norms in the two-barrier form's order (the same sweep counts)
    double v[2] = {0.0, 0.0};
    if (tid < nthr_norm)
      for (int e = tid; e < n * n; e += nthr_norm) {
        const int i = e / n, j = e - i * n;
        const double a = H[i * ldh + j];
        if (i == j) v[1] += a * a;
        else v[0] += a * a;
      }
    block_sum<2>(v, sh);
    if (!(v[0] > 1e-26 * v[1] + 1e-300)) break;
    ++nsweep;
    for (int r = 0; r < m; ++r) {
      int pk = 0, qk = 0;
      double ck = 1.0, sk = 0.0;
      JacItem it;
      if (has_items) {
        // lane k: the rotation of pair k mod npair (the lanes above npair
        // repeat it: branch-free, so the register reads below see every lane)
        jacobi_pair(r, kl, n2, &pk, &qk);
        jacobi_rot(H, n, ldh, pk, qk, &ck, &sk);
        it.load(H, ldh, Vt, ldv, n, npair, inv, nitem, tid, pk, qk);  // the first pass's item
      }
      __syncthreads();  // every rotation input is read before any block is written
      if (has_items) {
        for (int base = 0; base < nitem; base += nthr) {
          if (base + (tid & ~63) >= nitem) break;  // uniform per wavefront
          // later passes load after the barrier: their entries belong to
          // their own items only
          if (base > 0) it.load(H, ldh, Vt, ldv, n, npair, inv, nitem, base + tid, pk, qk);
          it.update(H, ldh, Vt, ldv, n, ck, sk);
        }
      }
      __syncthreads();
    }
  }
  return nsweep;
}

// Blocked Cholesky S = L L^T (lower, over A in place) and W = L^-1 (into Wm)
// for the global-memory solver, on one workgroup.  Panels of kCholB
// columns: the panel (already updated by the earlier panels) is factored in
// LDS column by column, written back, and the trailing matrix takes one
// rank-kCholB update from the panel rows held in LDS (4 x 4 register tiles)
// instead of kCholB rank-1 sweeps through global memory.  W is formed one
// block row at a time: thread c owns column c, sums the earlier block rows'
// contribution T[r][c] = sum_k L[i0+r][k] W[k][c] in registers, then finishes
// the block by forward substitution against the diagonal block, without
// barriers.  Returns false (A partly factored) at the first pivot <= 0.
// LDS: chol_inv_lds_doubles(n) doubles at `sm`.
constexpr int kCholB = 32;
__host__ __device__ constexpr int chol_inv_lds_doubles(int n) {
  return n * (kCholB + 1) > kCholB * (n + 1) ? n * (kCholB + 1) : kCholB * (n + 1);
}
__device__ __forceinline__ bool chol_inv_blocked(double* __restrict__ A, double* __restrict__ Wm, int n, int ld,
                                 double* __restrict__ sm, int tid, int nthr) {
  constexpr int B = kCholB, PS = kCholB + 1;
  __shared__ double piv[kCholB];
  __shared__ int bad;
  for (int p0 = 0; p0 < n; p0 += B) {
    const int pb = min(B, n - p0), m = n - p0;
    for (int e = tid; e < m * pb; e += nthr) {
      const int r = e / pb, c = e - r * pb;
      sm[r * PS + c] = A[(size_t)(p0 + r) * ld + p0 + c];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < pb; ++k) {
      const double d = sm[k * PS + k];
      if (!(d > 0.0)) {  // every thread reads the same pivot: a uniform exit
        if (tid == 0) bad = 1;
        break;
      }
      const double pk = sqrt(d), inv = 1.0 / pk;
      if (tid == 0) piv[k] = pk;
      for (int r = k + 1 + tid; r < m; r += nthr) sm[r * PS + k] *= inv;
      __syncthreads();
      const int w = pb - k - 1, rows = m - k - 1;
      for (int t = tid; t < rows * w; t += nthr) {
        const int r = k + 1 + t / w, j = k + 1 + t % w;
        if (r >= j) sm[r * PS + j] -= sm[r * PS + k] * sm[j * PS + k];
      }
      __syncthreads();
    }
    __syncthreads();
    if (bad) return false;
    for (int e = tid; e < m * pb; e += nthr) {
      const int r = e / pb, c = e - r * pb;
      if (r >= c) A[(size_t)(p0 + r) * ld + p0 + c] = r == c ? piv[c] : sm[r * PS + c];
    }
    // trailing update over rows/columns p0 + pb .. n-1 (lower triangle)
    const int mt = (m - pb + 3) / 4;
    for (int t = tid; t < mt * mt; t += nthr) {
      const int I = t / mt, J = t - I * mt;
      if (J > I) continue;
      const int r0 = pb + 4 * I, q0 = pb + 4 * J;
      double acc[4][4] = {};
      for (int c = 0; c < pb; ++c) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = r0 + u < m ? sm[(r0 + u) * PS + c] : 0.0;
          b[u] = q0 + u < m ? sm[(q0 + u) * PS + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = r0 + u, q = q0 + v;
          if (r < m && q <= r) A[(size_t)(p0 + r) * ld + p0 + q] -= acc[u][v];
        }
    }
    __syncthreads();
  }
  // W = L^-1, block row by block row
  for (int i0 = 0; i0 < n; i0 += B) {
    const int ib = min(B, n - i0), cols = i0 + ib, LS = cols | 1;
    // rows i0 .. i0+B-1 of L (columns < cols) into LDS; rows past n are zero
    for (int e = tid; e < B * cols; e += nthr) {
      const int r = e / cols, k = e - r * cols;
      sm[r * LS + k] = (r < ib && k <= i0 + r) ? A[(size_t)(i0 + r) * ld + k] : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < n; c += nthr) {
      if (c >= cols) {  // above the diagonal
        for (int r = 0; r < ib; ++r) Wm[(size_t)(i0 + r) * ld + c] = 0.0;
        continue;
      }
      double x[B];
#pragma unroll
      for (int r = 0; r < B; ++r) x[r] = 0.0;
      for (int k = c; k < i0; ++k) {
        const double w = Wm[(size_t)k * ld + c];
#pragma unroll
        for (int r = 0; r < B; ++r) x[r] = fma(sm[r * LS + k], w, x[r]);
      }
      // forward substitution against the diagonal block (rows past n stay 0)
#pragma unroll
      for (int r = 0; r < B; ++r) {
        if (r < ib) {
          double s = (i0 + r == c ? 1.0 : 0.0) - x[r];
#pragma unroll
          for (int q = 0; q < r; ++q) s = fma(-sm[r * LS + i0 + q], x[q], s);
          x[r] = s / sm[r * LS + i0 + r];
        }
      }
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (r < ib) Wm[(size_t)(i0 + r) * ld + c] = x[r];
    }
    __syncthreads();
  }
  return true;
}

// phase 0: the whole solve; 1: Cholesky and W = L^-1 only (the congruence,
// and M = W^T V then run over the whole GPU: k_sub_*; the Jacobi rounds too
// from g.jac_grid bands, k_jac_*); 3: the Jacobi rounds of the H' that
// k_sub_wh/k_sub_twt formed, in the workgroup (H' in LDS up to 128 bands);
// 2: eigenvalue order and the sorted M, eps from the converged H' and the
// product W^T V already in S.  Phases 1-3 keep W, V and the products in
// global memory.
// USE_LDS (see below) is a template parameter: the matrix pointers of each
// form then come from one address space only, so the LDS-resident ones are
// accessed with LDS instructions rather than flat ones
template <int USE_LDS>
__global__ void __launch_bounds__(kSubNT) k_subspace(const CandDesc* __restrict__ cds, int mode,
                                                     int max_sweeps, int phase) {
  constexpr int use_lds = USE_LDS;
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  const int n = cd.nb;
  const int tid = threadIdx.x, nthr = blockDim.x;
  // use_lds 1: the four matrices in LDS; 0: in global memory; 2: in global
  // memory except H', which the Jacobi rounds keep in LDS (up to 128 bands)
  const bool all_lds = use_lds == 1;
  // row stride of the four matrices: n + 1 in LDS (rows and columns of
  // FP64 entries then fall in different banks), n in global memory
  const int ld = all_lds ? n + 1 : n;
  extern __shared__ __align__(16) char smem[];
  double *P0, *P1, *P2, *P3;  // L, H / H', W = L^-1, scratch / V
  if (all_lds) {
    P0 = (double*)smem;
    P1 = P0 + n * ld;
    P2 = P1 + n * ld;
    P3 = P2 + n * ld;
    for (int e = tid; e < n * n; e += nthr) {
      const int i = e / n, j = e - i * n;
      P0[i * ld + j] = cd.S[e];
      P1[i * ld + j] = cd.Hs[e];
    }
  } else {
    P0 = cd.S;
    P1 = cd.Hs;
    P2 = cd.C;
    P3 = cd.M;
  }
  // H' from the congruence on (the input H stays in P1)
  const bool h_lds = use_lds == 2;
  double* H1 = h_lds ? (double*)smem : P1;
  const int ldh = h_lds ? n + 1 : ld;
  __shared__ int fail;
  __shared__ double sh[16 * 2];
  __shared__ int rank[640];
  __shared__ double rc[320], rs[320];
  __shared__ int rp[320], rq[320];
  long long* clk = cd.dbg_clk;
  if (phase == 2 && clk && tid == 0) {
    clk[3] = clock64();
    clk[5] = max_sweeps;  // the sweeps the grid rounds took
  }
  if (phase == 2 && cd.scal[S_ERR] == 2.0) {
    // this call's Cholesky failed: the rotation stays the identity
    for (int e = tid; e < n * n; e += nthr) cd.M[e] = (e / n == e % n) ? 1.0 : 0.0;
    return;
  }
  if (phase == 3) {
    // Jacobi of the H' that the products over the GPU formed (in Hs; V^T = I
    // in M), unless this call's Cholesky failed
    if (cd.scal[S_ERR] == 2.0) return;
    if (h_lds)
      for (int e = tid; e < n * n; e += nthr) {
        const int i = e / n, j = e - i * n;
        H1[i * ldh + j] = cd.Hs[e];
      }
    __syncthreads();
  }
  if (phase != 2) {
   if (phase != 3) {
    if (tid == 0) fail = 0;
    if (clk && tid == 0) clk[0] = clock64();
    __syncthreads();
    if (!all_lds) {
      // global-memory solver: blocked, panels in the dynamic LDS
      if (!chol_inv_blocked(P0, P2, n, ld, (double*)smem, tid, nthr)) {
        if (tid == 0) cd.scal[S_ERR] = 2.0;
        for (int e = tid; e < n * n; e += nthr) cd.M[e] = (e / n == e % n) ? 1.0 : 0.0;
        return;
      }
    } else {
      // Cholesky S = L L^T (lower, in place, right-looking; two barriers per
      // column).  The pivots are kept aside in P3 and written to the diagonal at
      // the end, so no thread overwrites a pivot another thread still reads.
      for (int k = 0; k < n; ++k) {
        __syncthreads();  // trailing update of the previous column is complete
        const double d = P0[k * ld + k];
        if (!(d > 0.0)) {
          if (tid == 0) fail = 1;
          break;
        }
        const double piv = sqrt(d);
        const double inv = 1.0 / piv;
        if (tid == 0) P3[k] = piv;
        for (int i = k + 1 + tid; i < n; i += nthr) P0[i * ld + k] *= inv;
        __syncthreads();
        const int m = n - k - 1;
        for (int t = tid; t < m * m; t += nthr) {
          const int i = k + 1 + t / m, j = k + 1 + t % m;
          if (j <= i) P0[i * ld + j] -= P0[i * ld + k] * P0[j * ld + k];
        }
      }
      __syncthreads();
      if (!fail)
        for (int k = tid; k < n; k += nthr) P0[k * ld + k] = P3[k];
      __syncthreads();
      if (fail) {
        if (tid == 0) cd.scal[S_ERR] = 2.0;
        for (int e = tid; e < n * n; e += nthr) cd.M[e] = (e / n == e % n) ? 1.0 : 0.0;
        return;
      }
      // W = L^-1 by elimination on [L | I]: at step j, rows i > j subtract
      // L[i][j] * row j (final since step j-1); row j+1 is complete after this
      // step and is divided by its pivot.  One barrier per step.
      for (int e = tid; e < n * n; e += nthr) {
        const int i = e / n, j = e % n;
        P2[i * ld + j] = i == j ? (i == 0 ? 1.0 / P0[0] : 1.0) : 0.0;
      }
      __syncthreads();
      for (int j = 0; j + 1 < n; ++j) {
        const int rows = n - 1 - j, cols = j + 1;
        for (int t = tid; t < rows * cols + 1; t += nthr) {
          if (t == rows * cols) {
            P2[(j + 1) * ld + j + 1] = 1.0 / P0[(j + 1) * ld + j + 1];
            continue;
          }
          const int i = j + 1 + t / cols, c = t % cols;
          double w = P2[i * ld + c] - P0[i * ld + j] * P2[j * ld + c];
          if (i == j + 1) w /= P0[i * ld + i];
          P2[i * ld + c] = w;
        }
        __syncthreads();
      }
    }
    if (clk && tid == 0) clk[1] = clock64();
    if (mode == 1) {
      for (int e = tid; e < n * n; e += nthr) cd.M[e] = P2[(e % n) * ld + e / n];
      return;
    }
    if (phase == 1) return;  // W is ready; the products run over the GPU
    // H' = W H W^T (symmetrised)
    if (all_lds) {
      // lane j: column j (32 or 64 columns per wavefront), rows over the
      // wavefronts; one operand of each product is an LDS broadcast
      const int lw = n <= 32 ? 32 : 64, j = tid & (lw - 1);
      const int r0 = (tid >> 6) * (64 / lw) + ((tid & 63) >= lw ? 1 : 0);
      const int rstep = (nthr >> 6) * (64 / lw);
      if (j < n)
        for (int i = r0; i < n; i += rstep) {
          double s = 0.0;
          for (int k = 0; k <= i; ++k) s = fma(P2[i * ld + k], P1[k * ld + j], s);
          P3[i * ld + j] = s;
        }
      __syncthreads();
      if (j < n)
        for (int i = r0; i < n; i += rstep) {
          double s = 0.0;
          for (int k = 0; k <= j; ++k) s = fma(P3[i * ld + k], P2[j * ld + k], s);
          H1[i * ldh + j] = s;
        }
      __syncthreads();
    } else {
      for (int e = tid; e < n * n; e += nthr) {
        const int i = e / n, j = e % n;
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s = fma(P2[i * ld + k], P1[k * ld + j], s);
        P3[i * ld + j] = s;
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += nthr) {
        const int i = e / n, j = e % n;
        double s = 0.0;
        for (int k = 0; k <= j; ++k) s = fma(P3[i * ld + k], P2[j * ld + k], s);
        H1[i * ldh + j] = s;
      }
      __syncthreads();
    }
    for (int e = tid; e < n * n; e += nthr) {
      const int i = e / n, j = e % n;
      if (i < j) {
        const double a = 0.5 * (H1[i * ldh + j] + H1[j * ldh + i]);
        H1[i * ldh + j] = a;
        H1[j * ldh + i] = a;
      }
      P3[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
   }
    // Cyclic Jacobi with the round-robin ordering of disjoint index pairs.
    // Phase A computes the rotations of a round; in phase B the threads take
    // the (row pair, column pair) 2x2 blocks, rotating them in place, then
    // V's columns.
    // Blocks whose two rotations are both the identity are skipped.  Stop when
    // the off-diagonal norm is below 1e-13 of the diagonal norm.
    const int n2 = n + (n & 1);
    const int npair = n2 / 2;
    if (clk && tid == 0) clk[2] = clock64();
    int nsweep = 0;
    const bool fast = npair <= kJacFastPairs;
    if (fast) nsweep = jacobi_sweeps_fast(H1, ldh, P3, ld, n, max_sweeps, sh, tid, nthr, nthr);
    for (int sweep = 0; sweep < (fast ? 0 : max_sweeps); ++sweep) {
      double v[2] = {0.0, 0.0};
      for (int e = tid; e < n * n; e += nthr) {
        const int i = e / n, j = e % n;
        const double a = H1[i * ldh + j];
        if (i == j) v[1] += a * a;
        else v[0] += a * a;
      }
      block_sum<2>(v, sh);
      if (!(v[0] > 1e-26 * v[1] + 1e-300)) break;
      ++nsweep;
      for (int r = 0; r < n2 - 1; ++r) {
        for (int k = tid; k < npair; k += nthr) {
          int p, q;
          jacobi_pair(r, k, n2, &p, &q);
          double c, sn;
          jacobi_rot(H1, n, ldh, p, q, &c, &sn);
          rp[k] = p;
          rq[k] = q;
          rc[k] = c;
          rs[k] = sn;
        }
        __syncthreads();
        // the (row pair P, column pair Q) blocks (two rotations each) on the
        // first half of the threads, consecutive threads taking consecutive
        // Q of one P; the column pairs of V (one rotation each, twice as
        // many) on the second half: both halves carry about the same work
        const int half = nthr / 2;
        if (tid < half) {
          for (int t = tid; t < npair * npair; t += half) {
            const int P = t / npair, Q = t - P * npair;
            const double sP = rs[P], sQ = rs[Q];
            if (sP == 0.0 && sQ == 0.0) continue;
            const double cP = rc[P], cQ = rc[Q];
            const int p1 = rp[P], p2 = rq[P], q1 = rp[Q], q2 = rq[Q];
            const bool p2v = p2 < n, q2v = q2 < n;
            const double a11 = H1[p1 * ldh + q1];
            const double a12 = q2v ? H1[p1 * ldh + q2] : 0.0;
            const double a21 = p2v ? H1[p2 * ldh + q1] : 0.0;
            const double a22 = (p2v && q2v) ? H1[p2 * ldh + q2] : 0.0;
            // rows: (a1j, a2j) -> (c a1j - s a2j, s a1j + c a2j)
            const double b11 = cP * a11 - sP * a21, b21 = sP * a11 + cP * a21;
            const double b12 = cP * a12 - sP * a22, b22 = sP * a12 + cP * a22;
            // columns: (bi1, bi2) -> (c bi1 - s bi2, s bi1 + c bi2)
            H1[p1 * ldh + q1] = cQ * b11 - sQ * b12;
            if (q2v) H1[p1 * ldh + q2] = sQ * b11 + cQ * b12;
            if (p2v) H1[p2 * ldh + q1] = cQ * b21 - sQ * b22;
            if (p2v && q2v) H1[p2 * ldh + q2] = sQ * b21 + cQ * b22;
          }
        } else {
          // V is stored transposed (P3[q][i] = V[i][q]): the column rotation of
          // pair P updates rows p1, p2 of P3 (consecutive threads, consecutive i)
          for (int t = tid - half; t < npair * n; t += half) {
            const int P = t / n, i = t - P * n;
            const double sP = rs[P];
            const int p1 = rp[P], p2 = rq[P];
            if (sP == 0.0 || p2 >= n) continue;
            const double cP = rc[P];
            const double vp = P3[p1 * ld + i], vq = P3[p2 * ld + i];
            P3[p1 * ld + i] = cP * vp - sP * vq;
            P3[p2 * ld + i] = sP * vp + cP * vq;
          }
        }
        __syncthreads();
      }
    }
    if (clk && tid == 0) {
      clk[3] = clock64();
      clk[5] = nsweep;
    }
    if (phase == 3) {
      // H' back for the sort (phase 2); M = W^T V runs over the GPU
      if (h_lds)
        for (int e = tid; e < n * n; e += nthr) {
          const int i = e / n, j = e - i * n;
          cd.Hs[e] = H1[i * ldh + j];
        }
      return;
    }
  }
  // ranks of the eigenvalues (ascending, ties by index)
  for (int i = tid; i < n; i += nthr) {
    const double li = H1[i * ldh + i];
    int rnk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = H1[j * ldh + j];
      if (lj < li || (lj == li && j < i)) ++rnk;
    }
    rank[i] = rnk;
  }
  // M = W^T V into P0 (L is no longer needed); P3 holds V^T.  In phase 2
  // the product has already been formed over the GPU (k_sub_compose).
  if (phase != 2 && all_lds) {
    // lane i: column i of M (V^T row i), rows j over the wavefronts
    const int lw = n <= 32 ? 32 : 64, i = tid & (lw - 1);
    const int r0 = (tid >> 6) * (64 / lw) + ((tid & 63) >= lw ? 1 : 0);
    const int rstep = (nthr >> 6) * (64 / lw);
    if (i < n)
      for (int j = r0; j < n; j += rstep) {
        double s = 0.0;
        for (int k = j; k < n; ++k) s = fma(P2[k * ld + j], P3[i * ld + k], s);
        P0[j * ld + i] = s;
      }
  } else if (phase != 2) {
    for (int e = tid; e < n * n; e += nthr) {
      const int j = e / n, i = e % n;
      double s = 0.0;
      for (int k = j; k < n; ++k) s = fma(P2[k * ld + j], P3[i * ld + k], s);
      P0[j * ld + i] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += nthr) {
    const int j = e / n, i = e % n;
    cd.M[j * n + rank[i]] = P0[j * ld + i];
  }
  for (int i = tid; i < n; i += nthr) cd.eps[rank[i]] = H1[i * ldh + i];
  if (clk && tid == 0) clk[4] = clock64();
}

// The Jacobi rounds of the mid path (65-128 bands) on their own: H' (formed
// over the GPU, in Hs) in LDS, V^T (= I, in M) rotated in global memory.  At
// 112 bands a sweep has 111 rounds of 3,136 items each; 1024 threads take a
// round's items in four passes where k_subspace's 512 (bounded by the
// registers of its Cholesky) need seven.  The off-diagonal norm keeps the partial sums
// of `nthr_norm` threads, so the results are those of k_subspace's phase 3
// bit for bit.
constexpr int kSubJacThreads = 1024;
__global__ void __launch_bounds__(kSubJacThreads) k_sub_jacobi(const CandDesc* __restrict__ cds,
                                                              int max_sweeps, int nthr_norm) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active || cd.scal[S_ERR] == 2.0) return;  // inactive, or this call's Cholesky failed
  const int n = cd.nb, tid = threadIdx.x, nthr = blockDim.x, ldh = n + 1;
  extern __shared__ __align__(16) char smem[];
  double* H = (double*)smem;
  __shared__ double sh[16 * 2];
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e / n, j = e - i * n;
    H[i * ldh + j] = cd.Hs[e];
  }
  __syncthreads();
  jacobi_sweeps_fast(H, ldh, cd.M, n, n, max_sweeps, sh, tid, nthr, min(nthr_norm, nthr));
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e / n, j = e - i * n;
    cd.Hs[e] = H[i * ldh + j];
  }
}

// ------------------------------------- subspace products over the GPU
// Large subspace problems: T = W H (W = L^-1 lower triangular, in C), then
// H' = T W^T symmetrised (both halves from one thread) and V = I, then after
// the Jacobi rounds M0 = W^T V (V stored transposed in M) into S.  One thread
// per output element, all candidates in one launch.
__global__ void __launch_bounds__(kNT) k_sub_wh(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.y];
  if (!cd.active) return;
  const int n = cd.nb;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e - i * n;
  const double* W = cd.C;
  double s = 0.0;
  for (int k = 0; k <= i; ++k) s = fma(W[i * n + k], cd.Hs[k * n + j], s);
  cd.S[e] = s;  // T
}
__global__ void __launch_bounds__(kNT) k_sub_twt(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.y];
  if (!cd.active) return;
  const int n = cd.nb;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e - i * n;
  cd.M[e] = i == j ? 1.0 : 0.0;  // V^T = I
  if (i > j) return;
  const double* W = cd.C;
  const double* T = cd.S;
  double a = 0.0, b = 0.0;  // H'[i][j] and H'[j][i]
  for (int k = 0; k <= j; ++k) a = fma(T[i * n + k], W[j * n + k], a);
  for (int k = 0; k <= i; ++k) b = fma(T[j * n + k], W[i * n + k], b);
  const double h = i == j ? a : 0.5 * (a + b);
  cd.Hs[i * n + j] = h;
  cd.Hs[j * n + i] = h;
}
__global__ void __launch_bounds__(kNT) k_sub_compose(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.y];
  if (!cd.active) return;
  const int n = cd.nb;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int j = e / n, i = e - j * n;
  const double* W = cd.C;
  const double* Vt = cd.M;
  double s = 0.0;
  for (int k = j; k < n; ++k) s = fma(W[k * n + j], Vt[i * n + k], s);
  cd.S[e] = s;
}

// ------------------------------------------- Jacobi rounds over the GPU
// For large band counts a round of the cyclic Jacobi iteration (the same
// round-robin pairs, rotations and 2x2 block updates as in k_subspace) is one
// launch over all candidates (k_jac_round).  The per-candidate convergence
// flag lives at the start of the reduction scratch (free while the subspace
// problem is solved).
constexpr int kJacDone = 0;  // 1.0 once the candidate's H' is diagonal

// Off-diagonal vs diagonal norm of H' (one block per candidate): sets the
// candidate's flag and done_all[c] (1 for inactive candidates).
__global__ void __launch_bounds__(kNT) k_jac_offnorm(const CandDesc* __restrict__ cds,
                                                     int* done_all) {
  const CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) {
    if (threadIdx.x == 0) done_all[blockIdx.x] = 1;
    return;
  }
  __shared__ double sh[16 * 2];
  const int n = cd.nb;
  double v[2] = {0.0, 0.0};
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const double a = cd.Hs[e];
    if (e / n == e % n) v[1] += a * a;
    else v[0] += a * a;
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    const int done = v[0] > 1e-26 * v[1] + 1e-300 ? 0 : 1;
    cd.red_part[kJacDone] = done;
    done_all[blockIdx.x] = done;
  }
}

// One Jacobi round over the GPU in a single launch: each thread computes the
// rotations it applies (block (P, Q): those of pairs P and Q; a column pair of
// V^T: that of pair P) from the round's source copy of H' and writes its
// block into the other copy (H' alternates between Hs and S, which is free
// while the rounds run), so no launch has to publish the rotations first.
// A sweep has an odd number of rounds (n2 - 1); it ends in S, and
// k_jac_copy brings H' back to Hs.  The rotations and the updates are those
// of the earlier two launches per round (the rotations, then the blocks),
// bit for bit; a launch per round fewer took the 128-atom cell from 711 to
// 638 ms per evaluation.
__global__ void __launch_bounds__(kNT) k_jac_round(const CandDesc* __restrict__ cds, int r) {
  const CandDesc& cd = cds[blockIdx.y];
  if (!cd.active || cd.red_part[kJacDone] != 0.0) return;
  const int n = cd.nb, n2 = n + (n & 1), npair = n2 / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double* A = (r & 1) ? cd.S : cd.Hs;
  double* B = (r & 1) ? cd.Hs : cd.S;
  double* Vt = cd.M;  // V stored transposed: Vt[q][i] = V[i][q]
  if (t < npair * npair) {
    const int P = t / npair, Q = t - P * npair;
    int p1, p2, q1, q2;
    jacobi_pair(r, P, n2, &p1, &p2);
    jacobi_pair(r, Q, n2, &q1, &q2);
    double cP, sP, cQ, sQ;
    jacobi_rot(A, n, n, p1, p2, &cP, &sP);
    jacobi_rot(A, n, n, q1, q2, &cQ, &sQ);
    const bool p2v = p2 < n, q2v = q2 < n;
    const double a11 = A[p1 * n + q1];
    const double a12 = q2v ? A[p1 * n + q2] : 0.0;
    const double a21 = p2v ? A[p2 * n + q1] : 0.0;
    const double a22 = (p2v && q2v) ? A[p2 * n + q2] : 0.0;
    const double b11 = cP * a11 - sP * a21, b21 = sP * a11 + cP * a21;
    const double b12 = cP * a12 - sP * a22, b22 = sP * a12 + cP * a22;
    B[p1 * n + q1] = cQ * b11 - sQ * b12;
    if (q2v) B[p1 * n + q2] = sQ * b11 + cQ * b12;
    if (p2v) B[p2 * n + q1] = cQ * b21 - sQ * b22;
    if (p2v && q2v) B[p2 * n + q2] = sQ * b21 + cQ * b22;
  } else if (t < npair * npair + npair * n) {
    const int u = t - npair * npair;
    const int P = u / n, i = u - P * n;
    int p1, p2;
    jacobi_pair(r, P, n2, &p1, &p2);
    if (p2 >= n) return;
    double cP, sP;
    jacobi_rot(A, n, n, p1, p2, &cP, &sP);
    if (sP == 0.0) return;
    const double vp = Vt[p1 * n + i], vq = Vt[p2 * n + i];
    Vt[p1 * n + i] = cP * vp - sP * vq;
    Vt[p2 * n + i] = sP * vp + cP * vq;
  }
}
__global__ void __launch_bounds__(kNT) k_jac_copy(const CandDesc* __restrict__ cds) {
  const CandDesc& cd = cds[blockIdx.y];
  if (!cd.active || cd.red_part[kJacDone] != 0.0) return;
  const int n = cd.nb;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) cd.Hs[e] = cd.S[e];
}

// Set or advance the batch's SCF iteration counter (one thread).
__global__ void k_iter_set(int* state, int value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *state = add ? *state + value : value;
}

// ---------------------------------------------------------- launch helpers
void launch_grid_fft(const LaunchCtx& L, int sign) {
  const BatchGeom& g = L.g;
  const int rpb = std::max(1, 1024 / g.N1max);
  const int rows = g.N2max * g.N3max;
  size_t lds_x = sizeof(cplx<double>) * (kMaxFftN + 2 * (size_t)rpb * g.N1max);
  prof_before("k_grid_fft_x", L.stream);
  hipLaunchKernelGGL(k_grid_fft_x, dim3((rows + rpb - 1) / rpb, 1, g.ncand), dim3(kNT), lds_x,
                     L.stream, L.desc, sign, rpb);
  check_launch("k_grid_fft_x");
  prof_after("k_grid_fft_x", L.stream);
  const int ntx = (g.N1max + kTX - 1) / kTX;
  size_t lds_y = sizeof(cplx<double>) * (kMaxFftN + 2 * (size_t)kTX * g.N2max);
  prof_before("k_grid_fft_yz", L.stream);
  hipLaunchKernelGGL(k_grid_fft_yz, dim3(ntx * g.N3max, 1, g.ncand), dim3(kNT), lds_y, L.stream,
                     L.desc, 1, sign);
  check_launch("k_grid_fft_yz");
  prof_after("k_grid_fft_yz", L.stream);
  size_t lds_z = sizeof(cplx<double>) * (kMaxFftN + 2 * (size_t)kTX * g.N3max);
  prof_before("k_grid_fft_yz", L.stream);
  hipLaunchKernelGGL(k_grid_fft_yz, dim3(ntx * g.N2max, 1, g.ncand), dim3(kNT), lds_z, L.stream,
                     L.desc, 2, sign);
  check_launch("k_grid_fft_yz");
  prof_after("k_grid_fft_yz", L.stream);
}

static int grid_blocks(const BatchGeom& g) { return std::min(1024, (g.ntot_max + kNT - 1) / kNT); }

void launch_density_finalize(const LaunchCtx& L) {
  prof_before("k_density_finalize", L.stream);
  hipLaunchKernelGGL(k_density_finalize, dim3(grid_blocks(L.g), 1, L.g.ncand), dim3(kNT), 0,
                     L.stream, L.desc);
  check_launch("k_density_finalize");
  prof_after("k_density_finalize", L.stream);
}
void launch_iter_set(const LaunchCtx& L, int* state, int value, int add) {
  hipLaunchKernelGGL(k_iter_set, dim3(1), dim3(64), 0, L.stream, state, value, add);
  check_launch("k_iter_set");
}
void launch_gspace_residual(const LaunchCtx& L) {
  prof_before("k_gspace_residual", L.stream);
  hipLaunchKernelGGL(k_gspace_residual, dim3(grid_blocks(L.g), 1, L.g.ncand), dim3(kNT), 0,
                     L.stream, L.desc);
  check_launch("k_gspace_residual");
  prof_after("k_gspace_residual", L.stream);
}
// Status scalars of every candidate into one array (one host copy per read).
__global__ void k_gather_scal(const CandDesc* __restrict__ cds, double* __restrict__ out) {
  const CandDesc& cd = cds[blockIdx.x];
  for (int k = threadIdx.x; k < S_COUNT; k += blockDim.x) out[(size_t)blockIdx.x * S_COUNT + k] = cd.scal[k];
}
void launch_gather_scal(const LaunchCtx& L, double* out) {
  hipLaunchKernelGGL(k_gather_scal, dim3(L.g.ncand), dim3(64), 0, L.stream, L.desc, out);
  check_launch("k_gather_scal");
}
// Residual gate of the all-band CG steps.  Algorithm 1 repeats its CG steps
// until the band residuals meet the convergence condition; here a candidate
// leaves the remaining CG steps of the current SCF iteration once every band
// holding charge has (f/2) |H psi - eps psi| <= tau (the residual weighted
// by the band's occupation fraction, which is how far it moves the density
// and the energy; a band with f near 0 does not hold the others back), with
// tau = max(tol, 0.1 sqrt(|dE| per atom)) from the previous SCF iteration's
// energy change (loose while the density still moves, tight near
// self-consistency).  The candidate's descriptor is masked on the device
// and S_CGSKIP set; k_cg_release undoes it before the iteration goes on.
// Not applied before the energy change is known (first two iterations of a
// solve).
__global__ void k_cg_gate(CandDesc* __restrict__ cds, double tol) {
  CandDesc& cd = cds[blockIdx.x];
  if (!cd.active) return;
  const double* sc = cd.scal;
  if (sc[S_ITER] < 2.0) return;
  const double de = sc[S_DE] / (double)max(cd.nat, 1);
  const double tau = fmax(tol, 0.1 * sqrt(de));
  double worst = 0.0;
  for (int i = threadIdx.x; i < cd.nb; i += 64)
    if (cd.occ[i] > 1e-6) worst = fmax(worst, 0.25 * cd.occ[i] * cd.occ[i] * cd.resn[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
  if (threadIdx.x == 0 && worst <= tau * tau) {
    cd.scal[S_CGSKIP] = 1.0;
    cd.active = 0;
  }
}

// phase 0: candidates that left the CG steps early are unmasked (for their
// final full subspace diagonalisation) and the ones that ran every step are
// held (masked, S_CGHOLD); phase 1: the held ones are unmasked.  Candidates
// masked by the host carry neither flag and stay masked.
__global__ void k_cg_release(CandDesc* __restrict__ cds, int n, int phase) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  CandDesc& cd = cds[c];
  double* sc = cd.scal;
  if (phase == 0) {
    if (sc[S_CGSKIP] != 0.0) {
      sc[S_CGSKIP] = 0.0;
      cd.active = 1;
    } else if (cd.active) {
      sc[S_CGHOLD] = 1.0;
      cd.active = 0;
    }
  } else if (sc[S_CGHOLD] != 0.0) {
    sc[S_CGHOLD] = 0.0;
    cd.active = 1;
  }
}

// A candidate whose SCF has converged (or failed) masks itself on the device
// for the rest of a captured multi-iteration graph; the host reads the
// status once per graph and keeps its own mask in step.
__global__ void k_mask_done(CandDesc* __restrict__ cds, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  CandDesc& cd = cds[c];
  if (cd.active && (cd.scal[S_CONV] != 0.0 || cd.scal[S_ERR] != 0.0)) cd.active = 0;
}

void launch_mask_done(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_mask_done, dim3((L.g.ncand + 63) / 64), dim3(64), 0, L.stream,
                     const_cast<CandDesc*>(L.desc), L.g.ncand);
  check_launch("k_mask_done");
}

void launch_cg_gate(const LaunchCtx& L, double tol) {
  hipLaunchKernelGGL(k_cg_gate, dim3(L.g.ncand), dim3(64), 0, L.stream, const_cast<CandDesc*>(L.desc),
                     tol);
  check_launch("k_cg_gate");
}

void launch_cg_release(const LaunchCtx& L, int phase) {
  hipLaunchKernelGGL(k_cg_release, dim3((L.g.ncand + 63) / 64), dim3(64), 0, L.stream,
                     const_cast<CandDesc*>(L.desc), L.g.ncand, phase);
  check_launch("k_cg_release");
}

void launch_scf_control(const LaunchCtx& L, double tol_e_atom, double tol_rho, double res_tol) {
  prof_before("k_scf_control", L.stream);
  hipLaunchKernelGGL(k_scf_control, dim3(L.g.ncand), dim3(64), 0, L.stream, L.desc, tol_e_atom,
                     tol_rho, res_tol);
  check_launch("k_scf_control");
  prof_after("k_scf_control", L.stream);
}
void launch_mix(const LaunchCtx& L, int initial, double alpha, double q0) {
  prof_before("k_mix", L.stream);
  hipLaunchKernelGGL(k_mix, dim3(grid_blocks(L.g), 1, L.g.ncand), dim3(kNT), 0, L.stream, L.desc,
                     initial, alpha, q0);
  check_launch("k_mix");
  prof_after("k_mix", L.stream);
}
void launch_setup_grid(const LaunchCtx& L) {
  prof_before("k_setup_grid", L.stream);
  hipLaunchKernelGGL(k_setup_grid, dim3(grid_blocks(L.g), 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_setup_grid");
  prof_after("k_setup_grid", L.stream);
}
void launch_ewald(const LaunchCtx& L) {
  const int nb = std::min(1024, (L.g.ew_ng_max + kNT - 1) / kNT);
  prof_before("k_ewald_recip", L.stream);
  hipLaunchKernelGGL(k_ewald_recip, dim3(nb, 1, L.g.ncand), dim3(kNT), 0, L.stream, L.desc,
                     L.species);
  check_launch("k_ewald_recip");
  prof_after("k_ewald_recip", L.stream);
  prof_before("k_ewald_atom", L.stream);
  hipLaunchKernelGGL(k_ewald_atom, dim3(L.g.nat_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_ewald_atom");
  prof_after("k_ewald_atom", L.stream);
}
void launch_force_local(const LaunchCtx& L) {
  prof_before("k_force_local", L.stream);
  hipLaunchKernelGGL(k_force_local, dim3(L.g.nat_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_force_local");
  prof_after("k_force_local", L.stream);
}
void launch_force_finalize(const LaunchCtx& L) {
  prof_before("k_force_finalize", L.stream);
  hipLaunchKernelGGL(k_force_finalize, dim3(L.g.ncand), dim3(kNT), 0, L.stream, L.desc);
  check_launch("k_force_finalize");
  prof_after("k_force_finalize", L.stream);
}
void launch_stress_grid(const LaunchCtx& L) {
  prof_before("k_stress_grid", L.stream);
  hipLaunchKernelGGL(k_stress_grid, dim3(kStressBlocks, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_stress_grid");
  prof_after("k_stress_grid", L.stream);
  prof_before("k_stress_ewald", L.stream);
  hipLaunchKernelGGL(k_stress_ewald, dim3(L.g.nat_max, 1, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc, L.species);
  check_launch("k_stress_ewald");
  prof_after("k_stress_ewald", L.stream);
  prof_before("k_stress_finalize", L.stream);
  hipLaunchKernelGGL(k_stress_finalize, dim3(L.g.ncand), dim3(kNT), 0, L.stream, L.desc,
                     L.species);
  check_launch("k_stress_finalize");
  prof_after("k_stress_finalize", L.stream);
}
void launch_occupations(const LaunchCtx& L) {
  prof_before("k_occupations", L.stream);
  hipLaunchKernelGGL(k_occupations, dim3(L.g.ncand), dim3(64), 0, L.stream, L.desc);
  check_launch("k_occupations");
  prof_after("k_occupations", L.stream);
}
// Where the subspace solver keeps its matrices: all four in LDS up to 64
// bands, H' alone in LDS up to 128 (the Jacobi rounds then touch global
// memory only for V's column pairs), else all in global memory; and the
// dynamic LDS that form needs (the blocked Cholesky's panels share it).
// LDS form of the subspace solver by band count: 1 up to 64 (all four
// matrices), 2 up to 128 (H' only), else 0
static int sub_lds_form(int n) { return n <= 64 ? 1 : (n <= 128 ? 2 : 0); }
static size_t sub_lds_bytes(int n, int form) {
  if (form == 1) return sizeof(double) * 4 * (size_t)n * (n + 1);
  const size_t chol = (size_t)chol_inv_lds_doubles(n);
  const size_t h = form == 2 ? (size_t)n * (n + 1) : 0;
  return sizeof(double) * std::max(chol, h);
}

static void launch_k_subspace(int form, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                              const CandDesc* desc, int mode, int max_sweeps, int phase) {
  switch (form) {
    case 1:
      hipLaunchKernelGGL(k_subspace<1>, grid, block, lds, st, desc, mode, max_sweeps, phase);
      break;
    case 2:
      hipLaunchKernelGGL(k_subspace<2>, grid, block, lds, st, desc, mode, max_sweeps, phase);
      break;
    default:
      hipLaunchKernelGGL(k_subspace<0>, grid, block, lds, st, desc, mode, max_sweeps, phase);
  }
  check_launch("k_subspace");
}

// One Jacobi sweep over the GPU (n2 - 1 rounds of two launches each),
// replayed from a graph captured once per (device, descriptor array,
// candidates, bands, stream): a sweep of 282 bands is 562 short launches, and
// the host's launch rate, not the kernels, set its pace.  The graphs live
// until the process ends (at most kSweepGraphs; past that, and on the legacy
// null stream, sweeps launch eagerly); the kernels read every size from the descriptors, so a graph
// stays valid for any batch whose descriptor array lands at the same address
// with the same candidate and band counts.
namespace {
struct SweepGraph {
  int dev;
  const void* desc;
  int ncand, n;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
};
constexpr size_t kSweepGraphs = 16;
std::mutex g_sweep_mu;
std::vector<SweepGraph> g_sweeps;
}  // namespace

static void jacobi_rounds(const LaunchCtx& L, int n, int n2, dim3 ga) {
  for (int r = 0; r < n2 - 1; ++r)
    hipLaunchKernelGGL(k_jac_round, ga, dim3(kNT), 0, L.stream, L.desc, r);
  hipLaunchKernelGGL(k_jac_copy, dim3((n * n + kNT - 1) / kNT, L.g.ncand), dim3(kNT), 0, L.stream,
                     L.desc);
}

static void jacobi_sweep(const LaunchCtx& L, int n, int n2, dim3 ga) {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "current device");
  std::lock_guard<std::mutex> lk(g_sweep_mu);
  for (const auto& e : g_sweeps)
    if (e.dev == dev && e.desc == (const void*)L.desc && e.ncand == L.g.ncand && e.n == n &&
        e.stream == L.stream) {
      hip_check(hipGraphLaunch(e.exec, L.stream), "Jacobi sweep");
      return;
    }
  // the legacy null stream cannot be captured
  if (g_sweeps.size() >= kSweepGraphs || L.stream == nullptr) {
    jacobi_rounds(L, n, n2, ga);
    check_launch("k_jac_round");
    return;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hip_check(hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal), "sweep capture");
  jacobi_rounds(L, n, n2, ga);
  hip_check(hipStreamEndCapture(L.stream, &graph), "sweep capture");
  hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "sweep graph");
  g_sweeps.push_back({dev, (const void*)L.desc, L.g.ncand, n, L.stream, graph, exec});
  hip_check(hipGraphLaunch(exec, L.stream), "Jacobi sweep");
}

void launch_subspace(const LaunchCtx& L, int mode, int max_sweeps) {
  // up to 64 bands the matrices live in LDS; the thread count is a tuning
  // parameter (a single wavefront makes barriers almost free).  From
  // g.jac_grid bands on, the Jacobi rounds run over the whole GPU (one
  // workgroup would take tens of microseconds per round in global memory);
  // that needs a host read of the convergence flags per sweep, so it is not
  // used while a graph is being captured.
  const int n = L.g.nb_max;
  const int use_lds = sub_lds_form(n);
  const size_t lds = sub_lds_bytes(n, use_lds);
  const int nthr = L.g.sub_threads;
  prof_before("k_subspace", L.stream);
  if (mode == 3 && n >= L.g.jac_grid && L.jac_done && host_sync_allowed()) {
    launch_k_subspace(0, dim3(L.g.ncand), dim3(nthr), sub_lds_bytes(n, 0), L.stream, L.desc, mode,
                      max_sweeps, 1);
    const dim3 ge((n * n + kNT - 1) / kNT, L.g.ncand);
    hipLaunchKernelGGL(k_sub_wh, ge, dim3(kNT), 0, L.stream, L.desc);
    hipLaunchKernelGGL(k_sub_twt, ge, dim3(kNT), 0, L.stream, L.desc);
    check_launch("k_sub_twt");
    const int n2 = n + (n & 1), npair = n2 / 2;
    const dim3 ga((npair * npair + npair * n + kNT - 1) / kNT, L.g.ncand);
    int done_sweeps = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      hipLaunchKernelGGL(k_jac_offnorm, dim3(L.g.ncand), dim3(kNT), 0, L.stream, L.desc,
                         L.jac_done);
      check_launch("k_jac_offnorm");
      hip_check(hipMemcpyAsync(L.jac_done_host, L.jac_done, sizeof(int) * L.g.ncand,
                               hipMemcpyDeviceToHost, L.stream),
                "Jacobi flags");
      hip_check(hipStreamSynchronize(L.stream), "Jacobi flags");
      bool all = true;
      for (int c = 0; c < L.g.ncand; ++c) all = all && L.jac_done_host[c] != 0;
      if (all) break;
      jacobi_sweep(L, n, n2, ga);
      ++done_sweeps;
    }
    hipLaunchKernelGGL(k_sub_compose, ge, dim3(kNT), 0, L.stream, L.desc);
    check_launch("k_sub_compose");
    // phase 2 takes the sweep count in place of the sweep limit (debug clocks)
    launch_k_subspace(0, dim3(L.g.ncand), dim3(nthr), 0, L.stream, L.desc, mode, done_sweeps, 2);
  } else if (mode == 3 && n > 64) {
    // Cholesky and W in the workgroup, the congruence and M = W^T V over the
    // whole GPU (one thread per element: these n^3 products were the slow
    // part of the one-workgroup solve in global memory), the Jacobi rounds
    // in the workgroup with H' in LDS up to 128 bands; no host sync, so the
    // same path serves graph capture
    const dim3 ge((n * n + kNT - 1) / kNT, L.g.ncand);
    launch_k_subspace(0, dim3(L.g.ncand), dim3(nthr), sub_lds_bytes(n, 0), L.stream, L.desc, mode,
                      max_sweeps, 1);
    hipLaunchKernelGGL(k_sub_wh, ge, dim3(kNT), 0, L.stream, L.desc);
    hipLaunchKernelGGL(k_sub_twt, ge, dim3(kNT), 0, L.stream, L.desc);
    if (n <= 128) {
      hipLaunchKernelGGL(k_sub_jacobi, dim3(L.g.ncand), dim3(kSubJacThreads),
                         sizeof(double) * (size_t)n * (n + 1), L.stream, L.desc, max_sweeps, nthr);
      check_launch("k_sub_jacobi");
    } else {
      launch_k_subspace(0, dim3(L.g.ncand), dim3(nthr), 0, L.stream, L.desc, mode, max_sweeps, 3);
    }
    hipLaunchKernelGGL(k_sub_compose, ge, dim3(kNT), 0, L.stream, L.desc);
    launch_k_subspace(0, dim3(L.g.ncand), dim3(nthr), 0, L.stream, L.desc, mode, max_sweeps, 2);
  } else {
    launch_k_subspace(use_lds, dim3(L.g.ncand), dim3(nthr), lds, L.stream, L.desc, mode, max_sweeps, 0);
  }
  prof_after("k_subspace", L.stream);
}

// ------------------------------------------------ allocation-free subspace
// Workspace of the allocation-free form of the subspace step (for callers
// that cannot allocate device memory: code under HIP graph capture, serving
// loops): one fixed device array per GPU holding the solver's descriptor,
// its status block and working copies of S and H plus the third matrix of
// the global-memory solver, for up to kNoAllocMaxN bands.  The array lives
// until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in, not a device address).  Every call on a GPU shares
// that GPU's array: calls that overlap on one GPU race.
constexpr size_t kNoAllocDescBytes = 1024;
constexpr size_t kNoAllocScalBytes = 256;
constexpr size_t kNoAllocMatBytes = (size_t)8 * kNoAllocMaxN * kNoAllocMaxN;
constexpr size_t kNoAllocBytes = kNoAllocDescBytes + kNoAllocScalBytes + 3 * kNoAllocMatBytes;
static_assert(sizeof(CandDesc) <= kNoAllocDescBytes, "descriptor slot too small");
static_assert(S_COUNT * 8 <= kNoAllocScalBytes, "status slot too small");
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kNoAllocDevices] = {};
}  // namespace

// Device address of this GPU's workspace array (the device must be current);
// taken once per device.
static char* noalloc_workspace(int device) {
  if (device < 0 || device >= kNoAllocDevices) throw_unsupported("device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the subspace workspace");
    g_noalloc_ptr[device] = (char*)p;
  }
  return g_noalloc_ptr[device];
}

// Descriptor into the workspace, status block cleared, S and H copied into
// the working matrices (the solver overwrites its inputs).
__global__ void k_noalloc_stage(CandDesc d, CandDesc* __restrict__ dst, const double* __restrict__ S,
                                const double* __restrict__ H, int nn) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *dst = d;
  if (e < S_COUNT) d.scal[e] = 0.0;
  if (e < nn) {
    d.S[e] = S[e];
    if (H) d.Hs[e] = H[e];
  }
}

__global__ void k_noalloc_status(const double* __restrict__ scal, int* __restrict__ status,
                                 int fail_code) {
  if (threadIdx.x == 0) *status = scal[S_ERR] != 0.0 ? fail_code : 0;
}

int subspace_noalloc(int device, int n, int mode, const double* S, const double* H, double* M,
                     double* eps, int* status, int fail_code, hipStream_t stream, int nthreads) {
  if (n < 1 || n > kNoAllocMaxN) throw_unsupported("band count outside 1..256 for the allocation-free subspace step");
  char* ws = noalloc_workspace(device);
  CandDesc d;
  memset(&d, 0, sizeof(d));
  d.nb = n;
  d.active = 1;
  d.scal = (double*)(ws + kNoAllocDescBytes);
  d.S = (double*)(ws + kNoAllocDescBytes + kNoAllocScalBytes);
  d.Hs = (double*)((char*)d.S + kNoAllocMatBytes);
  d.C = (double*)((char*)d.Hs + kNoAllocMatBytes);
  d.M = M;
  d.eps = eps;
  CandDesc* dd = (CandDesc*)ws;
  const int nn = n * n;
  const int nel = std::max(nn, (int)S_COUNT);
  hipLaunchKernelGGL(k_noalloc_stage, dim3((nel + kNT - 1) / kNT), dim3(kNT), 0, stream, d, dd, S,
                     mode == 3 ? H : nullptr, nn);
  check_launch("k_noalloc_stage");
  const int use_lds = sub_lds_form(n);
  const size_t lds = sub_lds_bytes(n, use_lds);
  launch_k_subspace(use_lds, dim3(1), dim3(nthreads), lds, stream, dd, mode, 40, 0);
  if (status) {
    hipLaunchKernelGGL(k_noalloc_status, dim3(1), dim3(64), 0, stream, d.scal, status, fail_code);
    check_launch("k_noalloc_status");
    return 0;
  }
  hip_check(hipStreamSynchronize(stream), "subspace step");
  double flag = 0.0;
  hip_check(hipMemcpy(&flag, d.scal + S_ERR, sizeof(double), hipMemcpyDeviceToHost), "status");
  return flag != 0.0 ? fail_code : 0;
}

void configure_wave();
void configure_kernels() {
  allow_lds((const void*)k_grid_fft_x);
  allow_lds((const void*)k_grid_fft_yz);
  allow_lds((const void*)k_subspace<0>);
  allow_lds((const void*)k_subspace<1>);
  allow_lds((const void*)k_subspace<2>);
  allow_lds((const void*)k_sub_jacobi);
  configure_wave();
  configure_plane_kernels();
  configure_kpt_kernels();
}

}  // namespace sgo
