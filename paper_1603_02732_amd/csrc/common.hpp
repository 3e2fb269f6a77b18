// Shared device/host definitions of the HIP engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgo {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }

constexpr int kMaxFftN = 128;     // longest 1-D transform along any axis
constexpr int kMaxStages = 8;
constexpr int kMaxHist = 8;       // Pulay history slots
constexpr int kNT = 256;          // threads of most kernels

// Scalars kept per candidate in device memory (double slots).
enum Scal {
  S_ETOT = 0, S_EKIN, S_ENL, S_ELOC, S_EH, S_EXC, S_EEW, S_ENTROPY_TERM,
  S_EBAND, S_VRHO, S_DRHO, S_DE, S_EPREV, S_MU, S_ENTROPY, S_CONV,
  S_ERR, S_ITER, S_NHIST, S_NSCF, S_EHARRIS, S_EWRECIP,
  S_CGSKIP, S_CGHOLD,  // residual gate of the CG steps (set and cleared within an iteration)
  S_COUNT = 32
};

// Radix plan of one transform length.
struct FftPlan {
  int n;
  int nstage;
  int radix[kMaxStages];
};

// Per-candidate device descriptor.  Pointers typed void* hold arrays of the
// wavefunction precision T (float or double); double* arrays are FP64.
struct CandDesc {
  int N1, N2, N3, ntot;
  int npwh, K, nb, npair;
  int Kp, pad_kp;   // Kp: row stride of band arrays (K rounded up to 32, zero padded)
  int nsp, nst, nproj, nat;
  int occ_kind, nocc, active, ncand_index;
  int pl_nx, pl_nxl, pl_sx, pl_pad;  // active x columns of the planes (register FFT kernels)
  int np16, pad_np;     // nproj rounded up to 16 (BF16 projector tiles)
  double sigma, nelec, omega, pad0;
  double A[9];
  double B[9];
  FftPlan plan[3];  // lengths N1, N2, N3
  // wavefunction side (precision T)
  void* X;
  void* HX;
  void* D;
  void* HD;
  void* sticks;   // cplx<T> [npair][N3][nst]
  void* veff_t;   // T [N3][N2][N1]
  void* beta;     // T [nproj][K]
  void* beta16;   // bfloat16 [2][np16][Kp] hi, lo parts (FP32_BF16PROJ form only)
  void* betaT16;  // bfloat16 [2][Kp][np16]
  const double* kin;     // [npwh]
  const int* gmeta;      // [npwh] stick | z << 20
  const int* sp_off;     // [nsp + 1]
  const int* stick_xy;   // [nst] i1 | i2 << 16
  const int* gmill;      // [npwh*3] Miller indices of the half sphere
  const double* hproj;   // [nproj]
  const int* proj_atom;  // [nproj]
  const int* proj_lm;    // [nproj] l*4 + m
  const double* proj_r;  // [nproj] projector width
  // subspace (FP64)
  double* S;       // [nb*nb]
  double* Hs;      // [nb*nb]
  double* M;       // [nb*nb]
  double* C;       // [max(nb,nproj)*nb] general product
  double* eps;     // [nb]
  double* occ;     // [nb]
  double* gam;     // [nb]  gamma of the previous CG step
  double* bandw;   // [nb]  per-band scratch
  double* resn;    // [nb]  |H psi - eps psi|^2 of each band at the last CG direction
  // grid side (FP64)
  double* rho_in_r;     // [ntot]
  double* rho_out_r;    // [ntot]
  double* veff_r;       // [ntot]
  cplx<double>* zgrid;  // [ntot] FFT work
  cplx<double>* vloc_G; // [ntot] on D, zero elsewhere
  cplx<double>* rho0_G; // [ntot]
  cplx<double>* rho_out_G;  // [ntot]
  void* hist_in;            // [kMaxHist][ntot] complex, FP64 or FP32 (hist_f32)
  void* hist_res;           // [kMaxHist][ntot]
  double* pulay;        // [kMaxHist*kMaxHist] residual dot products
  double* coef;         // [kMaxHist]
  double* dens_part;    // [nchunk][ntot]
  int ndens_chunk;
  int hist_len;         // history capacity in use
  int hist_f32;         // Pulay history stored as complex FP32 (FP32 bulk forms)
  // atoms (FP64)
  const double* pos;    // [nat*3]
  const int* spec;      // [nat]
  double* force;        // [nat*3] total
  double* force_ew;     // [nat*3]
  double* force_part;   // [nat*3*4] local / nonlocal scratch
  double* nlwork;       // [nproj*nb*4]
  double* stwork;       // stress partial sums, layout in stress_layout()
  double* stress;       // [9] total, then [6][9] parts (kin, nl, H, loc, xc, Ewald)
  double* scal;         // [S_COUNT]
  cplx<double>* ewS;    // [ew_ng] Ewald structure factors
  double ew_eta, ew_rcut, ew_gcut, pad2;
  int ew_m[3], ew_n[3];  // reciprocal / image enumeration half-widths
  int ew_ng, ew_nimg;
  long long* dbg_clk;   // optional phase timestamps of the subspace solver
  int* iter_state;      // SCF iteration counter of the batch (device memory)
  // reduction scratch: partial sums and tickets (zeroed at allocation)
  double* red_part;     // [kRedSlots]
  unsigned* tickets;    // [kTickets]
  unsigned seed;
  int pad1;
};

constexpr int kRedSlots = 1 << 16;

// Stress partial sums (doubles): per band kinetic [nb][6]; per projector and
// band (P, Q_xx..Q_xy) [nproj][nb][7]; grid blocks [kStressBlocks][16];
// per atom Ewald [nat][13].  Voigt order xx yy zz yz xz xy.
constexpr int kStressBlocks = 256;
struct StressLayout {
  size_t kin, nl, grid, ew, total;
};
__host__ __device__ inline StressLayout stress_layout(int nb, int nproj, int nat) {
  StressLayout L;
  L.kin = 0;
  L.nl = (size_t)6 * nb;
  L.grid = L.nl + (size_t)7 * nproj * nb;
  L.ew = L.grid + (size_t)16 * kStressBlocks;
  L.total = L.ew + (size_t)13 * nat;
  return L;
}
constexpr int kTickets = 512;
constexpr int kTicketGrid = 480;  // first ticket not used by the Gram products

// Species parameters on device (constant per batch).
struct SpeciesDev {
  double Z;
  int local_kind;
  int nkb;
  double p[3];
  int kb_l[4];
  double kb_r[4];
  double kb_h[4];
  double rho0_width;
};
constexpr int kMaxSpecies = 16;

}  // namespace sgo
