// Host-side launch wrappers of the HIP kernels (defined in kernels_*.hip).
#pragma once
#include "common.hpp"

namespace sgo {

// Which wavefunction-side array a kernel reads or writes.
enum WArr { W_X = 0, W_HX = 1, W_D = 2, W_HD = 3, W_BETA = 4 };
// Which FP64 matrix a product writes or reads.
enum MArr { M_S = 0, M_H = 1, M_M = 2, M_C = 3 };

// Launch geometry shared by all candidates of a batch (maxima over them).
// Default band count from which the subspace products and Jacobi rounds run
// over the whole GPU instead of one workgroup per candidate (BatchGeom
// jac_grid, tuning key SGO_JAC_GRID).
constexpr int kJacGridBandsDefault = 160;

struct BatchGeom {
  int ncand;
  int npair_max, nsp_max, nb_max, nproj_max, nat_max;
  int N1max, N2max, N3max, ntot_max, plane_max;
  int plane_reg;   // 1: FP32 register-FFT plane kernels for every candidate
  int pl_sx_max;   // largest compact plane row stride
  int gemm_f32;    // 1: FP32-MFMA band products in the FP32 path
  int gemm_waves = 8;  // wavefronts sharing a staged slice from 64 input rows (4, 6 or 8)
  int gram_tile = 0;   // Gram output tile: 64 rows when set to 64, else 32
  int gram_f32;    // 1: FP32-MFMA Gram products (FP64 sums of the K ranges)
  int bf16proj;    // 1: projector products with BF16 inputs (FP32_BF16PROJ form)
  size_t red_min_bytes;  // smallest reduction scratch of any candidate
  size_t lds_limit;      // dynamic LDS a kernel may use (device limit minus static use)
  int K_max;
  int sp_chunk;      // stick pairs per block of the z kernels
  int kc_len;        // K range per block of the split-K products
  int nkc_max;       // number of K ranges
  int dens_chunks;   // band-pair chunks of the density planes
  int ew_ng_max;     // reciprocal Ewald vectors enumerated (box size)
  int ew_nimg_max;
  int sub_threads;   // threads of the LDS-resident subspace solver
  int jac_grid = kJacGridBandsDefault;  // band count from which the subspace solve runs over the GPU
  int plane_group = 1;  // z-planes per workgroup of the H psi plane kernel (1: one per wavefront)
};

struct LaunchCtx {
  hipStream_t stream;
  const CandDesc* desc;      // device array [ncand]
  const SpeciesDev* species; // device array [kMaxSpecies]
  BatchGeom g;
  int* jac_done = nullptr;       // device [ncand]: per-candidate Jacobi convergence flags
  int* jac_done_host = nullptr;  // pinned host copy of them
};

// False while the calling thread captures a graph (no host synchronisation).
bool host_sync_allowed();

template <typename T> void launch_hpsi(const LaunchCtx& L, int src /*W_X or W_D*/);
template <typename T> void launch_density(const LaunchCtx& L);
template <typename T> void launch_gram(const LaunchCtx& L, int nprod, const int* a, const int* b,
                                       const int* out);
template <typename T> void launch_gemm_acc(const LaunchCtx& L, int narr, const int* y, const int* a,
                                           int mat, double alpha, double beta, int use_h);
template <typename T> void launch_cg_direction(const LaunchCtx& L, int first);
template <typename T> void launch_linemin(const LaunchCtx& L);
template <typename T> void launch_band_kinetic(const LaunchCtx& L);
template <typename T> void launch_init_random(const LaunchCtx& L);
template <typename T> void launch_setup_beta(const LaunchCtx& L);
template <typename T> void launch_force_nonlocal(const LaunchCtx& L);
template <typename T> void launch_stress_waves(const LaunchCtx& L);
template <typename T> void launch_potential_finalize(const LaunchCtx& L);
void launch_subspace(const LaunchCtx& L, int mode, int max_sweeps = 40);
// The subspace step with its workspace in a fixed per-device array (no
// allocation): S, H (mode 3) device inputs [n*n], M [n*n] and eps [n] device
// outputs; n <= kNoAllocMaxN.  With status != NULL it only enqueues on
// `stream` and a kernel writes 0 or fail_code to *status; otherwise it waits
// for the stream and returns 0 or fail_code.
constexpr int kNoAllocMaxN = 256;
int subspace_noalloc(int device, int n, int mode, const double* S, const double* H, double* M,
                     double* eps, int* status, int fail_code, hipStream_t stream, int nthreads);
void launch_occupations(const LaunchCtx& L);
void launch_grid_fft(const LaunchCtx& L, int sign);
void launch_density_finalize(const LaunchCtx& L);
void launch_gspace_residual(const LaunchCtx& L);
// res_tol > 0: convergence also needs the charged bands' residuals at the
// gate (max(res_tol, 0.1 sqrt(tol_e_atom))).
void launch_scf_control(const LaunchCtx& L, double tol_e_atom, double tol_rho, double res_tol);
// Residual gate of the CG steps (masks candidates whose bands meet the
// residual condition, device side) and its release (phase 0, then 1).
void launch_cg_gate(const LaunchCtx& L, double tol);
// Converged or failed candidates masked on the device (multi-iteration graphs).
void launch_mask_done(const LaunchCtx& L);
void launch_cg_release(const LaunchCtx& L, int phase);
void launch_iter_set(const LaunchCtx& L, int* state, int value, int add);
void launch_mix(const LaunchCtx& L, int initial, double alpha, double q0);
void launch_setup_grid(const LaunchCtx& L);
void launch_ewald(const LaunchCtx& L);
void launch_force_local(const LaunchCtx& L);
void launch_force_finalize(const LaunchCtx& L);
void launch_stress_grid(const LaunchCtx& L);
void launch_gather_scal(const LaunchCtx& L, double* out);  // [ncand][S_COUNT]  // grid, Ewald and finalize kernels

// Enable large dynamic LDS for every kernel (once per process per device).
void configure_kernels();
// Register-FFT plane kernels (FP32, line lengths 2^a 3^b 5^c up to 64).
bool plane_reg_length_ok(int n);
size_t plane_reg_lds(const BatchGeom& g, bool density);
void launch_plane_hpsi_reg(const LaunchCtx& L);
// Planes per workgroup of the grouped H psi plane kernel for this geometry
// (1: the one-plane kernel; `forced` > 0 asks for that size where it fits).
int plane_group_size(const BatchGeom& g, size_t lds_per_cu, int forced);
size_t plane_group_lds(const BatchGeom& g, int group);
void launch_plane_density_reg(const LaunchCtx& L);
void launch_z_inverse_reg(const LaunchCtx& L, int src);
void launch_z_forward_reg(const LaunchCtx& L, int src, int dst);
void configure_plane_kernels();
// ---- k-point sampling (kernels_kpt.hip): complex bands on the shifted
// sphere |k+G|^2/2 <= Ecut of one k-point, FP64
struct KptBands {
  int npw, nb, nproj;
  const int* box;        // [npw] index of each coefficient in the [N3][N2][N1] grid
  const double* kin;     // [npw] |k+G|^2 / 2
  const double* q;       // [npw][3] k + G (Cartesian, bohr^-1)
  cplx<double>* beta;    // [nproj][npw] projectors at k + G
};
void kpt_zero(hipStream_t s, cplx<double>* a, long n);
void kpt_scatter_bands(hipStream_t s, cplx<double>* zk, const cplx<double>* X, const KptBands& kb, long ntot);
void kpt_fft3(hipStream_t s, cplx<double>* zk, int nb, const int N[3], const FftPlan* plans, int sign);
void kpt_hpsi(hipStream_t s, const KptBands& kb, const cplx<double>* X, cplx<double>* Y, cplx<double>* zk,
              const double* veff, const int N[3], const FftPlan* plans, cplx<double>* P, const double* h);
void kpt_zdot(hipStream_t s, const cplx<double>* A, int na, const cplx<double>* B, int nbb, int npw,
              cplx<double>* C, int ldc, const double* q, int qa);
void kpt_zgemm(hipStream_t s, const cplx<double>* X, int nx, const cplx<double>* M, int ldm, cplx<double>* Y,
               int ny, int npw, double alpha, double beta, const double* h);
void kpt_copy(hipStream_t s, cplx<double>* dst, const cplx<double>* src, long n);
void kpt_beta(hipStream_t s, const KptBands& kb, const int* patom, const int* plm, const double* pr,
              const double* pos, double omega);
void kpt_subspace(hipStream_t s, cplx<double>* S, cplx<double>* H, cplx<double>* W, cplx<double>* V,
                  cplx<double>* M, double* eps, int n, int mode, int* fail);
void kpt_cg_dir(hipStream_t s, const KptBands& kb, const cplx<double>* X, const cplx<double>* HX,
                cplx<double>* D, const double* eps, double* gam, int first);
void kpt_linemin(hipStream_t s, const KptBands& kb, cplx<double>* X, cplx<double>* HX,
                 const cplx<double>* D, const cplx<double>* HD);
void kpt_init(hipStream_t s, const KptBands& kb, cplx<double>* X, unsigned seed, int kidx);
void kpt_occupations(hipStream_t s, const double* eps, const double* wk, int nk, int nb, double nelec,
                     int kind, double sigma, double* occ, double* scal);
void kpt_band_kinetic(hipStream_t s, const KptBands& kb, const cplx<double>* X, double* out);
void kpt_kinetic_total(hipStream_t s, const double* bandw_k, const double* occ_k, const double* wk, int nk,
                       int nb, double* occ_s, double* bandw_s, int nb_s);
void kpt_density(hipStream_t s, const cplx<double>* zk, const double* occ, double wk, int nb, long ntot,
                 double* dens, int first);
void kpt_force_nl(hipStream_t s, const cplx<double>* P, const cplx<double>* dP, int nproj, int nb,
                  const double* h, const int* patom, const double* occ, double wk, int nat, double* fnl,
                  int first);
void kpt_force_total(hipStream_t s, const double* floc, const double* fnl, const double* few, int nat,
                     double* force, double* fnl_part);
void configure_kpt_kernels();
// BF16-input projector products (FP32_BF16PROJ form).
void launch_beta_bf16(const LaunchCtx& L);
void launch_proj_bf16(const LaunchCtx& L, int src, int dst);
// Raise the dynamic-LDS limit of one kernel to what the device allows.
void allow_lds(const void* kernel);
// Report a failed launch by kernel name (throws on the host side).
void check_launch(const char* name);
// Throws the library error for a failed HIP runtime call.
void hip_check(hipError_t e, const char* what);
// Reject a launch shape the kernels do not support (throws on the host side).
void throw_unsupported(const char* what);
// Optional event timing of every launch of one named kernel.
void prof_before(const char* name, hipStream_t s);
// `rows`: coefficient rows (band or projector rows of length K) that one
// candidate's share of the launch reads or writes, where a launcher states it
void prof_after(const char* name, hipStream_t s, long long rows = 0);

}  // namespace sgo
