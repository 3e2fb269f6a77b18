/*
 * sgo.h -- C-ABI of the MI355X plane-wave Kohn-Sham energy/force engine.
 *
 * The library evaluates, for one atomic structure or for a whole population
 * of candidate structures, the self-consistent Gamma-point plane-wave
 * Kohn-Sham total energy and the Hellmann-Feynman forces: the energy-and-force
 * call that every local relaxation of every differential-evolution candidate
 * makes in the structure-search engine (Section 2.1, Fig. 1; Section 2.4).
 * The electronic minimisation follows the all-band preconditioned conjugate
 * gradient scheme of Algorithm 1 (residual, preconditioning, projection,
 * line minimisation, orthogonalisation, subspace diagonalisation) inside the
 * density-mixing SCF loop described in Section 2.4.
 *
 * Units: Hartree atomic units throughout.  Lattice = three row vectors a_1,
 * a_2, a_3 in bohr (row-major 3x3, lattice[3*i + k] = k-th Cartesian
 * component of a_i).  Positions are Cartesian bohr, energies Ha, forces
 * Ha/bohr, stress Ha/bohr^3 with stress_ab = (1/Omega) dE/d(eps_ab).
 *
 * Conventions:
 *  - Every function returns SGO_OK (0) or a negative status; nothing throws
 *    across the boundary.  sgo_last_error() returns a message owned by the
 *    handle (thread-local storage when the handle is NULL).
 *  - Input arrays are host memory, copied during the call; the caller keeps
 *    ownership.  Output arrays are caller-owned host memory, written during
 *    the call.  All device memory is allocated and owned by the handle.
 *  - Handles are not thread-safe; use one handle per host thread.  All device
 *    work of a handle runs on its stream (default: the device's null stream,
 *    or the one set with sgo_set_stream).
 *  - Call order for a single structure: set_species (each species used) ->
 *    set_cell -> set_atoms -> set_cutoff -> scf -> {energy, forces,
 *    eigenvalues, stress}.  A violation returns SGO_ESTATE.  Calling
 *    set_atoms after scf keeps the wavefunctions and density as a warm start;
 *    set_cell, set_cutoff or set_species discard them.
 */
#ifndef SGO_H
#define SGO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SGO_OK = 0,
  SGO_EINVAL = -1,   /* bad argument: NULL pointer, size out of range, ... */
  SGO_ENOMEM = -2,   /* device or host allocation failed */
  SGO_EDEVICE = -3,  /* HIP runtime error (no device, launch failure, ...) */
  SGO_ENOTCONV = -4, /* SCF hit max_iter; results are readable but flagged */
  SGO_ENUMERIC = -5, /* NaN/Inf or a non-positive overlap pivot */
  SGO_ESTATE = -6    /* call made out of order */
};

/* Arithmetic of the bulk wavefunction work (FFTs, H*psi, projector and
 * subspace products).  The subspace Cholesky and diagonalisation, the Ewald
 * sum, the density/potential grid work and every energy sum are FP64 in all
 * modes.  SGO_FP32_BF16PROJ is SGO_FP32 with the Kleinman-Bylander projector
 * products of H*psi (P = beta^T psi, H psi += beta (h P)) on BF16 MFMA with
 * FP32 accumulation; every operand is split into two BF16 parts (hi + lo)
 * and a product is hi*hi + hi*lo + lo*hi (a single BF16 rounding moves the
 * cluster-population energy by ~5e-5 Ha/atom; the split keeps it within
 * the FP32 form's tolerance).  Forces and stress keep FP32 projections with
 * FP64 sums. */
enum { SGO_FP64 = 0, SGO_FP32 = 1, SGO_FP32_BF16PROJ = 2 };

enum { SGO_LOCAL_AH = 0, SGO_LOCAL_GAUSS = 1 };
enum { SGO_OCC_FIXED = 0, SGO_OCC_FERMI = 1 };

/* Analytic pseudopotential of one species.
 *  local_kind == SGO_LOCAL_AH:
 *     v(r) = -(Z/r) erf(sqrt(p0) r) + (p1 + p2 r^2) exp(-p0 r^2)
 *  local_kind == SGO_LOCAL_GAUSS (p0 = rloc):
 *     v(r) = -(Z/r) erf(r/(sqrt2 p0)) + exp(-r^2/(2 p0^2)) [p1 + p2 (r/p0)^2]
 *  nkb Kleinman-Bylander channels (l = 0 or 1), radial projector
 *     p_l(r) ~ r^l exp(-r^2/(2 kb_r^2)), normalised, channel energy kb_h.
 *  rho0_width: width (bohr) of the normalised Gaussian of charge Z placed on
 *  each atom to build the starting density. */
typedef struct {
  double Z;
  int local_kind;
  double p[3];
  int nkb;
  int kb_l[4];
  double kb_r[4];
  double kb_h[4];
  double rho0_width;
} sgo_species;

typedef struct {
  int max_iter;      /* SCF iterations (default 100) */
  int ncg;           /* all-band CG steps per SCF iteration (default 3) */
  int ncg_first;     /* CG steps in the first iteration (default 8) */
  double tol_e;      /* |E_k - E_{k-1}| stop, Ha per atom (default 1e-5) */
  double tol_rho;    /* Omega/Ntot sum|rho_out - rho_in| / N_el stop (default 1e-4) */
  double mix_alpha;  /* Pulay/Kerker mixing weight (default 0.5) */
  double kerker_q0;  /* Kerker wavevector, bohr^-1 (default 0.8, robust for
                        dense cells; isolated clusters in a vacuum box converge
                        in fewer iterations with weak damping, e.g. 0.3 with
                        mix_alpha 0.3) */
  int history;       /* Pulay history length, 2..8 (default 8) */
  unsigned seed;     /* seed of the starting wavefunctions (default 1) */
  int use_graph;     /* K >= 1: capture K SCF iterations in one HIP graph and
                        replay it, structures that converge inside it masking
                        themselves on the device, the status read back once
                        per K iterations; 0 (default): eager launches, the
                        status read after every iteration */
  double cg_tol;     /* residual gate of the CG steps (Algorithm 1 repeats them
                        until the residuals meet the convergence condition):
                        0 (default) runs ncg (ncg_first) steps every SCF
                        iteration; > 0 lets a structure stop its steps in an
                        iteration once every band holding charge has
                        (f/2) |H psi - eps psi| <= max(cg_tol, 0.1 sqrt(|dE|
                        per atom of the previous iteration)) (Ha; f in [0, 2]
                        the band's occupation), ncg staying the limit; from
                        the third iteration of a solve on.  With cg_tol > 0
                        a structure also counts as converged only when those
                        weighted residuals are <= max(cg_tol, 0.1 sqrt(tol_e)) */
} sgo_scf_opts;

typedef struct {
  int iterations;
  int converged;
  double de;         /* last |E_k - E_{k-1}| (Ha, whole cell) */
  double drho;       /* last density residual (see tol_rho) */
} sgo_scf_info;

typedef struct {
  double total;      /* free energy E - sigma S (Ha) */
  double kinetic, nonlocal, local, hartree, xc, ewald, entropy; /* entropy = -sigma S */
  double band;       /* sum_i f_i eps_i */
  double fermi;      /* chemical potential (Ha) */
} sgo_energy_terms;

typedef struct sgo_ctx sgo_ctx;
typedef struct sgo_batch sgo_batch;

/* Fill opts with the defaults listed above. */
void sgo_default_opts(sgo_scf_opts* opts);

/* Version string of the library (static storage). */
const char* sgo_version(void);

/* Create a handle on HIP device `device` with precision SGO_FP64, SGO_FP32
 * or SGO_FP32_BF16PROJ.
 * *out receives the handle (caller destroys it with sgo_destroy). */
int sgo_create(sgo_ctx** out, int device, int precision);
int sgo_destroy(sgo_ctx* ctx);

/* Run all device work of the handle on `hip_stream` (a hipStream_t, e.g. the
 * current PyTorch stream); NULL selects the null stream. */
int sgo_set_stream(sgo_ctx* ctx, void* hip_stream);

/* Device memory of the structures (one arena per structure: bands, sticks,
 * grids, history; the bulk of the footprint) from the caller's allocator,
 * e.g. a framework's caching allocator: alloc(bytes, user) returns device
 * memory of `bytes` on the handle's device (256-byte aligned) or NULL;
 * dealloc(ptr, user) releases it (called after the device has finished with
 * it).  Both NULL restores hipMalloc/hipFree.  Arenas of the previous
 * allocator are released at once (the next solve starts cold).  Small
 * descriptor and status buffers stay with the library. */
int sgo_set_allocator(sgo_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                      void (*dealloc)(void* ptr, void* user), void* user);

/* Register species `id` (0 <= id < 16).  Copies *sp. */
int sgo_set_species(sgo_ctx* ctx, int id, const sgo_species* sp);

/* Set the cell (9 doubles, rows a_i); rejects non-positive volume. */
int sgo_set_cell(sgo_ctx* ctx, const double lattice[9]);

/* Set natoms atoms: species ids [natoms] and Cartesian positions
 * [natoms*3].  Rejects unknown species and atoms closer than 1e-3 bohr
 * (minimum image).  Warm start is kept if the count and species agree. */
int sgo_set_atoms(sgo_ctx* ctx, int natoms, const int* species, const double* pos);

/* Plane-wave cutoff (Ha), FFT grid fft[3] (each N_i must hold the sphere:
 * N_i >= 2 max|m_i| + 1, and factor into 2, 3, 5; at most 128) and the
 * number of bands (must hold the electrons for fixed occupations).
 * fft = {0, 0, 0} (or any zero entry) selects the smallest 2^a 3^b 5^c length
 * with spacing |a_i|/N_i <= 0.375 bohr that holds the sphere; nbands = 0
 * selects the even ceil(1.2 N_occ) (N_occ = ceil(N_el / 2)).  sgo_grid_info
 * reports what was chosen.
 * Occupations: SGO_OCC_FIXED (2 per band, lowest first) or SGO_OCC_FERMI
 * with smearing width sigma (Ha). */
int sgo_set_cutoff(sgo_ctx* ctx, double ecut, const int fft[3], int nbands,
                   int occ_kind, double sigma);

/* Self-consistent field solve (Section 2.4, Algorithm 1).  opts may be NULL
 * (defaults); info may be NULL.  Returns SGO_ENOTCONV if max_iter is reached
 * (results still readable). */
int sgo_scf(sgo_ctx* ctx, const sgo_scf_opts* opts, sgo_scf_info* info);

/* Total free energy and (nullable) its parts after sgo_scf: the energy of
 * the structure that the evaluation level returns to the relaxation and
 * search levels (Section 2.1, Fig. 1), at the self-consistent density of
 * Section 2.4. */
int sgo_energy(sgo_ctx* ctx, double* etot, sgo_energy_terms* terms);

/* Hellmann-Feynman forces [natoms*3] after sgo_scf (local, nonlocal and
 * Ewald parts; -dF/dR of the free energy at self-consistency): the atomic
 * forces of the structure that the local relaxations consume (Section 2.1,
 * Fig. 1; Section 2.3). */
int sgo_forces(sgo_ctx* ctx, double* forces);

/* Fixed-basis stress after sgo_scf.  The paper evaluates energies and
 * forces only; the stress is this library's addition, the strain derivative
 * of the same discrete functional, so that the energy of a cell can be
 * differentiated in its lattice vectors (the 128-atom silicon supercell is
 * measured with energy, forces and stress).
 * sigma_ab = (1/Omega) dF/d eps_ab for the homogeneous strain
 * r -> (1 + eps) r of cell and atoms together, at the current Miller set and
 * fixed coefficients and occupations (the Mermin free energy is stationary
 * in both at self-consistency).  Ha/bohr^3, row-major symmetric [3][3]; a
 * cell under compression has negative diagonal entries (sigma = -pressure
 * for an isotropic cell).  parts (nullable) receives [6][3][3]: kinetic,
 * nonlocal, Hartree, local, exchange-correlation and Ewald contributions,
 * summing to stress.  Runs the stress kernels on the converged state; the
 * structure must have been solved (SGO_ESTATE otherwise). */
int sgo_stress(sgo_ctx* ctx, double stress[9], double* parts);

/* Eigenvalues [nbands] (ascending) and, if occ != NULL, occupations: the
 * eps_i of the last subspace diagonalisation of Algorithm 1 at
 * self-consistency, and the occupations of Section 2.4's output density. */
int sgo_eigenvalues(sgo_ctx* ctx, double* eig, double* occ);

/* Adjoint of the energy (the gradient the relaxations of Section 2.3 follow,
 * for a caller that differentiates a function of the energy):
 * grad_pos = gE * dE/dR = -gE * F  [natoms*3] and,
 * if grad_lattice != NULL, gE * dE/dA [3][3] (A rows = lattice vectors) with
 * the Cartesian positions as given held fixed and the Miller set of the
 * current basis held fixed: dE/dA = A^-T (Omega sigma + sum_I R_I F_I^T),
 * from the stress sigma (sgo_stress) and forces. */
int sgo_adjoint(sgo_ctx* ctx, double gE, double* grad_pos, double* grad_lattice);

/* Brillouin-zone sampling with k-points (Section 2.3 allows "rough
 * K-points" for the energy evaluations of a search); SGO_FP64 handles only.
 * kfrac [nk][3]: k in units of the reciprocal lattice vectors
 * (k = sum_i kfrac_i b_i, b = 2 pi A^-T); weights [nk], positive, normalised
 * by the library.  Each k has its own shifted sphere |k+G|^2/2 <= Ecut of
 * complex coefficients (one complex FFT per band, complex Hermitian
 * subspace matrices); the density sums the k-points with their weights, and
 * the occupations share one chemical potential (Fermi-Dirac) or fill the
 * lowest N_el/2 states of every k (fixed).  nk = 0 returns to the
 * Gamma-point path.  Call after sgo_set_cutoff; sgo_scf, sgo_energy and
 * sgo_forces then use the k-points (sgo_stress, sgo_eigenvalues and the
 * lattice gradient of sgo_adjoint return SGO_EINVAL).  SGO_EINVAL for a
 * non-FP64 handle, non-positive weights or non-finite k; SGO_EINVAL at
 * sgo_scf when the FFT grid does not hold a k-point's sphere. */
int sgo_set_kpoints(sgo_ctx* ctx, int nk, const double* kfrac, const double* weights);
/* Eigenvalues eig [nk][nbands] (ascending per k) and, if occ != NULL, the
 * occupations of the last k-point solve (the eps_nk of the subspace
 * diagonalisation of Algorithm 1 at each k); SGO_ESTATE before one. */
int sgo_kpoint_eigenvalues(sgo_ctx* ctx, double* eig, double* occ);

/* Drop the warm-start wavefunctions and density. */
int sgo_reset(sgo_ctx* ctx);

/* Sizes of the plane-wave basis: number of half-sphere G vectors (the
 * Gamma-point packing stores one of each +-G pair) and of projectors. */
int sgo_basis_size(sgo_ctx* ctx, int* npw_half, int* nproj);

/* Miller indices [npw_half*3] of the half-sphere in storage order.  A band is
 * stored as 2*npw_half reals: for G != 0, sqrt2 Re c_G, sqrt2 Im c_G; for
 * G = 0, c_0 and 0.  The dot product of two stored bands is <psi_a|psi_b>. */
int sgo_basis_millers(sgo_ctx* ctx, int* millers);

/* Apply H[V] to nb packed bands (host arrays): veff [N3][N2][N1] (x fastest,
 * r = sum n_i/N_i a_i), psi [nb][2*npw_half] -> hpsi (same layout).  Uses the
 * atoms and cutoff already set; needs no SCF.  For checking the operator. */
int sgo_apply_h(sgo_ctx* ctx, const double* veff, int nb, const double* psi, double* hpsi);

/* Current SCF output density rho(r) [N3][N2][N1] and effective potential
 * V_eff(r) (either may be NULL) after sgo_scf. */
int sgo_get_density(sgo_ctx* ctx, double* rho, double* veff);

const char* sgo_last_error(const sgo_ctx* ctx);

/* Sizes of the current structure: info[0..9] = N1, N2, N3, N1*N2*N3, npw_half,
 * nbands, band pairs (two real bands share one complex FFT), z-sticks of the
 * sphere, stick pairs (+-(m1,m2)), projectors. */
int sgo_grid_info(sgo_ctx* ctx, int info[10]);

/* The FP64 subspace step on host matrices (n <= 640): Cholesky S = L L^T
 * (Gram-Schmidt in band order: the orthogonalisation step of Algorithm 1) and, for
 * mode 3, diagonalisation of H' = L^-1 H L^-T (subspace diagonalisation).
 * Writes M [n*n] (row-major; new band i = sum_j old band j * M[j*n+i]):
 * mode 1: M = L^-T; mode 3: M = L^-T V with eigenvalues eps [n] ascending.
 * Runs the same kernel the SCF uses `reps` times and returns the mean time
 * per call; clocks (nullable, 6 entries) receives device timestamps of the
 * solver phases and the Jacobi sweep count.  SGO_ENUMERIC if S is not
 * positive definite. */
int sgo_subspace_solve(int device, int n, int mode, const double* S, const double* H,
                       double* M, double* eps, int reps, double* ms_per_call,
                       long long* clocks);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): the subspace step of
 * sgo_subspace_solve on device arrays, with its workspace (descriptor,
 * status block, working copies of S and H and one more n x n matrix) in a
 * fixed array of the library on each GPU (about 1.5 MiB, held until the
 * process ends).  S, H [n*n] (H ignored for mode 1) are device inputs, left
 * unchanged; M [n*n] and eps [n] (mode 3) are device outputs in the layout
 * of sgo_subspace_solve; all are owned by the caller.  Work is enqueued on
 * hip_stream (NULL: the null stream) of `device`.  status (device int,
 * nullable): when given, the call only enqueues, and *status receives 0 or
 * SGO_ENUMERIC (S not positive definite) in stream order; when NULL, the
 * call waits for the stream and returns SGO_ENUMERIC itself.  n must be
 * 1..256 (SGO_EINVAL otherwise: the workspace holds no more); the solve runs
 * in one workgroup at every size.  Calls no allocator.  All calls on one GPU
 * share its workspace, which keeps the last call's contents: calls that
 * overlap on one GPU (other streams, other host threads) race. */
int sgo_subspace_solve_noalloc(int device, int n, int mode, const double* S, const double* H,
                               double* M, double* eps, int* status, void* hip_stream);

/* Launch-schedule tuning (process-wide; read when a solve starts).  Keys:
 * "SGO_GRAM_KC" (K range of one split-K Gram block, multiple of 32),
 * "SGO_SUB_THREADS" (threads of the subspace solver's workgroup, 64..512; the
 * Jacobi rounds of 65 to 128 bands always run on 1024 threads),
 * "SGO_SP_CHUNK" (stick pairs per block of the LDS z transforms, used by
 * FP64 and by lines longer than 64; the FP32 register z passes take 16),
 * "SGO_DENS_CHUNKS" (band-pair chunks of the density planes),
 * "SGO_RR_SWEEPS" (Jacobi sweeps of the intermediate subspace steps),
 * "SGO_PLANE_KERNEL" (FP32 plane transforms: 1 = register-resident line
 * FFTs, the default where every line length is 2^a 3^b 5^c <= 64;
 * 2 = LDS Stockham passes, used for FP64 and longer lines),
 * "SGO_GEMM_KERNEL" (FP32 band products X M: 1 = FP32 MFMA with FP32
 * accumulation, the default; 2 = FP64 MFMA on the FP32 data),
 * "SGO_GEMM_WAVES" (wavefronts that share one staged 64-column slice of the
 * FP32 MFMA band products from 64 input rows: 4 (32-row output tiles), 6 or
 * 8 (16-row tiles, the default)),
 * "SGO_GRAM_TILE" (output tile of the Gram products: 32 rows, the default,
 * or 64),
 * "SGO_GRAM_KERNEL" (FP32 Gram products S, H, C: 1 = FP64 MFMA, each product
 * exact, the default; 2 = FP32 MFMA with FP32 sums over each wavefront's
 * K share (at most SGO_GRAM_KC/4 terms) and FP64 sums of those),
 * "SGO_PCG_TRIAL" (cap of the PCG trial step on the largest atom
 * displacement, milli-bohr, default 100), "SGO_PCG_FLOOR" (eigenvalue floor
 * of the PCG preconditioner, thousandths of max|tau|, default 100),
 * "SGO_JAC_GRID" (band count from which the subspace products and Jacobi
 * rounds run over the whole GPU instead of one workgroup per candidate,
 * default 160), "SGO_PLANE_GROUP" (consecutive z-planes per four-wavefront
 * workgroup of the FP32 register H psi plane kernel, 2..8; 1 = one plane per
 * wavefront; by default the size that keeps the most lanes busy while two
 * groups still share a compute unit's LDS, or 1 where no group saves 10%),
 * "SGO_COMPACT" (1, the default: once some candidates of a population have
 * converged, the SCF iterations launch over the active ones only; 0: every
 * launch spans the whole population, converged candidates returning at once).
 * value <= 0 restores the default (or the environment variable of the same
 * name).  SGO_EINVAL for an unknown key.  sgo_get_tuning returns the value
 * set (0 if none). */
int sgo_set_tuning(const char* key, int value);
int sgo_get_tuning(const char* key);

/* Measurement hooks (process-wide): from sgo_profile_begin until
 * sgo_profile_end, every launch of the kernel named `kernel` (for example
 * "k_plane_hpsi") is bracketed by a pair of HIP events recorded on the stream
 * it is launched on.  sgo_profile_end waits for the events and returns the
 * number of launches, their summed duration in milliseconds and (nullable)
 * the sum over those launches of the candidates still active in each (a
 * population launch returns at once for converged candidates).  For kernels
 * whose traffic depends on the call (the band rotation / accumulation
 * k_gemm_acc), `cand_rows` (nullable) returns the sum over the launches of
 * active candidates times the coefficient rows of length K one candidate's
 * share reads or writes (0 for kernels that do not state it). */
int sgo_profile_begin(const char* kernel);
int sgo_profile_end(int* launches, double* total_ms, long long* cand_launches,
                    long long* cand_rows, double* union_ms);

/* ---- Population of candidates, solved together (Section 2.4 last
 * paragraph: the relaxations of one generation may run side by side).  The
 * batch holds up to `capacity` candidates with their own cells, atoms,
 * cutoffs, grids and band counts; every kernel launch covers all active
 * candidates, and converged candidates are masked out. */
int sgo_batch_create(sgo_batch** out, int device, int precision, int capacity);
int sgo_batch_destroy(sgo_batch* b);
int sgo_batch_set_stream(sgo_batch* b, void* hip_stream);
/* Caller allocator for the candidates' arenas (as sgo_set_allocator). */
int sgo_batch_set_allocator(sgo_batch* b, void* (*alloc)(size_t bytes, void* user),
                            void (*dealloc)(void* ptr, void* user), void* user);
int sgo_batch_set_species(sgo_batch* b, int id, const sgo_species* sp);
/* Append a candidate of the generation's population (Section 2.4, last
 * paragraph; Section 2.2: the individuals of one DE generation are relaxed
 * independently); *index_out receives its index (add order).  Arguments as
 * for sgo_set_cell, sgo_set_atoms and sgo_set_cutoff; SGO_EINVAL on the same
 * conditions, or when the batch is full. */
int sgo_batch_add(sgo_batch* b, const double lattice[9], int natoms, const int* species,
                  const double* pos, double ecut, const int fft[3], int nbands,
                  int occ_kind, double sigma, int* index_out);
/* Move the atoms of candidate i (warm start kept). */
int sgo_batch_set_atoms(sgo_batch* b, int i, const double* pos);
/* Solve every candidate: the self-consistent loop of Section 2.4 with the
 * all-band CG of Algorithm 1, for all candidates of the population at once
 * (Section 2.4, last paragraph: the relaxations of a generation run side by
 * side).  energies [n], forces [sum natoms*3] in add order,
 * status [n] per candidate (SGO_OK, SGO_ENOTCONV or SGO_ENUMERIC); any of the
 * three may be NULL.  Returns the worst status. */
int sgo_batch_scf(sgo_batch* b, const sgo_scf_opts* opts, double* energies, double* forces,
                  int* status);
/* Solve n batches at once, each from its own host thread on its own stream
 * (sgo_batch_set_stream; the batches must not share a stream or a handle).
 * A population split into a few batches keeps the GPU busy while each
 * batch waits in its latency-bound phases (the FP64 subspace solves, the SCF
 * control, the status read-back).  energies, forces and status are laid out
 * as for sgo_batch_scf, concatenated in batch order (each nullable); each
 * batch's own error text stays with its handle.  Returns the first error
 * other than SGO_ENOTCONV/SGO_ENUMERIC that a batch returned (batch order),
 * else the worst status as for sgo_batch_scf.  The measurement hooks
 * (sgo_profile_begin/end) count the launches of every batch.  The batches
 * overlap only if their streams sit on distinct hardware queues: HIP's
 * default of 4 queues per process is shared with the runtime's own streams,
 * so set GPU_MAX_HW_QUEUES to at least n + 4 before the runtime starts (with
 * the default, 4 batches ran 30% slower than on 8 queues). */
int sgo_batches_scf(sgo_batch* const* batches, int n, const sgo_scf_opts* opts,
                    double* energies, double* forces, int* status);
int sgo_batch_info(sgo_batch* b, int i, sgo_scf_info* info);
/* Conventional CG relaxation of every candidate, nsteps steps (Section 2.3
 * names CG among the relaxation options): Polak-Ribiere directions built
 * from the Hellmann-Feynman forces, a secant line search on F.d (trial step
 * 0.1 bohr along the largest direction component, capped by twice the
 * previous step; secant step clamped to [0.1, 4] x trial), two batched
 * warm-started evaluations per step.  energies [n][nsteps+1] (nullable)
 * receives the energy before the first and after each step; forces and
 * positions [sum natoms*3] (nullable) the final ones, status [n] per
 * candidate.  Returns the worst status. */
int sgo_batch_relax_cg(sgo_batch* b, int nsteps, const sgo_scf_opts* opts, double* energies,
                       double* forces, double* positions, int* status);
/* Preconditioned CG relaxation (Section 2.3, the PCG option): a Morse pair
 * force field E = sum_{i<j} D [(1 - e^{-a (r - r0)})^2 - 1] is fitted to
 * every (positions, forces) sample of the candidate's relaxation so far
 * (sgo_ff_fit), its Hessian inverted over the modes with non-zero eigenvalue
 * (sgo_ff_preconditioner) gives P, and the CG directions become
 * d = P F + beta d with beta = max(0, F_new.P(F_new - F) / F.P F).  Trial
 * step min(1, 0.1 bohr / max_atom |d|), capped by twice the previous step,
 * then the secant step of sgo_batch_relax_cg; two batched evaluations per
 * step.  P is rebuilt every `refit` steps (0: only at the start).  Outputs
 * as sgo_batch_relax_cg; params (nullable) [n][3] = the last fit (D, a, r0)
 * of each candidate. */
int sgo_batch_relax_pcg(sgo_batch* b, int nsteps, int refit, const sgo_scf_opts* opts,
                        double* energies, double* forces, double* positions, double* params,
                        int* status);

/* Curved line search relaxation (Section 2.3, the CLS option; the paper
 * gives its outline only, these steps re-derive it).  Before every step the
 * Morse field of sgo_batch_relax_pcg is refitted to all samples, and its
 * steepest-descent path from the current structure (sgo_ff_guided_curve) is
 * the guided curve x(s); the DFT energy is minimised along the curve with
 * the secant step on g(s) = -F(x(s)).x'(s): trial s1 = min(curve length,
 * 0.3 bohr, twice the previous step), secant s2 clamped to [0.1, 4] s1 and
 * to the curve's end.  Two batched evaluations per step.  Outputs as
 * sgo_batch_relax_pcg. */
int sgo_batch_relax_cls(sgo_batch* b, int nsteps, const sgo_scf_opts* opts, double* energies,
                        double* forces, double* positions, double* params, int* status);

/* Force-field pieces of the PCG preconditioner (host code).  params =
 * {D (Ha), a (1/bohr), r0 (bohr)}; pairs by minimum image over the 27
 * neighbouring cells.  sgo_ff_morse: energy and forces (each nullable).
 * sgo_ff_hessian: analytic Hessian [3n][3n] (row-major, coordinate 3I + k).
 * sgo_ff_fit: least-squares fit of the forces of nsamples geometries
 * (pos, forces [nsamples][natoms][3]): D is the linear optimum for each
 * (a, r0), taken from a 51 x 41 grid (a = 0.5 ... 3.0, r0 = 0.80 ... 1.60
 * of the smallest sampled distance) and refined by a compass search inside
 * that box (30 step halvings); defaults (0.1, 1.0, smallest distance) when no grid point gives
 * D > 0.  sgo_ff_preconditioner: P [m][m] = sum over eigenpairs (tau, v) of
 * H with |tau| > 1e-6 max|tau| of v v^T / max(|tau|, 0.1 max|tau|): the
 * translations (tau = 0) are dropped and negative curvature counts by its
 * magnitude, so P is positive semi-definite. */
int sgo_ff_morse(const double lattice[9], int natoms, const double* pos, const double params[3],
                 double* energy, double* forces);
int sgo_ff_hessian(const double lattice[9], int natoms, const double* pos, const double params[3],
                   double* H);
int sgo_ff_fit(const double lattice[9], int natoms, int nsamples, const double* pos,
               const double* forces, double params[3]);
int sgo_ff_preconditioner(int m, const double* H, double* P);
/* Guided curve of the CLS relaxation: nodes x_0 = x0, x_{k+1} = x_k +
 * 0.02 F(x_k) / max_atom |F(x_k)| (the steepest-descent path of the Morse
 * field, the most-forced atom moving 0.02 bohr per node) until
 * max_atom |F| < 1e-3 Ha/bohr or 200 steps.  nodes [max_nodes][natoms][3];
 * *nnodes = number written (at most 201).  SGO_EINVAL when max_nodes is too
 * small. */
int sgo_ff_guided_curve(const double lattice[9], int natoms, const double params[3],
                        const double* x0, int max_nodes, double* nodes, int* nnodes);

/* Drop the warm-start wavefunctions of every candidate (next solve is cold). */
int sgo_batch_reset(sgo_batch* b);
/* Read back the state of candidate i after sgo_batch_scf (each pointer may be
 * NULL): sizes info[10] as in sgo_grid_info; Miller indices [npw_half*3] of
 * its basis; bands psi [nbands][2*npw_half] in the packed layout described at
 * sgo_basis_millers (FP64 copies of the stored precision), eigenvalues and
 * occupations [nbands]; output density rho and input potential veff
 * [N3][N2][N1]; energy terms. */
int sgo_batch_get_state(sgo_batch* b, int i, int* info, int* millers, double* psi, double* eig,
                        double* occ, double* rho, double* veff, sgo_energy_terms* terms);
/* Input density of candidate i's last SCF iteration, rho_in [N3][N2][N1]
 * (the mixed density of Section 2.4 from which the V_eff of
 * sgo_batch_get_state was built); SGO_ESTATE before a solve. */
int sgo_batch_get_input_density(sgo_batch* b, int i, double* rho_in);
/* Fixed-basis stress [n][3][3] of every solved candidate (conventions of
 * sgo_stress); candidates not yet solved get SGO_ESTATE. */
int sgo_batch_stress(sgo_batch* b, double* stress);
int sgo_batch_size(sgo_batch* b, int* n);

/* ---- Structure-search operators (Section 2.2: initialisation with distance
 * checks, mutation, cut-and-splice crossover, greedy selection).  Host code,
 * no device work.  Structures are Cartesian positions [natoms][3] in bohr in
 * one fixed cell; every random number is an argument, so equal draws give
 * equal results.  Outputs are caller-owned. */
enum { SGO_DE_TRIANGLE = 0, SGO_DE_CLASSIC = 1 };
enum { SGO_DE_PLANE = 0, SGO_DE_SPHERE = 1 };

/* Mutant from three donors x1..x3 (ncoord doubles each) with fitness values
 * f1..f3.  SGO_DE_TRIANGLE: Eq. 2, v = (x1+x2+x3)/3 + (p2-p1)(x1-x2) +
 * (p3-p2)(x2-x3) + (p1-p3)(x3-x1), p_k = |f_k| / (|f1|+|f2|+|f3|) (1/3 each
 * when all are zero).  SGO_DE_CLASSIC: Eq. 1, v = x3 + F (x1 - x2).
 * SGO_EINVAL for an unknown scheme or NULL arrays. */
int sgo_de_mutate(int ncoord, const double* x1, const double* x2, const double* x3, double f1,
                  double f2, double f3, int scheme, double F, double* v);

/* Plane cut-and-splice (Section 2.2, Fig. 2a).  Parents p1, p2 [natoms][3]
 * share the species array `species` [natoms].  The child takes P1's atoms
 * strictly on the +n side of the plane through P1's centroid and P2's atoms
 * on the other side of (or on) the plane through P2's centroid, translated
 * by centroid(P1) - centroid(P2).  If the per-species counts differ from
 * P1's, n turns about `axis` (made orthogonal to n) to the first angle in
 * [0, 2 pi) that gives them; theta (nullable) receives that angle.  Child
 * slot order: for each species, P1's atoms (ascending index) fill its slots
 * first, then P2's.  source (nullable) [natoms][2] = (parent 0/1, atom
 * index) of each child atom.  SGO_ENUMERIC when no angle gives P1's
 * composition; SGO_EINVAL for a zero normal or an axis parallel to it. */
int sgo_de_cross_plane(int natoms, const int* species, const double* p1, const double* p2,
                       const double normal[3], const double axis[3], double* child, int* source,
                       double* theta);

/* Sphere cut-and-splice (Section 2.2, Fig. 2b).  Spheres of `radius` about
 * each parent's centroid + offset.  The child takes P2's atoms inside its
 * sphere (translated as above) and, per species, the atoms of P1 farthest
 * from its sphere centre that complete P1's count.  Slot order and source as
 * for the plane scheme. */
int sgo_de_cross_sphere(int natoms, const int* species, const double* p1, const double* p2,
                        const double offset[3], double radius, double* child, int* source);

/* Smallest interatomic distance (minimum image over the 27 neighbouring
 * cells; +inf for fewer than two atoms). */
int sgo_de_min_distance(const double lattice[9], int natoms, const double* pos, double* dmin);

/* Structure similarity: mean absolute difference of the sorted
 * pair-distance lists (bohr; 0 for identical structures up to permutation,
 * translation and rotation when no distance wraps). */
int sgo_de_similarity(const double lattice[9], int natoms, const double* pa, const double* pb,
                      double* s);

/* Random initial structure (Section 2.2, population initialisation).
 * region 0: whole cell, fractional (u1,u2,u3); 1: ball of radius params[0]
 * about the cell centre, r = R u1^(1/3), cos(polar) = 2u2-1, azimuth 2 pi u3;
 * 2: slab, fractional x = u1, y = u2 and z within params[0] bohr of the
 * middle plane.  Each trial atom consumes three of the `nuniform` uniforms
 * in [0,1); a trial closer than dmin (minimum image) to a placed atom is
 * dropped.  *used (nullable) = uniforms consumed.  SGO_ENUMERIC when they
 * run out before natoms atoms are placed. */
int sgo_de_init_positions(const double lattice[9], int natoms, int region, const double* params,
                          double dmin, const double* uniforms, int nuniform, double* pos,
                          int* used);

/* Perturbed cell for a new individual (Section 2.2, population
 * initialisation): lattice vector k scaled by 1 + delta (2 u[k] - 1).
 * SGO_EINVAL for NULL arrays or delta < 0. */
int sgo_de_jitter_cell(const double lattice[9], double delta, const double u[3], double out[9]);

/* Greedy selection: take[i] = 1 when the child converged (child_status NULL
 * or SGO_OK) and e_child[i] < e_parent[i]. */
int sgo_de_select(int n, const double* e_parent, const double* e_child, const int* child_status,
                  int* take);

/* One generation on a population batch: for each target i, mutant from the
 * donors of its first acceptable draw, crossover with the target (P1 = the
 * mutant, P2 = the target), child rejected when two atoms are closer than
 * max(dmin, 1e-3 bohr) (the evaluator refuses coincident atoms) or, with
 * sim_tol > 0, less than sim_tol from any parent; then relax_steps batched CG
 * steps (sgo_batch_relax_cg) of every child and greedy selection.  A target
 * whose draws are all rejected relaxes its own structure instead. */
typedef struct {
  int mutation;       /* SGO_DE_TRIANGLE or SGO_DE_CLASSIC */
  int crossover;      /* SGO_DE_PLANE or SGO_DE_SPHERE */
  double F;           /* Eq. 1 scale (classic mutation) */
  int fitness_shift;  /* 1: fitness = E - min E of the parents (lower energy,
                         larger weight in Eq. 2); 0: fitness = E */
  int relax_steps;    /* CG steps per child, >= 0 */
  double dmin;        /* bohr */
  double sim_tol;     /* bohr; 0 disables the similarity check */
  int attempts;       /* draws per target, >= 1 */
} sgo_de_opts;

typedef struct {      /* random numbers of one attempt for one target */
  int r[3];           /* donor indices, distinct and different from the target */
  double normal[3];   /* plane scheme */
  double axis[3];
  double offset[3];   /* sphere scheme */
  double radius;
} sgo_de_draw;

/* parents [sum natoms*3] and e_parent [n] describe the current generation in
 * the batch's add order (every candidate must share one species array and
 * cell); draws [n][attempts].  Outputs (each nullable): trial [sum natoms*3]
 * the children before relaxation, attempt_used [n] (-1: no draw accepted),
 * e_trial [n] the relaxed children's energies, survivors [sum natoms*3] and
 * e_survivor [n] the next generation, take [n] the selection, status [n].
 * The batch's candidates are left at the survivors' positions.  SGO_EINVAL
 * for invalid draws or options; otherwise the worst relaxation status. */
int sgo_batch_de_generation(sgo_batch* b, const sgo_de_opts* de, const sgo_scf_opts* opts,
                            const double* parents, const double* e_parent,
                            const sgo_de_draw* draws, double* trial, int* attempt_used,
                            double* e_trial, double* survivors, double* e_survivor, int* take,
                            int* status);
const char* sgo_batch_last_error(const sgo_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* SGO_H */
