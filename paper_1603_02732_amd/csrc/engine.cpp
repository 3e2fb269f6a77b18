// Host side of the engine: plane-wave basis bookkeeping, device memory
// layout, the SCF driver (Section 2.4) around the all-band CG eigensolver
// (Algorithm 1), and the C-ABI declared in sgo.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/sgo.h"
#include "common.hpp"
#include "de.hpp"
#include "launch.hpp"
#include "pcg.hpp"

namespace sgo {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Error(SGO_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

static const double kPiH = 3.14159265358979323846;

static int g_lds_limit = 64 * 1024;

// Launch-shape tuning parameters: values set through sgo_set_tuning (by the
// autotuner) take precedence over the environment, then the defaults.
static std::map<std::string, int> g_tuning;
static int tune(const char* name, int def) {
  auto it = g_tuning.find(name);
  if (it != g_tuning.end() && it->second > 0) return it->second;
  const char* v = std::getenv(name);
  if (!v || !*v) return def;
  const int x = std::atoi(v);
  return x > 0 ? x : def;
}

void allow_lds(const void* kernel) {
  hipFuncAttributes a;
  HIPCHK(hipFuncGetAttributes(&a, kernel));
  const int dyn = g_lds_limit - (int)a.sharedSizeBytes;
  if (dyn > 0) HIPCHK(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, dyn));
}

struct ProfState {
  bool on = false;
  std::string name;
  long long cand_launches = 0;  // sum over profiled launches of the active candidates
  long long cand_rows = 0;      // sum over profiled launches of active x row passes
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t used = 0;
};
// Process-wide measurement hooks.  Batches may be solved from several host
// threads at once (sgo_batches_scf): the shared state is guarded, and what
// belongs to one thread's launch sequence (candidates active in its current
// launches, the event pair it has open, whether it is capturing a graph) is
// thread-local.
static ProfState g_prof;
static std::mutex g_prof_mu;
static thread_local bool g_capturing = false;  // no event records inside a captured graph
static thread_local int t_active = 0;
static thread_local size_t t_pending = 0;

void prof_before(const char* name, hipStream_t s) {
  if (!g_prof.on || g_capturing || g_prof.name != name) return;
  hipEvent_t e;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.used + 2 > g_prof.ev.size()) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t x;
        HIPCHK(hipEventCreate(&x));
        g_prof.ev.push_back(x);
      }
    }
    t_pending = g_prof.used;
    g_prof.used += 2;
    e = g_prof.ev[t_pending];
  }
  HIPCHK(hipEventRecord(e, s));
}
void prof_after(const char* name, hipStream_t s, long long rows) {
  if (!g_prof.on || g_capturing || g_prof.name != name) return;
  hipEvent_t e;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    e = g_prof.ev[t_pending + 1];
    g_prof.cand_launches += t_active;
    g_prof.cand_rows += (long long)t_active * rows;
  }
  HIPCHK(hipEventRecord(e, s));
}

bool host_sync_allowed() { return !g_capturing; }

// Device LDS limit and the kernels' dynamic-LDS attributes, once per
// process (handles may be created from several threads).
static std::once_flag g_config_once;
void configure_once(int device) {
  std::call_once(g_config_once, [device] {
    int lim = 0;
    HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    g_lds_limit = lim;
    (void)hipGetLastError();
    configure_kernels();
  });
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(SGO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void throw_unsupported(const char* what) { throw Error(SGO_EINVAL, what); }

void check_launch(const char* name) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    throw Error(SGO_EDEVICE, std::string("launch of ") + name + " failed: " + hipGetErrorString(e));
}

// --------------------------------------------------------------- utilities
static bool fft_plan(int n, FftPlan& p) {
  p.n = n;
  p.nstage = 0;
  int m = n;
  const int order[4] = {4, 2, 3, 5};
  for (int r : order) {
    while (m % r == 0) {
      if (p.nstage >= kMaxStages) return false;
      p.radix[p.nstage++] = r;
      m /= r;
    }
  }
  return m == 1 && n >= 1 && n <= kMaxFftN;
}

static void inv3(const double* A, double* Ai, double* det) {
  const double a = A[0], b = A[1], c = A[2], d = A[3], e = A[4], f = A[5], g = A[6], h = A[7],
               i = A[8];
  const double D = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  *det = D;
  Ai[0] = (e * i - f * h) / D;
  Ai[1] = (c * h - b * i) / D;
  Ai[2] = (b * f - c * e) / D;
  Ai[3] = (f * g - d * i) / D;
  Ai[4] = (a * i - c * g) / D;
  Ai[5] = (c * d - a * f) / D;
  Ai[6] = (d * h - e * g) / D;
  Ai[7] = (b * g - a * h) / D;
  Ai[8] = (a * e - b * d) / D;
}

// ------------------------------------------------------------- candidates
struct HostCand {
  // inputs
  double A[9];
  int nat = 0;
  std::vector<int> spec;
  std::vector<double> pos;
  double ecut = 0;
  int N[3] = {0, 0, 0};
  int nb = 0;
  int occ_kind = 0;
  double sigma = 0;
  // derived
  double omega = 0, B[9];
  double nelec = 0;
  int nocc = 0;
  int npwh = 0, K = 0, Kp = 0, nsp = 0, nst = 0, npair = 0, nproj = 0, ntot = 0;
  std::vector<int> gmill, gmeta, sp_off, stick_xy, proj_atom, proj_lm;
  int pl_nx = 0, pl_nxl = 0, pl_sx = 1;  // active plane columns (register FFT kernels)
  int N_req[3] = {0, 0, 0}, nb_req = 0;  // as requested (0: automatic)
  std::vector<double> kin, hproj, proj_r;
  FftPlan plan[3];
  double ew_eta = 0, ew_rcut = 0, ew_gcut = 0;
  int ew_m[3], ew_n[3], ew_ng = 0, ew_nimg = 0;
  int hist_len = kMaxHist;
  int dens_chunks = 1;
  size_t red_doubles = 0;
  // device
  char* mem = nullptr;
  size_t mem_size = 0;
  CandDesc d;
  bool built = false;
  bool have_psi = false;
  bool have_scf = false;
  sgo_scf_info info{};
  int status = SGO_OK;
};

struct SpeciesHost {
  bool set = false;
  SpeciesDev d;
};

class Engine {
 public:
  Engine(int device, int precision, int capacity)
      : device_(device), prec_(precision), capacity_(capacity) {
    if (precision != SGO_FP64 && precision != SGO_FP32 && precision != SGO_FP32_BF16PROJ)
      throw Error(SGO_EINVAL, "bad precision");
    if (capacity < 1) throw Error(SGO_EINVAL, "capacity must be >= 1");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(SGO_EINVAL, "no such HIP device");
    HIPCHK(hipSetDevice(device));
    configure_once(device);
    HIPCHK(hipMalloc(&d_species_, sizeof(SpeciesDev) * kMaxSpecies));
    HIPCHK(hipMemset(d_species_, 0, sizeof(SpeciesDev) * kMaxSpecies));
    HIPCHK(hipMalloc(&d_iter_, 64));
    HIPCHK(hipMemset(d_iter_, 0, 64));
    species_.resize(kMaxSpecies);
  }
  ~Engine() {
    (void)hipSetDevice(device_);
    k_free();
    for (auto& c : cands_) free_cand(c);
    if (d_species_) (void)hipFree(d_species_);
    if (d_desc_) (void)hipFree(d_desc_);
    if (d_desc_act_) (void)hipFree(d_desc_act_);
    if (d_iter_) (void)hipFree(d_iter_);
    if (d_scal_all_) (void)hipFree(d_scal_all_);
    if (h_scal_all_) (void)hipHostFree(h_scal_all_);
    if (d_jac_done_) (void)hipFree(d_jac_done_);
    if (h_jac_done_) (void)hipHostFree(h_jac_done_);
    if (own_stream_) (void)hipStreamDestroy(own_stream_);
  }

  void set_stream(void* s) { stream_ = (hipStream_t)s; }

  void set_species(int id, const sgo_species* sp) {
    if (id < 0 || id >= kMaxSpecies || !sp) throw Error(SGO_EINVAL, "bad species id or pointer");
    if (!(sp->Z >= 0) || sp->nkb < 0 || sp->nkb > 4) throw Error(SGO_EINVAL, "bad species data");
    if (sp->local_kind != SGO_LOCAL_AH && sp->local_kind != SGO_LOCAL_GAUSS)
      throw Error(SGO_EINVAL, "unknown local potential kind");
    if (!(sp->p[0] > 0)) throw Error(SGO_EINVAL, "local potential width must be positive");
    SpeciesDev d{};
    d.Z = sp->Z;
    d.local_kind = sp->local_kind;
    d.nkb = sp->nkb;
    for (int k = 0; k < 3; ++k) d.p[k] = sp->p[k];
    for (int k = 0; k < sp->nkb; ++k) {
      if (sp->kb_l[k] < 0 || sp->kb_l[k] > 1 || !(sp->kb_r[k] > 0))
        throw Error(SGO_EINVAL, "KB channels must have l in {0,1} and r > 0");
      d.kb_l[k] = sp->kb_l[k];
      d.kb_r[k] = sp->kb_r[k];
      d.kb_h[k] = sp->kb_h[k];
    }
    d.rho0_width = sp->rho0_width > 0 ? sp->rho0_width : 0.5;
    species_[id].set = true;
    species_[id].d = d;
    HIPCHK(hipSetDevice(device_));
    HIPCHK(hipMemcpy(d_species_ + id, &d, sizeof(d), hipMemcpyHostToDevice));
    for (auto& c : cands_) {
      c.built = false;
      c.have_psi = false;
      c.have_scf = false;
    }
  }

  int add(const double* lat, int nat, const int* spec, const double* pos, double ecut,
          const int* fft, int nb, int occ_kind, double sigma) {
    if ((int)cands_.size() >= capacity_) throw Error(SGO_EINVAL, "batch is full");
    HostCand c;
    fill_cand(c, lat, nat, spec, pos, ecut, fft, nb, occ_kind, sigma);
    cands_.push_back(std::move(c));
    desc_dirty_ = true;
    return (int)cands_.size() - 1;
  }

  void fill_cand(HostCand& c, const double* lat, int nat, const int* spec, const double* pos,
                 double ecut, const int* fft, int nb, int occ_kind, double sigma) {
    if (!lat || !spec || !pos || !fft) throw Error(SGO_EINVAL, "NULL argument");
    if (nat <= 0) throw Error(SGO_EINVAL, "natoms must be positive");
    if (!(ecut > 0)) throw Error(SGO_EINVAL, "ecut must be positive");
    if (nb < 0) throw Error(SGO_EINVAL, "nbands must be positive (or 0: automatic)");
    if (fft[0] < 0 || fft[1] < 0 || fft[2] < 0) throw Error(SGO_EINVAL, "negative FFT length");
    if (occ_kind != SGO_OCC_FIXED && occ_kind != SGO_OCC_FERMI)
      throw Error(SGO_EINVAL, "unknown occupation kind");
    if (occ_kind == SGO_OCC_FERMI && !(sigma > 0)) throw Error(SGO_EINVAL, "sigma must be > 0");
    std::memcpy(c.A, lat, sizeof(double) * 9);
    double Ai[9], det;
    inv3(c.A, Ai, &det);
    if (!(std::fabs(det) > 1e-12)) throw Error(SGO_EINVAL, "cell volume must be positive");
    c.nat = nat;
    c.spec.assign(spec, spec + nat);
    for (int I = 0; I < nat; ++I)
      if (spec[I] < 0 || spec[I] >= kMaxSpecies || !species_[spec[I]].set)
        throw Error(SGO_EINVAL, "atom uses an unregistered species");
    c.pos.assign(pos, pos + 3 * nat);
    check_distances(c);
    c.ecut = ecut;
    for (int k = 0; k < 3; ++k) c.N[k] = c.N_req[k] = fft[k];
    c.nb = c.nb_req = nb;
    c.occ_kind = occ_kind;
    c.sigma = sigma;
    c.built = false;
    c.have_psi = false;
    c.have_scf = false;
    build_basis(c);  // validates grid and bands now, so errors surface at the call
  }

  void check_distances(const HostCand& c) {
    double Ai[9], det;
    inv3(c.A, Ai, &det);
    for (int I = 0; I < c.nat; ++I)
      for (int J = I + 1; J < c.nat; ++J) {
        double d[3], f[3];
        for (int k = 0; k < 3; ++k) d[k] = c.pos[3 * I + k] - c.pos[3 * J + k];
        // fractional, minimum image: d = f A  (rows of A are lattice vectors)
        for (int k = 0; k < 3; ++k) f[k] = d[0] * Ai[0 * 3 + k] + d[1] * Ai[1 * 3 + k] + d[2] * Ai[2 * 3 + k];
        for (int k = 0; k < 3; ++k) f[k] -= std::round(f[k]);
        double r2 = 0;
        for (int k = 0; k < 3; ++k) {
          const double x = f[0] * c.A[0 * 3 + k] + f[1] * c.A[1 * 3 + k] + f[2] * c.A[2 * 3 + k];
          r2 += x * x;
        }
        if (r2 < 1e-6) throw Error(SGO_EINVAL, "two atoms closer than 1e-3 bohr");
      }
  }

  // Half-sphere basis, sticks, maps, projector list, Ewald ranges.
  void build_basis(HostCand& c) {
    double Ai[9], det;
    inv3(c.A, Ai, &det);
    c.omega = std::fabs(det);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) c.B[i * 3 + k] = 2.0 * kPiH * Ai[k * 3 + i];  // B = 2 pi A^-T
    const double gmax = std::sqrt(2.0 * c.ecut);
    int mm[3];
    for (int i = 0; i < 3; ++i) {
      const double an = std::sqrt(c.A[3 * i] * c.A[3 * i] + c.A[3 * i + 1] * c.A[3 * i + 1] +
                                  c.A[3 * i + 2] * c.A[3 * i + 2]);
      mm[i] = (int)std::floor(gmax * an / (2 * kPiH)) + 1;
    }
    std::vector<std::array<int, 3>> full;
    int mabs[3] = {0, 0, 0};
    for (int a = -mm[0]; a <= mm[0]; ++a)
      for (int b = -mm[1]; b <= mm[1]; ++b)
        for (int g = -mm[2]; g <= mm[2]; ++g) {
          double G[3];
          for (int k = 0; k < 3; ++k) G[k] = a * c.B[k] + b * c.B[3 + k] + g * c.B[6 + k];
          const double e = 0.5 * (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
          if (e <= c.ecut) {
            full.push_back({a, b, g});
            mabs[0] = std::max(mabs[0], std::abs(a));
            mabs[1] = std::max(mabs[1], std::abs(b));
            mabs[2] = std::max(mabs[2], std::abs(g));
          }
        }
    for (int i = 0; i < 3; ++i) {
      if (c.N_req[i] == 0) {
        // automatic grid: smallest 2^a 3^b 5^c >= max(|a_i| / 0.375, 2 m_max + 1)
        const double an = std::sqrt(c.A[3 * i] * c.A[3 * i] + c.A[3 * i + 1] * c.A[3 * i + 1] +
                                    c.A[3 * i + 2] * c.A[3 * i + 2]);
        const int want = std::max((int)std::ceil(an / 0.375 - 1e-9), 2 * mabs[i] + 1);
        int n = want;
        FftPlan tmp;
        while (n <= kMaxFftN && !fft_plan(n, tmp)) ++n;
        if (n > kMaxFftN) throw Error(SGO_EINVAL, "automatic FFT grid exceeds 128 points");
        c.N[i] = n;
      }
      if (c.N[i] < 2 * mabs[i] + 1)
        throw Error(SGO_EINVAL, "FFT grid too small for the wavefunction sphere");
      if (!fft_plan(c.N[i], c.plan[i]))
        throw Error(SGO_EINVAL, "FFT lengths must factor into 2,3,5 and be <= 128");
    }
    c.ntot = c.N[0] * c.N[1] * c.N[2];
    // sticks: canonical (m1,m2) with m2 > 0 or (m2 == 0 and m1 >= 0)
    std::map<std::pair<int, int>, int> seen;
    for (auto& m : full) seen[{m[0], m[1]}] = 1;
    std::vector<std::pair<int, int>> canon;
    for (auto& kv : seen) {
      const int a = kv.first.first, b = kv.first.second;
      if ((a == 0 && b == 0)) continue;
      if (b > 0 || (b == 0 && a > 0)) canon.push_back({a, b});
    }
    std::sort(canon.begin(), canon.end(), [](const std::pair<int, int>& x,
                                             const std::pair<int, int>& y) {
      return x.second != y.second ? x.second < y.second : x.first < y.first;
    });
    std::map<std::pair<int, int>, int> stick_of, pair_of;
    std::vector<std::pair<int, int>> sticks;
    sticks.push_back({0, 0});
    stick_of[{0, 0}] = 0;
    pair_of[{0, 0}] = 0;
    for (size_t q = 0; q < canon.size(); ++q) {
      auto s = canon[q];
      std::pair<int, int> ms = {-s.first, -s.second};
      stick_of[s] = (int)sticks.size();
      sticks.push_back(s);
      stick_of[ms] = (int)sticks.size();
      sticks.push_back(ms);
      pair_of[s] = (int)q + 1;
      pair_of[ms] = (int)q + 1;
    }
    c.nsp = (int)canon.size() + 1;
    c.nst = (int)sticks.size();
    // half sphere ordered by stick pair, then m3, m2, m1
    std::vector<std::array<int, 4>> half;  // pair, m1, m2, m3
    for (auto& m : full) {
      const bool in_half = m[2] > 0 || (m[2] == 0 && (m[1] > 0 || (m[1] == 0 && m[0] >= 0)));
      if (in_half) half.push_back({pair_of[{m[0], m[1]}], m[0], m[1], m[2]});
    }
    std::sort(half.begin(), half.end(), [](const std::array<int, 4>& x, const std::array<int, 4>& y) {
      if (x[0] != y[0]) return x[0] < y[0];
      if (x[3] != y[3]) return x[3] < y[3];
      if (x[2] != y[2]) return x[2] < y[2];
      return x[1] < y[1];
    });
    c.npwh = (int)half.size();
    c.K = 2 * c.npwh;
    c.Kp = (c.K + 31) / 32 * 32;
    if (half.empty() || half[0][1] != 0 || half[0][2] != 0 || half[0][3] != 0)
      throw Error(SGO_EINVAL, "internal: G = 0 must lead the basis");
    c.gmill.resize(3 * c.npwh);
    c.gmeta.resize(c.npwh);
    c.kin.resize(c.npwh);
    c.sp_off.assign(c.nsp + 1, 0);
    for (int g = 0; g < c.npwh; ++g) {
      const auto& h = half[g];
      c.gmill[3 * g] = h[1];
      c.gmill[3 * g + 1] = h[2];
      c.gmill[3 * g + 2] = h[3];
      const int s = stick_of[{h[1], h[2]}];
      c.gmeta[g] = s | (((h[3] % c.N[2] + c.N[2]) % c.N[2]) << 20);
      double G[3];
      for (int k = 0; k < 3; ++k) G[k] = h[1] * c.B[k] + h[2] * c.B[3 + k] + h[3] * c.B[6 + k];
      c.kin[g] = 0.5 * (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
      c.sp_off[h[0] + 1]++;
    }
    for (int q = 0; q < c.nsp; ++q) c.sp_off[q + 1] += c.sp_off[q];
    c.stick_xy.resize(c.nst);
    int m1max = 0;
    for (int s = 0; s < c.nst; ++s) {
      const int i1 = ((sticks[s].first % c.N[0]) + c.N[0]) % c.N[0];
      const int i2 = ((sticks[s].second % c.N[1]) + c.N[1]) % c.N[1];
      c.stick_xy[s] = i1 | (i2 << 16);
      m1max = std::max(m1max, std::abs(sticks[s].first));
    }
    // active x columns of the planes: x <= m1max and x >= N1 - m1max
    c.pl_nx = std::min(2 * m1max + 1, c.N[0]);
    c.pl_nxl = c.pl_nx == c.N[0] ? c.N[0] : m1max + 1;
    c.pl_sx = c.pl_nx | 1;
    // electrons, occupations
    c.nelec = 0;
    for (int I = 0; I < c.nat; ++I) c.nelec += species_[c.spec[I]].d.Z;
    if (c.nb_req == 0) {
      // automatic band count: even ceil(1.2 N_occ)
      const int nocc = (int)std::ceil(0.5 * c.nelec - 1e-9);
      int nb = (int)std::ceil(1.2 * nocc - 1e-9);
      if (nb % 2) ++nb;
      c.nb = std::max(nb, nocc + 1);
    } else {
      c.nb = c.nb_req;
    }
    if (c.occ_kind == SGO_OCC_FIXED) {
      const double h = 0.5 * c.nelec;
      c.nocc = (int)std::llround(h);
      if (std::fabs(c.nocc - h) > 1e-9) throw Error(SGO_EINVAL, "fixed occupations need an even electron count");
      if (c.nocc > c.nb) throw Error(SGO_EINVAL, "nbands cannot hold the electrons");
    } else {
      c.nocc = 0;
      if (c.nelec > 2.0 * c.nb - 1e-9) throw Error(SGO_EINVAL, "nbands cannot hold the electrons");
    }
    c.npair = (c.nb + 1) / 2;
    // projectors
    c.proj_atom.clear();
    c.proj_lm.clear();
    c.proj_r.clear();
    c.hproj.clear();
    for (int I = 0; I < c.nat; ++I) {
      const SpeciesDev& s = species_[c.spec[I]].d;
      for (int k = 0; k < s.nkb; ++k) {
        const int l = s.kb_l[k];
        for (int m = 0; m < 2 * l + 1; ++m) {
          c.proj_atom.push_back(I);
          c.proj_lm.push_back(l * 4 + m);
          c.proj_r.push_back(s.kb_r[k]);
          c.hproj.push_back(s.kb_h[k]);
        }
      }
    }
    c.nproj = (int)c.proj_atom.size();
    // Ewald ranges: erfc(eta rcut) and exp(-gcut^2/4eta^2) below ~1e-17
    c.ew_eta = std::sqrt(kPiH) * std::pow(c.nat / (c.omega * c.omega), 1.0 / 6.0);
    c.ew_rcut = 6.2 / c.ew_eta;
    c.ew_gcut = 2.0 * c.ew_eta * 6.2;
    double diag = 0;
    for (int k = 0; k < 3; ++k) {
      const double s = c.A[k] + c.A[3 + k] + c.A[6 + k];
      diag += s * s;
    }
    double reach = c.ew_rcut + std::sqrt(diag);
    for (int i = 0; i < 3; ++i) {
      const double bn = std::sqrt(c.B[3 * i] * c.B[3 * i] + c.B[3 * i + 1] * c.B[3 * i + 1] +
                                  c.B[3 * i + 2] * c.B[3 * i + 2]);
      const double an = std::sqrt(c.A[3 * i] * c.A[3 * i] + c.A[3 * i + 1] * c.A[3 * i + 1] +
                                  c.A[3 * i + 2] * c.A[3 * i + 2]);
      c.ew_n[i] = (int)std::ceil(reach * bn / (2 * kPiH)) + 1;
      c.ew_m[i] = (int)std::ceil(c.ew_gcut * an / (2 * kPiH)) + 1;
    }
    c.ew_ng = (2 * c.ew_m[0] + 1) * (2 * c.ew_m[1] + 1) * (2 * c.ew_m[2] + 1);
    c.ew_nimg = (2 * c.ew_n[0] + 1) * (2 * c.ew_n[1] + 1) * (2 * c.ew_n[2] + 1);
  }

  size_t tsize() const { return prec_ == SGO_FP64 ? sizeof(double) : sizeof(float); }
  // Pulay history element: complex FP64, or complex FP32 in the FP32 bulk
  // forms (sums and coefficients stay FP64)
  size_t hist_bytes() const { return prec_ == SGO_FP64 ? 16 : 8; }

  // One device allocation per candidate, carved into 256-byte-aligned arrays.
  void alloc_cand(HostCand& c, const BatchGeom& g) {
    free_cand(c);
    const size_t ts = tsize();
    const size_t nb = c.nb, K = c.Kp, nt = c.ntot, nbm = std::max(c.nb, c.nproj);
    const size_t np16 = (size_t)(c.nproj + 15) / 16 * 16;
    const int ntile = (std::max(c.nb, c.nproj) + 63) / 64;
    c.red_doubles = std::max((size_t)kRedSlots, (size_t)2 * ntile * ntile * 32 * 4096);
    c.dens_chunks = g.dens_chunks;
    struct Item {
      void** p;
      size_t bytes;
    };
    CandDesc& d = c.d;
    std::memset(&d, 0, sizeof(d));
    std::vector<Item> items = {
        {&d.X, nb * K * ts}, {&d.HX, nb * K * ts}, {&d.D, nb * K * ts}, {&d.HD, nb * K * ts},
        {&d.sticks, (size_t)c.npair * c.N[2] * c.nst * 2 * ts}, {&d.veff_t, nt * ts},
        {&d.beta, (size_t)c.nproj * K * ts + 256},
        {&d.beta16, prec_ == SGO_FP32_BF16PROJ ? (size_t)2 * np16 * K * 2 + 256 : 0},
        {&d.betaT16, prec_ == SGO_FP32_BF16PROJ ? (size_t)2 * np16 * K * 2 + 256 : 0},
        {(void**)&d.kin, c.npwh * sizeof(double)}, {(void**)&d.gmeta, c.npwh * sizeof(int)},
        {(void**)&d.sp_off, (c.nsp + 1) * sizeof(int)}, {(void**)&d.stick_xy, c.nst * sizeof(int)},
        {(void**)&d.gmill, 3 * c.npwh * sizeof(int)},
        {(void**)&d.hproj, c.nproj * sizeof(double) + 8}, {(void**)&d.proj_atom, c.nproj * sizeof(int) + 8},
        {(void**)&d.proj_lm, c.nproj * sizeof(int) + 8}, {(void**)&d.proj_r, c.nproj * sizeof(double) + 8},
        {(void**)&d.S, nb * nb * 8}, {(void**)&d.Hs, nb * nb * 8}, {(void**)&d.M, nb * nb * 8},
        {(void**)&d.C, nbm * nb * 8}, {(void**)&d.eps, nb * 8}, {(void**)&d.occ, nb * 8},
        {(void**)&d.gam, nb * 8}, {(void**)&d.bandw, nb * 8}, {(void**)&d.resn, nb * 8},
        {(void**)&d.rho_in_r, nt * 8}, {(void**)&d.rho_out_r, nt * 8}, {(void**)&d.veff_r, nt * 8},
        {(void**)&d.zgrid, nt * 16}, {(void**)&d.vloc_G, nt * 16}, {(void**)&d.rho0_G, nt * 16},
        {(void**)&d.rho_out_G, nt * 16}, {(void**)&d.hist_in, kMaxHist * nt * hist_bytes()},
        {(void**)&d.hist_res, kMaxHist * nt * hist_bytes()}, {(void**)&d.pulay, kMaxHist * kMaxHist * 8},
        {(void**)&d.coef, kMaxHist * 8}, {(void**)&d.dens_part, (size_t)c.dens_chunks * nt * 8},
        {(void**)&d.pos, (size_t)3 * c.nat * 8}, {(void**)&d.spec, (size_t)c.nat * sizeof(int)},
        {(void**)&d.force, (size_t)3 * c.nat * 8}, {(void**)&d.force_ew, (size_t)3 * c.nat * 8},
        {(void**)&d.force_part, (size_t)6 * c.nat * 8}, {(void**)&d.nlwork, (size_t)c.nproj * nb * 4 * 8 + 8},
        {(void**)&d.stwork, stress_layout(c.nb, c.nproj, c.nat).total * 8},
        {(void**)&d.stress, (size_t)72 * 8},
        {(void**)&d.scal, S_COUNT * 8}, {(void**)&d.ewS, (size_t)c.ew_ng * 16},
        {(void**)&d.red_part, c.red_doubles * 8}, {(void**)&d.tickets, kTickets * sizeof(unsigned)},
    };
    size_t total = 0;
    for (auto& it : items) total += (it.bytes + 255) / 256 * 256;
    HIPCHK(hipSetDevice(device_));
    if (alloc_fn_) {
      c.mem = (char*)alloc_fn_(total, alloc_user_);
      if (!c.mem) throw Error(SGO_ENOMEM, "device allocation failed (caller allocator)");
    } else if (hipMalloc(&c.mem, total) != hipSuccess) {
      c.mem = nullptr;
      throw Error(SGO_ENOMEM, "device allocation failed");
    }
    c.mem_size = total;
    // stream-ordered (the legacy null stream would wait on every blocking
    // stream, and fail while another batch's thread captures a graph)
    HIPCHK(hipMemsetAsync(c.mem, 0, total, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    size_t off = 0;
    for (auto& it : items) {
      *it.p = c.mem + off;
      off += (it.bytes + 255) / 256 * 256;
    }
    upload_static(c);
    c.built = true;
  }

  void upload_static(HostCand& c) {
    CandDesc& d = c.d;
    d.N1 = c.N[0];
    d.N2 = c.N[1];
    d.N3 = c.N[2];
    d.ntot = c.ntot;
    d.npwh = c.npwh;
    d.K = c.K;
    d.Kp = c.Kp;
    d.nb = c.nb;
    d.npair = c.npair;
    d.nsp = c.nsp;
    d.nst = c.nst;
    d.nproj = c.nproj;
    d.nat = c.nat;
    d.np16 = (c.nproj + 15) / 16 * 16;
    d.pl_nx = c.pl_nx;
    d.pl_nxl = c.pl_nxl;
    d.pl_sx = c.pl_sx;
    d.occ_kind = c.occ_kind;
    d.nocc = c.nocc;
    d.active = 1;
    d.sigma = c.sigma;
    d.nelec = c.nelec;
    d.omega = c.omega;
    std::memcpy(d.A, c.A, sizeof(d.A));
    std::memcpy(d.B, c.B, sizeof(d.B));
    for (int k = 0; k < 3; ++k) d.plan[k] = c.plan[k];
    d.ndens_chunk = c.dens_chunks;
    d.hist_len = c.hist_len;
    d.hist_f32 = prec_ == SGO_FP64 ? 0 : 1;
    d.ew_eta = c.ew_eta;
    d.ew_rcut = c.ew_rcut;
    d.ew_gcut = c.ew_gcut;
    for (int k = 0; k < 3; ++k) {
      d.ew_m[k] = c.ew_m[k];
      d.ew_n[k] = c.ew_n[k];
    }
    d.ew_ng = c.ew_ng;
    d.ew_nimg = c.ew_nimg;
    auto up = [&](const void* dst, const void* src, size_t bytes) {
      if (bytes) {
        HIPCHK(hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
      }
    };
    up(d.kin, c.kin.data(), c.npwh * 8);
    up(d.gmeta, c.gmeta.data(), c.npwh * 4);
    up(d.sp_off, c.sp_off.data(), (c.nsp + 1) * 4);
    up(d.stick_xy, c.stick_xy.data(), c.nst * 4);
    up(d.gmill, c.gmill.data(), 3 * c.npwh * 4);
    up(d.hproj, c.hproj.data(), c.nproj * 8);
    up(d.proj_atom, c.proj_atom.data(), c.nproj * 4);
    up(d.proj_lm, c.proj_lm.data(), c.nproj * 4);
    up(d.proj_r, c.proj_r.data(), c.nproj * 8);
    up(d.spec, c.spec.data(), c.nat * 4);
    up(d.pos, c.pos.data(), 3 * c.nat * 8);
  }

  void free_cand(HostCand& c) {
    if (c.mem) {
      (void)hipSetDevice(device_);
      if (free_fn_) {
        (void)hipDeviceSynchronize();  // the caller's allocator may reuse it at once
        free_fn_(c.mem, alloc_user_);
      } else {
        (void)hipFree(c.mem);
      }
    }
    c.mem = nullptr;
    c.built = false;
  }

  BatchGeom geometry() const {
    BatchGeom g{};
    g.ncand = (int)cands_.size();
    for (auto& c : cands_) {
      g.npair_max = std::max(g.npair_max, c.npair);
      g.nsp_max = std::max(g.nsp_max, c.nsp);
      g.nb_max = std::max(g.nb_max, c.nb);
      g.nproj_max = std::max(g.nproj_max, c.nproj);
      g.nat_max = std::max(g.nat_max, c.nat);
      g.N1max = std::max(g.N1max, c.N[0]);
      g.N2max = std::max(g.N2max, c.N[1]);
      g.N3max = std::max(g.N3max, c.N[2]);
      g.ntot_max = std::max(g.ntot_max, c.ntot);
      g.plane_max = std::max(g.plane_max, c.N[0] * c.N[1]);
      g.K_max = std::max(g.K_max, c.K);
      g.ew_ng_max = std::max(g.ew_ng_max, c.ew_ng);
      g.pl_sx_max = std::max(g.pl_sx_max, c.pl_sx);
    }
    g.sp_chunk = std::max(1, tune("SGO_SP_CHUNK", std::max(1, 640 / std::max(1, g.N3max))));
    {  // the z kernels hold 2 x (2 sp_chunk) sticks of N3 complex values in LDS
      const size_t cplx_bytes = 2 * tsize();
      const int cap = (int)(((size_t)g_lds_limit / cplx_bytes - kMaxFftN) / (4 * (size_t)std::max(1, g.N3max)));
      g.sp_chunk = std::max(1, std::min(g.sp_chunk, cap));
    }
    g.kc_len = std::max(tune("SGO_GRAM_KC", 256), ((g.K_max + 31) / 32 + 31) / 32 * 32);
    g.kc_len = (g.kc_len + 31) / 32 * 32;
    g.sub_threads = std::max(64, std::min(512, tune("SGO_SUB_THREADS", 512) / 64 * 64));
    g.jac_grid = tune("SGO_JAC_GRID", kJacGridBandsDefault);
    g.nkc_max = (g.K_max + g.kc_len - 1) / g.kc_len;
    // FP32 register-FFT plane kernels when every line length is supported
    // and the compact plane (plus the density accumulator) fits the LDS
    g.plane_reg = tsize() == 4 && tune("SGO_PLANE_KERNEL", 1) == 1 ? 1 : 0;
    for (auto& c : cands_)
      if (!plane_reg_length_ok(c.N[0]) || !plane_reg_length_ok(c.N[1]) ||
          !plane_reg_length_ok(c.N[2]))
        g.plane_reg = 0;
    if (plane_reg_lds(g, true) > (size_t)g_lds_limit) g.plane_reg = 0;
    // consecutive z-planes per workgroup of the H psi plane kernel where
    // that fills the lanes better (tuning key SGO_PLANE_GROUP, 1 = off)
    g.plane_group = g.plane_reg ? plane_group_size(g, (size_t)g_lds_limit, tune("SGO_PLANE_GROUP", 0)) : 1;
    g.gemm_f32 = tune("SGO_GEMM_KERNEL", 1) == 1 ? 1 : 0;
    g.gemm_waves = tune("SGO_GEMM_WAVES", 8);
    g.gram_tile = tune("SGO_GRAM_TILE", 0);
    g.gram_f32 = tsize() == 4 && tune("SGO_GRAM_KERNEL", 1) == 2 ? 1 : 0;
    g.bf16proj = prec_ == SGO_FP32_BF16PROJ ? 1 : 0;
    g.lds_limit = (size_t)g_lds_limit;
    g.red_min_bytes = (size_t)-1;
    for (auto& c : cands_) {
      const int ntile = (std::max(c.nb, c.nproj) + 63) / 64;
      const size_t rd = std::max((size_t)kRedSlots, (size_t)2 * ntile * ntile * 32 * 4096);
      g.red_min_bytes = std::min(g.red_min_bytes, rd * 8);
    }
    // band-pair chunks of the density planes: enough blocks to fill the chip
    // (planes x candidates x chunks >= 512 blocks of 4 waves, or 4096
    // one-wave blocks for the register-FFT kernel), no more (each chunk is a
    // grid of partial sums)
    const int planes = std::max(1, g.N3max * g.ncand);
    const int want = g.plane_reg ? 4096 : 512;
    g.dens_chunks = std::max(1, std::min(g.npair_max, tune("SGO_DENS_CHUNKS", (want + planes - 1) / planes)));
    return g;
  }

  void check_lds(const BatchGeom& g) {
    const size_t ts = tsize();
    const size_t plane = 2 * ts * (2 * kMaxFftN + 2 * (size_t)g.plane_max);
    if (plane > (size_t)g_lds_limit)
      throw Error(SGO_EINVAL, "FFT plane N1*N2 too large for LDS at this precision");
    if (g.plane_max > 48 * kNT) throw Error(SGO_EINVAL, "FFT plane N1*N2 exceeds 12288");
    if (g.nb_max > 320) throw Error(SGO_EINVAL, "nbands exceeds 320");
    if (std::max(g.nb_max, g.nproj_max) > 600) throw Error(SGO_EINVAL, "too many projectors");
  }

  void upload_desc() {
    std::vector<CandDesc> h(cands_.size());
    int nact = 0;
    for (size_t i = 0; i < cands_.size(); ++i) {
      h[i] = cands_[i].d;
      h[i].ncand_index = (int)i;
      nact += h[i].active ? 1 : 0;
    }
    t_active = nact;
    if (!d_desc_ || desc_cap_ < cands_.size()) {
      if (d_desc_) (void)hipFree(d_desc_);
      HIPCHK(hipMalloc(&d_desc_, sizeof(CandDesc) * cands_.size()));
      desc_cap_ = cands_.size();
    }
    HIPCHK(hipMemcpyAsync(d_desc_, h.data(), sizeof(CandDesc) * h.size(), hipMemcpyHostToDevice,
                          stream_));
    HIPCHK(hipStreamSynchronize(stream_));
  }

  LaunchCtx ctx(const BatchGeom& g) {
    LaunchCtx L;
    L.stream = stream_;
    L.desc = d_desc_;
    L.species = d_species_;
    L.g = g;
    if (!d_jac_done_) {
      HIPCHK(hipMalloc(&d_jac_done_, sizeof(int) * capacity_));
      HIPCHK(hipHostMalloc((void**)&h_jac_done_, sizeof(int) * capacity_, hipHostMallocDefault));
    }
    L.jac_done = d_jac_done_;
    L.jac_done_host = h_jac_done_;
    return L;
  }

  // Launch context over the active candidates only (the population's tail:
  // converged candidates would otherwise still fill every launch grid).
  // The descriptors of the active candidates are uploaded contiguously; the
  // grid extents are the maxima over them, while every parameter that fixes
  // a buffer layout (K ranges, density chunks, stick chunks, plane groups,
  // thread counts) stays that of the whole batch.  act receives the indices.
  LaunchCtx ctx_active(const BatchGeom& full, std::vector<int>& act) {
    act.clear();
    std::vector<CandDesc> h;
    for (size_t i = 0; i < cands_.size(); ++i)
      if (cands_[i].d.active) {
        act.push_back((int)i);
        h.push_back(cands_[i].d);
        h.back().ncand_index = (int)i;
      }
    if (h.empty()) return ctx(full);
    if (!d_desc_act_ || desc_act_cap_ < h.size()) {
      if (d_desc_act_) (void)hipFree(d_desc_act_);
      HIPCHK(hipMalloc(&d_desc_act_, sizeof(CandDesc) * cands_.size()));
      desc_act_cap_ = cands_.size();
    }
    HIPCHK(hipMemcpyAsync(d_desc_act_, h.data(), sizeof(CandDesc) * h.size(), hipMemcpyHostToDevice,
                          stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    BatchGeom g = full;
    g.ncand = (int)h.size();
    g.npair_max = g.nsp_max = g.nb_max = g.nproj_max = g.nat_max = 0;
    g.N1max = g.N2max = g.N3max = g.ntot_max = g.plane_max = g.K_max = g.pl_sx_max = 0;
    for (int i : act) {
      const HostCand& c = cands_[i];
      g.npair_max = std::max(g.npair_max, c.npair);
      g.nsp_max = std::max(g.nsp_max, c.nsp);
      g.nb_max = std::max(g.nb_max, c.nb);
      g.nproj_max = std::max(g.nproj_max, c.nproj);
      g.nat_max = std::max(g.nat_max, c.nat);
      g.N1max = std::max(g.N1max, c.N[0]);
      g.N2max = std::max(g.N2max, c.N[1]);
      g.N3max = std::max(g.N3max, c.N[2]);
      g.ntot_max = std::max(g.ntot_max, c.ntot);
      g.plane_max = std::max(g.plane_max, c.N[0] * c.N[1]);
      g.K_max = std::max(g.K_max, c.K);
      g.pl_sx_max = std::max(g.pl_sx_max, c.pl_sx);
    }
    g.nkc_max = (g.K_max + g.kc_len - 1) / g.kc_len;
    LaunchCtx L = ctx(g);
    L.desc = d_desc_act_;
    return L;
  }

  // Build every candidate that needs it and run the per-geometry setup.
  BatchGeom prepare(unsigned seed, int hist) {
    if (cands_.empty()) throw Error(SGO_ESTATE, "no structure set");
    HIPCHK(hipSetDevice(device_));
    BatchGeom g = geometry();
    check_lds(g);
    for (auto& c : cands_) {
      c.hist_len = hist;
      if (!c.built || c.dens_chunks != g.dens_chunks) {
        alloc_cand(c, g);
        c.have_psi = false;
      } else {
        c.d.hist_len = hist;
        c.d.ndens_chunk = c.dens_chunks;
        HIPCHK(hipMemcpyAsync((void*)c.d.pos, c.pos.data(), 3 * c.nat * 8, hipMemcpyHostToDevice,
                              stream_));
        HIPCHK(hipStreamSynchronize(stream_));
      }
      c.d.seed = seed;
      c.d.active = 1;
      c.d.iter_state = d_iter_;
      c.status = SGO_OK;
      c.info = sgo_scf_info{};
      HIPCHK(hipMemsetAsync(c.d.scal, 0, S_COUNT * 8, stream_));
    }
    upload_desc();
    return g;
  }

  template <typename T>
  void setup_geometry(const LaunchCtx& L) {
    launch_setup_grid(L);
    launch_setup_beta<T>(L);
    launch_ewald(L);
  }

  // Orthonormalise (Cholesky) and rotate to the Ritz vectors of the band
  // subspace.  Intermediate calls within an SCF iteration may stop after
  // `sweeps` Jacobi sweeps; the last one converges fully.
  template <typename T>
  void subspace_rotate(const LaunchCtx& L, bool with_d, int sweeps) {
    int a[2] = {W_X, W_X}, b[2] = {W_X, W_HX}, o[2] = {M_S, M_H};
    launch_gram<T>(L, 2, a, b, o);
    launch_subspace(L, 3, sweeps);
    int y[3] = {W_X, W_HX, W_D};
    launch_gemm_acc<T>(L, with_d ? 3 : 2, y, y, M_M, 0.0, 1.0, 0);
  }

  // All-band CG of Algorithm 1: at most ncg steps; with cg_tol > 0 a
  // candidate stops once its residuals meet the gate (k_cg_gate) and then
  // gets the full subspace diagonalisation the last step would have given.
  template <typename T>
  void eigensolver(const LaunchCtx& L, int ncg, double cg_tol) {
    const int inter = tune("SGO_RR_SWEEPS", 1);
    launch_hpsi<T>(L, W_X);
    subspace_rotate<T>(L, false, inter);
    for (int k = 0; k < ncg; ++k) {
      launch_cg_direction<T>(L, k == 0 ? 1 : 0);
      if (cg_tol > 0.0) launch_cg_gate(L, cg_tol);
      int a[1] = {W_X}, b[1] = {W_D}, o[1] = {M_C};
      launch_gram<T>(L, 1, a, b, o);
      int y[1] = {W_D}, aa[1] = {W_X};
      launch_gemm_acc<T>(L, 1, y, aa, M_C, 1.0, -1.0, 0);
      launch_hpsi<T>(L, W_D);
      launch_linemin<T>(L);
      subspace_rotate<T>(L, true, k + 1 == ncg ? 40 : inter);
    }
    if (cg_tol > 0.0) {
      launch_cg_release(L, 0);
      subspace_rotate<T>(L, false, 40);
      launch_cg_release(L, 1);
    }
  }

  template <typename T>
  void init_wavefunctions(const LaunchCtx& L) {
    launch_init_random<T>(L);
    int a[1] = {W_X}, b[1] = {W_X}, o[1] = {M_S};
    launch_gram<T>(L, 1, a, b, o);
    launch_subspace(L, 1);
    int y[1] = {W_X};
    launch_gemm_acc<T>(L, 1, y, y, M_M, 0.0, 1.0, 0);
  }

  // Status scalars of every candidate: one gather kernel and one copy into
  // pinned host memory.
  void read_scal(std::vector<std::array<double, S_COUNT>>& out) {
    const size_t n = cands_.size();
    out.resize(n);
    if (scal_cap_ < n) {
      if (d_scal_all_) (void)hipFree(d_scal_all_);
      if (h_scal_all_) (void)hipHostFree(h_scal_all_);
      d_scal_all_ = nullptr;
      h_scal_all_ = nullptr;
      scal_cap_ = 0;
      HIPCHK(hipMalloc(&d_scal_all_, n * S_COUNT * 8));
      HIPCHK(hipHostMalloc((void**)&h_scal_all_, n * S_COUNT * 8, hipHostMallocDefault));
      scal_cap_ = n;
    }
    LaunchCtx L = ctx(BatchGeom{});
    L.g.ncand = (int)n;
    launch_gather_scal(L, d_scal_all_);
    HIPCHK(hipMemcpyAsync(h_scal_all_, d_scal_all_, n * S_COUNT * 8, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    for (size_t i = 0; i < n; ++i) std::memcpy(out[i].data(), h_scal_all_ + i * S_COUNT, S_COUNT * 8);
  }

  // One SCF iteration after the first: mix the previous output into the new
  // input potential, solve (Algorithm 1), occupations, output density,
  // residual and Pulay row, energies and convergence flags, advance the
  // device-side iteration counter.  Captured once into a HIP graph when
  // opts.use_graph is set (K iterations per graph for use_graph = K).
  template <typename T>
  void iteration_body(const LaunchCtx& L, const sgo_scf_opts& o) {
    launch_mix(L, 0, o.mix_alpha, o.kerker_q0);
    launch_grid_fft(L, +1);
    launch_potential_finalize<T>(L);
    iteration_solve<T>(L, o, o.ncg);
  }
  template <typename T>
  void iteration_solve(const LaunchCtx& L, const sgo_scf_opts& o, int ncg) {
    eigensolver<T>(L, ncg, o.cg_tol);
    launch_occupations(L);
    launch_band_kinetic<T>(L);
    launch_density<T>(L);
    launch_density_finalize(L);
    launch_grid_fft(L, -1);
    launch_gspace_residual(L);
    launch_scf_control(L, o.tol_e, o.tol_rho, o.cg_tol);
    launch_iter_set(L, d_iter_, 1, 1);
    launch_mask_done(L);
  }

  // Read the status block of every active candidate; mask out the converged
  // and failed ones.  Returns the number still active.
  int update_active(int it) {
    (void)it;  // per-candidate counts come from the device (S_ITER)
    std::vector<std::array<double, S_COUNT>> sc;
    read_scal(sc);
    bool changed = false;
    int nactive = 0;
    for (size_t i = 0; i < cands_.size(); ++i) {
      HostCand& c = cands_[i];
      if (!c.d.active) continue;
      c.info.iterations = (int)sc[i][S_ITER];
      c.info.de = sc[i][S_DE];
      c.info.drho = sc[i][S_DRHO];
      if (sc[i][S_ERR] != 0.0) {
        c.status = SGO_ENUMERIC;
        c.d.active = 0;
        changed = true;
      } else if (sc[i][S_CONV] != 0.0) {
        c.info.converged = 1;
        c.d.active = 0;
        changed = true;
      }
      nactive += c.d.active;
    }
    if (changed) upload_desc();
    return nactive;
  }

  template <typename T>
  int scf_t(const sgo_scf_opts& o) {
    const int hist = std::max(2, std::min(kMaxHist, o.history));
    BatchGeom g = prepare(o.seed, hist);
    hipStream_t user_stream = stream_;
    // a stream of its own when none is set and something will be captured:
    // the K-iteration graphs, or the Jacobi sweeps over the GPU
    if ((o.use_graph || g.nb_max >= g.jac_grid) && !stream_) {
      if (!own_stream_) HIPCHK(hipStreamCreateWithFlags(&own_stream_, hipStreamNonBlocking));
      stream_ = own_stream_;
    }
    struct Restore {
      Engine* e;
      hipStream_t s;
      ~Restore() { e->stream_ = s; }
    } restore{this, user_stream};
    LaunchCtx L = ctx(g);
    bool all_warm = true;
    for (auto& c : cands_) all_warm = all_warm && c.have_psi;
    launch_iter_set(L, d_iter_, 0, 0);
    setup_geometry<T>(L);
    if (!all_warm) init_wavefunctions<T>(L);
    launch_mix(L, 1, o.mix_alpha, o.kerker_q0);
    launch_grid_fft(L, +1);
    launch_potential_finalize<T>(L);
    iteration_solve<T>(L, o, all_warm ? o.ncg : o.ncg_first);
    HIPCHK(hipGetLastError());
    int it = 0;
    int nactive = update_active(it);
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    // the iterations launch over the active candidates only once some have
    // converged (tuning key SGO_COMPACT, 0 = off)
    const bool compact = tune("SGO_COMPACT", 1) != 0;
    LaunchCtx Li = L;
    std::vector<int> act_now, act_prev;
    // use_graph = K >= 1: K iterations per captured graph (candidates that
    // converge inside it mask themselves on the device, k_mask_done), the
    // status read once per K; iterations left over before max_iter run eagerly
    const int K = std::max(1, o.use_graph);
    for (it = 1; it < o.max_iter && nactive > 0;) {
      const int k = (o.use_graph && it + K <= o.max_iter) ? K : 1;
      if (compact && nactive < (int)cands_.size()) {
        act_now.clear();
        for (size_t i = 0; i < cands_.size(); ++i)
          if (cands_[i].d.active) act_now.push_back((int)i);
        if (act_now != act_prev) {
          Li = ctx_active(g, act_prev);
          if (exec) {
            (void)hipGraphExecDestroy(exec);
            exec = nullptr;
          }
          if (graph) {
            (void)hipGraphDestroy(graph);
            graph = nullptr;
          }
        }
      }
      if (o.use_graph && k == K) {
        if (!exec) {
          g_capturing = true;
          HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
          try {
            for (int r = 0; r < K; ++r) iteration_body<T>(Li, o);
          } catch (...) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(stream_, &dummy);
            g_capturing = false;
            throw;
          }
          HIPCHK(hipStreamEndCapture(stream_, &graph));
          g_capturing = false;
          HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(exec, stream_));
      } else {
        iteration_body<T>(Li, o);
      }
      HIPCHK(hipGetLastError());
      it += k;
      nactive = update_active(it - 1);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto& c : cands_) {
      if (c.d.active) c.status = SGO_ENOTCONV;
      c.d.active = 1;
      c.have_psi = true;
      c.have_scf = true;
    }
    upload_desc();
    // forces of every candidate from its final state
    launch_force_local(L);
    launch_force_nonlocal<T>(L);
    launch_force_finalize(L);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    int worst = SGO_OK;
    for (auto& c : cands_)
      if (c.status < worst) worst = c.status;
    return worst;
  }

  // Fixed-basis stress of every candidate that holds a converged state
  // (others are masked), into each candidate's d.stress.
  template <typename T>
  void stress_t() {
    BatchGeom g = geometry();
    for (auto& c : cands_) c.d.active = c.have_scf ? 1 : 0;
    upload_desc();
    LaunchCtx L = ctx(g);
    launch_stress_waves<T>(L);
    launch_stress_grid(L);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    for (auto& c : cands_) c.d.active = 1;
    upload_desc();
  }
  void stress() {
    HIPCHK(hipSetDevice(device_));
    if (prec_ == SGO_FP64) stress_t<double>();
    else stress_t<float>();
  }

  // ---- k-point sampling of one structure (FP64): the "rough K-points"
  // of Section 2.3.  Each k has its shifted sphere |k+G|^2/2 <= Ecut of
  // complex coefficients; the grid side (density, potentials, mixing,
  // energies, local and Ewald forces) is the structure's Gamma setup.
  struct KPt {
    double kf[3] = {0, 0, 0};
    double w = 0;
    int npw = 0;
    char* mem = nullptr;
    KptBands kb{};
    cplx<double>*X = nullptr, *HX = nullptr, *D = nullptr, *HD = nullptr;
  };
  std::vector<KPt> kpts_;
  char* kshared_ = nullptr;
  cplx<double>*kz_ = nullptr, *kS_ = nullptr, *kH_ = nullptr, *kW_ = nullptr, *kV_ = nullptr,
              *kM_ = nullptr, *kC_ = nullptr, *kP_ = nullptr, *kdP_ = nullptr, *ktmp_ = nullptr;
  double *keps_ = nullptr, *kocc_ = nullptr, *kgam_ = nullptr, *kbandw_ = nullptr, *kw_ = nullptr,
         *kfnl_ = nullptr;
  int* kfail_ = nullptr;
  int k_nb_ = 0;
  bool k_solved_ = false;

  bool kmode() const { return !kpts_.empty(); }
  int nkpts() const { return (int)kpts_.size(); }

  void k_free() {
    for (auto& k : kpts_)
      if (k.mem) {
        (void)hipFree(k.mem);
        k.mem = nullptr;
      }
    if (kshared_) (void)hipFree(kshared_);
    kshared_ = nullptr;
    k_nb_ = 0;
  }

  void set_kpoints(int nk, const double* kf, const double* w) {
    if (nk < 0 || (nk > 0 && (!kf || !w))) throw Error(SGO_EINVAL, "bad k-point arguments");
    if (nk > 0 && prec_ != SGO_FP64) throw Error(SGO_EINVAL, "k-point sampling needs an SGO_FP64 handle");
    double tot = 0.0;
    for (int i = 0; i < nk; ++i) {
      if (!(w[i] > 0.0)) throw Error(SGO_EINVAL, "k-point weights must be positive");
      for (int a = 0; a < 3; ++a)
        if (!std::isfinite(kf[3 * i + a])) throw Error(SGO_EINVAL, "k-point coordinates must be finite");
      tot += w[i];
    }
    HIPCHK(hipSetDevice(device_));
    HIPCHK(hipDeviceSynchronize());
    k_free();
    kpts_.clear();
    k_solved_ = false;
    for (int i = 0; i < nk; ++i) {
      KPt k;
      for (int a = 0; a < 3; ++a) k.kf[a] = kf[3 * i + a];
      k.w = w[i] / tot;
      kpts_.push_back(k);
    }
  }

  // Host basis of every k (shifted sphere, grid indices, |k+G|^2/2, k+G)
  // and the device arrays: per k the basis, projectors and bands; shared
  // FFT grids, subspace matrices and per-(k, band) scalars.
  void k_build(HostCand& c) {
    k_free();
    const int nb = c.nb, nproj = c.nproj, nk = nkpts();
    const double gmax = std::sqrt(2.0 * c.ecut);
    int npw_max = 0;
    std::vector<std::vector<int>> boxes(nk);
    std::vector<std::vector<double>> kins(nk), qs(nk);
    for (int ik = 0; ik < nk; ++ik) {
      KPt& k = kpts_[ik];
      int mmax[3];
      for (int i = 0; i < 3; ++i) {
        const double an = std::sqrt(c.A[3 * i] * c.A[3 * i] + c.A[3 * i + 1] * c.A[3 * i + 1] +
                                    c.A[3 * i + 2] * c.A[3 * i + 2]);
        mmax[i] = (int)std::floor(gmax * an / (2.0 * M_PI) + std::fabs(k.kf[i])) + 1;
      }
      for (int m1 = -mmax[0]; m1 <= mmax[0]; ++m1)
        for (int m2 = -mmax[1]; m2 <= mmax[1]; ++m2)
          for (int m3 = -mmax[2]; m3 <= mmax[2]; ++m3) {
            const double f[3] = {m1 + k.kf[0], m2 + k.kf[1], m3 + k.kf[2]};
            double q[3];
            for (int a = 0; a < 3; ++a) q[a] = f[0] * c.B[a] + f[1] * c.B[3 + a] + f[2] * c.B[6 + a];
            const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            if (0.5 * q2 > c.ecut) continue;
            const int m[3] = {m1, m2, m3};
            for (int a = 0; a < 3; ++a)
              if (2 * std::abs(m[a]) + 1 > c.N[a])
                throw Error(SGO_EINVAL, "FFT grid too small for the wavefunction sphere at a k-point");
            const int x = ((m1 % c.N[0]) + c.N[0]) % c.N[0], y = ((m2 % c.N[1]) + c.N[1]) % c.N[1],
                      z = ((m3 % c.N[2]) + c.N[2]) % c.N[2];
            boxes[ik].push_back((z * c.N[1] + y) * c.N[0] + x);
            kins[ik].push_back(0.5 * q2);
            for (int a = 0; a < 3; ++a) qs[ik].push_back(q[a]);
          }
      k.npw = (int)boxes[ik].size();
      if (k.npw < nb) throw Error(SGO_EINVAL, "fewer plane waves than bands at a k-point");
      npw_max = std::max(npw_max, k.npw);
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t zc = sizeof(cplx<double>);
    for (int ik = 0; ik < nk; ++ik) {
      KPt& k = kpts_[ik];
      const size_t n = k.npw;
      const size_t bytes = al(n * 4) + al(n * 8) + al(n * 24) + al((size_t)nproj * n * zc) + 4 * al((size_t)nb * n * zc);
      HIPCHK(hipMalloc(&k.mem, bytes));
      char* p = k.mem;
      int* box = (int*)p;
      p += al(n * 4);
      double* kin = (double*)p;
      p += al(n * 8);
      double* q = (double*)p;
      p += al(n * 24);
      k.kb.beta = (cplx<double>*)p;
      p += al((size_t)nproj * n * zc);
      k.X = (cplx<double>*)p;
      p += al((size_t)nb * n * zc);
      k.HX = (cplx<double>*)p;
      p += al((size_t)nb * n * zc);
      k.D = (cplx<double>*)p;
      p += al((size_t)nb * n * zc);
      k.HD = (cplx<double>*)p;
      HIPCHK(hipMemcpy(box, boxes[ik].data(), n * 4, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(kin, kins[ik].data(), n * 8, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(q, qs[ik].data(), n * 24, hipMemcpyHostToDevice));
      k.kb.npw = k.npw;
      k.kb.nb = nb;
      k.kb.nproj = nproj;
      k.kb.box = box;
      k.kb.kin = kin;
      k.kb.q = q;
    }
    const size_t nbb = (size_t)nb * nb, nkb = (size_t)nk * nb;
    const size_t pw = std::max<size_t>(nproj, 1) * nb;
    const size_t bytes = al((size_t)nb * c.ntot * zc) + 6 * al(nbb * zc) + al(pw * zc) + al(3 * pw * zc) +
                         al((size_t)nb * npw_max * zc) + 4 * al(nkb * 8) + al((size_t)nk * 8) +
                         al((size_t)3 * c.nat * 8) + al(8);
    HIPCHK(hipMalloc(&kshared_, bytes));
    char* p = kshared_;
    auto take = [&](size_t b) {
      char* r = p;
      p += al(b);
      return r;
    };
    kz_ = (cplx<double>*)take((size_t)nb * c.ntot * zc);
    kS_ = (cplx<double>*)take(nbb * zc);
    kH_ = (cplx<double>*)take(nbb * zc);
    kW_ = (cplx<double>*)take(nbb * zc);
    kV_ = (cplx<double>*)take(nbb * zc);
    kM_ = (cplx<double>*)take(nbb * zc);
    kC_ = (cplx<double>*)take(nbb * zc);
    kP_ = (cplx<double>*)take(pw * zc);
    kdP_ = (cplx<double>*)take(3 * pw * zc);
    ktmp_ = (cplx<double>*)take((size_t)nb * npw_max * zc);
    keps_ = (double*)take(nkb * 8);
    kocc_ = (double*)take(nkb * 8);
    kgam_ = (double*)take(nkb * 8);
    kbandw_ = (double*)take(nkb * 8);
    kw_ = (double*)take((size_t)nk * 8);
    kfnl_ = (double*)take((size_t)3 * c.nat * 8);
    kfail_ = (int*)take(8);
    std::vector<double> w(nk);
    for (int ik = 0; ik < nk; ++ik) w[ik] = kpts_[ik].w;
    HIPCHK(hipMemcpy(kw_, w.data(), nk * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(kfail_, 0, 8));
    k_nb_ = nb;
  }

  // Rayleigh-Ritz of one k: S = X^H X, H = X^H HX, Cholesky and complex
  // Jacobi (k_kpt_subspace), then X, HX (and D) <- . M
  void k_rr(const HostCand& c, KPt& k, double* eps, bool with_d) {
    const int nb = c.nb, npw = k.npw;
    kpt_zdot(stream_, k.X, nb, k.X, nb, npw, kS_, nb, nullptr, 0);
    kpt_zdot(stream_, k.X, nb, k.HX, nb, npw, kH_, nb, nullptr, 0);
    kpt_subspace(stream_, kS_, kH_, kW_, kV_, kM_, eps, nb, 3, kfail_);
    cplx<double>* arr[3] = {k.X, k.HX, k.D};
    for (int a = 0; a < (with_d ? 3 : 2); ++a) {
      kpt_zgemm(stream_, arr[a], nb, kM_, nb, ktmp_, nb, npw, 1.0, 0.0, nullptr);
      kpt_copy(stream_, arr[a], ktmp_, (long)nb * npw);
    }
  }

  // Algorithm 1 at one k: H psi, subspace diagonalisation, then ncg steps
  // of residual, preconditioning, projection, line minimisation and
  // Rayleigh-Ritz.
  void k_eigensolve(const HostCand& c, int ik, int ncg) {
    KPt& k = kpts_[ik];
    double* eps = keps_ + (size_t)ik * c.nb;
    double* gam = kgam_ + (size_t)ik * c.nb;
    kpt_hpsi(stream_, k.kb, k.X, k.HX, kz_, c.d.veff_r, c.N, c.plan, kP_, c.d.hproj);
    k_rr(c, k, eps, false);
    for (int st = 0; st < ncg; ++st) {
      kpt_cg_dir(stream_, k.kb, k.X, k.HX, k.D, eps, gam, st == 0 ? 1 : 0);
      kpt_zdot(stream_, k.X, c.nb, k.D, c.nb, k.npw, kC_, c.nb, nullptr, 0);
      kpt_zgemm(stream_, k.X, c.nb, kC_, c.nb, k.D, c.nb, k.npw, -1.0, 1.0, nullptr);
      kpt_hpsi(stream_, k.kb, k.D, k.HD, kz_, c.d.veff_r, c.N, c.plan, kP_, c.d.hproj);
      kpt_linemin(stream_, k.kb, k.X, k.HX, k.D, k.HD);
      k_rr(c, k, eps, true);
    }
  }

  // One SCF iteration at the k-points: bands of every k, occupations with
  // one chemical potential, the k-weighted density into the structure's
  // density chunk, then the Gamma path's density, residual and control.
  void k_iteration(const LaunchCtx& L, HostCand& c, const sgo_scf_opts& o, int ncg) {
    const int nk = nkpts(), nb = c.nb;
    for (int ik = 0; ik < nk; ++ik) k_eigensolve(c, ik, ncg);
    kpt_occupations(stream_, keps_, kw_, nk, nb, c.nelec, c.occ_kind, c.sigma, kocc_, c.d.scal);
    for (int ik = 0; ik < nk; ++ik) kpt_band_kinetic(stream_, kpts_[ik].kb, kpts_[ik].X, kbandw_ + (size_t)ik * nb);
    kpt_kinetic_total(stream_, kbandw_, kocc_, kw_, nk, nb, c.d.occ, c.d.bandw, c.nb);
    for (int ik = 0; ik < nk; ++ik) {
      KPt& k = kpts_[ik];
      kpt_zero(stream_, kz_, (long)nb * c.ntot);
      k_density_grid(c, k);
      kpt_density(stream_, kz_, kocc_ + (size_t)ik * nb, k.w, nb, c.ntot, c.d.dens_part, ik == 0 ? 1 : 0);
    }
    launch_density_finalize(L);
    launch_grid_fft(L, -1);
    launch_gspace_residual(L);
    launch_scf_control(L, o.tol_e, o.tol_rho, 0.0);
    launch_iter_set(L, d_iter_, 1, 1);
  }

  // u_n(r) of every band of k on the grid (kz_)
  void k_density_grid(const HostCand& c, KPt& k) {
    kpt_scatter_bands(stream_, kz_, k.X, k.kb, c.ntot);
    kpt_fft3(stream_, kz_, c.nb, c.N, c.plan, +1);
  }

  int scf_k(const sgo_scf_opts& o) {
    if (cands_.size() != 1) throw Error(SGO_EINVAL, "k-point sampling is for a single structure");
    const int hist = std::max(2, std::min(kMaxHist, o.history));
    BatchGeom g = prepare(o.seed, hist);
    HostCand& c = cands_[0];
    LaunchCtx L = ctx(g);
    launch_iter_set(L, d_iter_, 0, 0);
    setup_geometry<double>(L);
    k_build(c);
    for (auto& k : kpts_) kpt_beta(stream_, k.kb, c.d.proj_atom, c.d.proj_lm, c.d.proj_r, c.d.pos, c.omega);
    // the k density goes into the structure's first density chunk
    c.d.ndens_chunk = 1;
    upload_desc();
    struct RestoreChunks {
      HostCand& c;
      ~RestoreChunks() { c.d.ndens_chunk = c.dens_chunks; }
    } restore{c};
    for (int ik = 0; ik < nkpts(); ++ik) {
      KPt& k = kpts_[ik];
      kpt_init(stream_, k.kb, k.X, o.seed, ik);
    }
    launch_mix(L, 1, o.mix_alpha, o.kerker_q0);
    launch_grid_fft(L, +1);
    launch_potential_finalize<double>(L);
    k_iteration(L, c, o, o.ncg_first);
    HIPCHK(hipGetLastError());
    int it = 0;
    int nactive = update_active(it);
    for (it = 1; it < o.max_iter && nactive > 0; ++it) {
      launch_mix(L, 0, o.mix_alpha, o.kerker_q0);
      launch_grid_fft(L, +1);
      launch_potential_finalize<double>(L);
      k_iteration(L, c, o, o.ncg);
      HIPCHK(hipGetLastError());
      nactive = update_active(it);
    }
    int fail = 0;
    HIPCHK(hipMemcpy(&fail, kfail_, sizeof(int), hipMemcpyDeviceToHost));
    if (c.d.active) c.status = SGO_ENOTCONV;
    if (fail) c.status = SGO_ENUMERIC;
    c.d.active = 1;
    upload_desc();
    // forces: local (from rho) + nonlocal at every k + Ewald
    launch_force_local(L);
    for (int ik = 0; ik < nkpts(); ++ik) {
      KPt& k = kpts_[ik];
      if (c.nproj > 0) {
        kpt_zdot(stream_, k.kb.beta, c.nproj, k.X, c.nb, k.npw, kP_, c.nb, nullptr, 0);
        for (int a = 0; a < 3; ++a)
          kpt_zdot(stream_, k.kb.beta, c.nproj, k.X, c.nb, k.npw, kdP_ + (size_t)a * c.nproj * c.nb, c.nb,
                   k.kb.q, a);
      }
      kpt_force_nl(stream_, kP_, kdP_, c.nproj, c.nb, c.d.hproj, c.d.proj_atom, kocc_ + (size_t)ik * c.nb,
                   k.w, c.nat, kfnl_, ik == 0 ? 1 : 0);
    }
    kpt_force_total(stream_, c.d.force_part, kfnl_, c.d.force_ew, c.nat, c.d.force,
                    c.d.force_part + 3 * c.nat);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    c.have_psi = false;  // the Gamma bands were not solved
    c.have_scf = true;
    k_solved_ = true;
    return c.status;
  }

  void kpoint_eigenvalues(double* eig, double* occ) {
    if (!k_solved_) throw Error(SGO_ESTATE, "no k-point solve");
    HIPCHK(hipSetDevice(device_));
    const size_t n = (size_t)nkpts() * k_nb_;
    HIPCHK(hipMemcpy(eig, keps_, n * 8, hipMemcpyDeviceToHost));
    if (occ) HIPCHK(hipMemcpy(occ, kocc_, n * 8, hipMemcpyDeviceToHost));
  }

  int scf(const sgo_scf_opts& o) {
    HIPCHK(hipSetDevice(device_));
    if (kmode()) return scf_k(o);
    return prec_ == SGO_FP64 ? scf_t<double>(o) : scf_t<float>(o);
  }

  // Conventional CG relaxation of every candidate (Section 2.3 lists it
  // among the relaxation options): Polak-Ribiere directions and a secant
  // line search on F.d, two batched evaluations per step, warm-started.
  //   trial step  alpha1 = 0.1 bohr / max_i |d_i| (capped by the previous step x 2)
  //   secant      alpha2 = alpha1 s0 / (s0 - s1), s = -F.d, clamped to [0.1, 4] alpha1
  //   direction   d <- F_new + max(0, F_new.(F_new - F) / F.F) d
  // energies [n][nsteps+1] records the energy after each accepted step.
  int relax_cg(int nsteps, const sgo_scf_opts& o, double* energies) {
    return relax(nsteps, o, energies, -1, nullptr);
  }

  // PCG (Section 2.3): the same secant line search along d = P F + beta d,
  // beta = max(0, F_new.P(F_new - F) / F.P F), trial step min(1, 0.1 bohr /
  // max_atom |d|) capped by twice the previous step; P is the inverse Hessian
  // of a Morse force field fitted to every (positions, forces) sample of the
  // candidate's relaxation, rebuilt every `refit` steps (0: only at the
  // start).  params (nullable) [n][3] receives the last fit.
  int relax_pcg(int nsteps, const sgo_scf_opts& o, double* energies, int refit, double* params) {
    return relax(nsteps, o, energies, refit, params);
  }

  // CLS (Section 2.3, re-derived): before every step the Morse field is
  // refitted to all samples; its steepest-descent path from the current
  // structure (steps moving the most-forced atom by h = 0.02 bohr, until
  // max|F_FF| < 1e-3 or 200 steps) is the guided curve x(s), s = path
  // parameter in bohr of largest displacement; the DFT energy is minimised
  // along it with the secant step on g(s) = -F(x(s)).x'(s): trial
  // s1 = min(s_end, 0.3, 2 s_prev), s2 clamped to [0.1, 4] s1 and s_end.
  int relax_cls(int nsteps, const sgo_scf_opts& o, double* energies, double* params) {
    const int n = (int)cands_.size();
    const double h = 0.02, ftol = 1e-3, s_cap = 0.3;
    const int kmax = 200;
    std::vector<std::vector<double>> x(n), F(n), x1(n), F1(n), nodes(n), samp_x(n), samp_f(n);
    std::vector<std::array<double, 3>> prm(n);
    std::vector<double> E(n), s_prev(n, 0.0), s1(n), s_end(n), g0(n);
    std::vector<int> status(n, SGO_OK);
    auto evaluate = [&](std::vector<std::vector<double>>& pos, std::vector<std::vector<double>>& force,
                        std::vector<double>* en) {
      for (int i = 0; i < n; ++i) move_atoms(i, pos[i].data());
      (void)scf(o);
      for (int i = 0; i < n; ++i) {
        HostCand& c = cands_[i];
        force[i].resize(3 * c.nat);
        get(c.d.force, force[i].data(), 3 * c.nat * sizeof(double));
        if (en) {
          double sc[S_COUNT];
          get_scal(c, sc);
          (*en)[i] = sc[S_ETOT];
        }
        if (c.status < status[i]) status[i] = c.status;
      }
    };
    // x(s) on candidate i's polyline and the tangent of the segment holding s
    auto point = [&](int i, double s, std::vector<double>& out, std::vector<double>* tang) {
      const size_t m = x[i].size();
      const int K = (int)(nodes[i].size() / m) - 1;
      int k = (int)std::floor(s / h);
      k = std::max(0, std::min(k, K - 1));
      const double t = s / h - k;
      const double* a = nodes[i].data() + (size_t)k * m;
      const double* b = a + m;
      out.resize(m);
      for (size_t c = 0; c < m; ++c) out[c] = a[c] + t * (b[c] - a[c]);
      if (tang) {
        tang->resize(m);
        for (size_t c = 0; c < m; ++c) (*tang)[c] = (b[c] - a[c]) / h;
      }
    };
    auto build_curves = [&]() {
      const int nt = std::max(1, std::min({n, (int)std::thread::hardware_concurrency(), 16}));
      std::vector<std::thread> pool;
      std::vector<std::exception_ptr> err(nt);
      for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
          try {
            for (int i = t; i < n; i += nt) {
              const HostCand& c = cands_[i];
              const int m = 3 * c.nat;
              ff::fit(c.A, c.nat, (int)(samp_x[i].size() / m), samp_x[i].data(),
                      samp_f[i].data(), prm[i].data());
              ff::guided_curve(c.A, c.nat, prm[i].data(), x[i].data(), h, ftol, kmax, nodes[i]);
              if ((int)nodes[i].size() == m) {  // field at rest: one step along the DFT forces
                double fm = 0.0;
                for (int I = 0; I < c.nat; ++I)
                  fm = std::max(fm, std::sqrt(F[i][3 * I] * F[i][3 * I] + F[i][3 * I + 1] * F[i][3 * I + 1] +
                                              F[i][3 * I + 2] * F[i][3 * I + 2]));
                for (int q = 0; q < m; ++q) nodes[i].push_back(x[i][q] + (fm > 0 ? h * F[i][q] / fm : 0.0));
              }
            }
          } catch (...) {
            err[t] = std::current_exception();
          }
        });
      for (auto& th : pool) th.join();
      for (auto& e : err)
        if (e) std::rethrow_exception(e);
    };
    for (int i = 0; i < n; ++i) x[i] = cands_[i].pos;
    evaluate(x, F, &E);
    for (int i = 0; i < n; ++i) {
      samp_x[i] = x[i];
      samp_f[i] = F[i];
      if (energies) energies[(size_t)i * (nsteps + 1)] = E[i];
    }
    std::vector<double> tang;
    for (int step = 1; step <= nsteps; ++step) {
      build_curves();
      for (int i = 0; i < n; ++i) {
        const size_t m = x[i].size();
        s_end[i] = h * (double)(nodes[i].size() / m - 1);
        std::vector<double> p0;
        point(i, 0.0, p0, &tang);
        double g = 0.0;
        for (size_t c = 0; c < m; ++c) g -= F[i][c] * tang[c];
        g0[i] = g;
        double s = std::min(s_end[i], s_cap);
        if (s_prev[i] > 0) s = std::min(s, 2.0 * s_prev[i]);
        s1[i] = s;
        point(i, s, x1[i], nullptr);
      }
      evaluate(x1, F1, nullptr);
      for (int i = 0; i < n; ++i) {
        std::vector<double> p1;
        point(i, s1[i], p1, &tang);
        double g1 = 0.0;
        for (size_t c = 0; c < tang.size(); ++c) g1 -= F1[i][c] * tang[c];
        double s2 = (g1 - g0[i]) > 0 ? s1[i] * g0[i] / (g0[i] - g1) : 4.0 * s1[i];
        s2 = std::max(0.1 * s1[i], std::min(4.0 * s1[i], s2));
        s2 = std::min(s2, s_end[i]);
        s_prev[i] = s2;
        point(i, s2, x1[i], nullptr);
      }
      evaluate(x1, F1, &E);
      for (int i = 0; i < n; ++i) {
        x[i] = x1[i];
        F[i] = F1[i];
        samp_x[i].insert(samp_x[i].end(), x[i].begin(), x[i].end());
        samp_f[i].insert(samp_f[i].end(), F[i].begin(), F[i].end());
        if (energies) energies[(size_t)i * (nsteps + 1) + step] = E[i];
      }
    }
    int worst = SGO_OK;
    for (int i = 0; i < n; ++i) {
      cands_[i].status = status[i];
      worst = std::min(worst, status[i]);
      if (params)
        for (int k = 0; k < 3; ++k) params[3 * i + k] = prm[i][k];
    }
    return worst;
  }

  int relax(int nsteps, const sgo_scf_opts& o, double* energies, int refit, double* params) {
    const int n = (int)cands_.size();
    const bool pcg = refit >= 0;
    std::vector<std::vector<double>> P(n), samp_x(n), samp_f(n);
    std::vector<std::array<double, 3>> prm(n);
    const double trial_cap = tune("SGO_PCG_TRIAL", 100) * 1e-3;  // bohr
    const double floor = tune("SGO_PCG_FLOOR", 100) * 1e-3;       // of max|tau|
    auto build_P = [&](int i, const std::vector<double>& xi) {
      const HostCand& c = cands_[i];
      const int m = 3 * c.nat;
      ff::fit(c.A, c.nat, (int)(samp_x[i].size() / m), samp_x[i].data(), samp_f[i].data(),
              prm[i].data());
      std::vector<double> H((size_t)m * m);
      ff::morse_hessian(c.A, c.nat, xi.data(), prm[i].data(), H.data());
      P[i].resize((size_t)m * m);
      ff::preconditioner(m, H.data(), P[i].data(), floor);
    };
    // the fits of different candidates are independent: spread them over host threads
    auto build_all = [&](const std::vector<std::vector<double>>& xs) {
      const int nt = std::max(1, std::min({n, (int)std::thread::hardware_concurrency(), 16}));
      std::vector<std::thread> pool;
      std::vector<std::exception_ptr> err(nt);
      for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
          try {
            for (int i = t; i < n; i += nt) build_P(i, xs[i]);
          } catch (...) {
            err[t] = std::current_exception();
          }
        });
      for (auto& th : pool) th.join();
      for (auto& e : err)
        if (e) std::rethrow_exception(e);
    };
    auto apply_P = [&](int i, const std::vector<double>& f, std::vector<double>& out) {
      const size_t m = f.size();
      out.assign(m, 0.0);
      for (size_t k = 0; k < m; ++k) {
        double acc = 0.0;
        for (size_t l = 0; l < m; ++l) acc += P[i][k * m + l] * f[l];
        out[k] = acc;
      }
    };
    std::vector<std::vector<double>> x(n), F(n), d(n), x1(n), F1(n);
    std::vector<double> E(n), alpha_prev(n, 0.0);
    std::vector<int> status(n, SGO_OK);
    auto evaluate = [&](std::vector<std::vector<double>>& pos, std::vector<std::vector<double>>& force,
                        std::vector<double>* en) {
      for (int i = 0; i < n; ++i) move_atoms(i, pos[i].data());
      const int rc = scf(o);
      (void)rc;
      for (int i = 0; i < n; ++i) {
        HostCand& c = cands_[i];
        force[i].resize(3 * c.nat);
        get(c.d.force, force[i].data(), 3 * c.nat * sizeof(double));
        if (en) {
          double s[S_COUNT];
          get_scal(c, s);
          (*en)[i] = s[S_ETOT];
        }
        if (c.status < status[i]) status[i] = c.status;
      }
    };
    for (int i = 0; i < n; ++i) x[i] = cands_[i].pos;
    evaluate(x, F, &E);
    std::vector<double> pf, pg;
    if (pcg) {
      for (int i = 0; i < n; ++i) {
        samp_x[i] = x[i];
        samp_f[i] = F[i];
      }
      build_all(x);
    }
    for (int i = 0; i < n; ++i) {
      if (pcg)
        apply_P(i, F[i], d[i]);
      else
        d[i] = F[i];
      if (energies) energies[(size_t)i * (nsteps + 1)] = E[i];
    }
    std::vector<double> alpha1(n), s0(n);
    for (int step = 1; step <= nsteps; ++step) {
      for (int i = 0; i < n; ++i) {
        double dmax = 0.0, fd = 0.0;
        for (size_t k = 0; k < d[i].size(); k += 3) {
          const double m = std::sqrt(d[i][k] * d[i][k] + d[i][k + 1] * d[i][k + 1] + d[i][k + 2] * d[i][k + 2]);
          dmax = std::max(dmax, m);
        }
        for (size_t k = 0; k < d[i].size(); ++k) fd += F[i][k] * d[i][k];
        double a = dmax > 0 ? (pcg ? std::min(1.0, trial_cap / dmax) : 0.1 / dmax) : 0.0;
        if (alpha_prev[i] > 0) a = std::min(a, 2.0 * alpha_prev[i]);
        alpha1[i] = a;
        s0[i] = -fd;
        x1[i] = x[i];
        for (size_t k = 0; k < x1[i].size(); ++k) x1[i][k] += a * d[i][k];
      }
      evaluate(x1, F1, nullptr);
      for (int i = 0; i < n; ++i) {
        double s1 = 0.0;
        for (size_t k = 0; k < d[i].size(); ++k) s1 -= F1[i][k] * d[i][k];
        double a2 = (s1 - s0[i]) > 0 ? alpha1[i] * s0[i] / (s0[i] - s1) : 4.0 * alpha1[i];
        a2 = std::max(0.1 * alpha1[i], std::min(4.0 * alpha1[i], a2));
        alpha_prev[i] = a2;
        x1[i] = x[i];
        for (size_t k = 0; k < x1[i].size(); ++k) x1[i][k] += a2 * d[i][k];
      }
      evaluate(x1, F1, &E);
      if (pcg) {
        for (int i = 0; i < n; ++i) {
          samp_x[i].insert(samp_x[i].end(), x1[i].begin(), x1[i].end());
          samp_f[i].insert(samp_f[i].end(), F1[i].begin(), F1[i].end());
        }
        if (refit > 0 && step % refit == 0) build_all(x1);
      }
      for (int i = 0; i < n; ++i) {
        double num = 0.0, den = 0.0;
        if (pcg) {
          apply_P(i, F1[i], pg);
          apply_P(i, F[i], pf);
          for (size_t k = 0; k < F1[i].size(); ++k) {
            num += F1[i][k] * (pg[k] - pf[k]);
            den += F[i][k] * pf[k];
          }
          const double beta = den > 0 ? std::max(0.0, num / den) : 0.0;
          for (size_t k = 0; k < d[i].size(); ++k) d[i][k] = pg[k] + beta * d[i][k];
        } else {
          for (size_t k = 0; k < F1[i].size(); ++k) {
            num += F1[i][k] * (F1[i][k] - F[i][k]);
            den += F[i][k] * F[i][k];
          }
          const double beta = den > 0 ? std::max(0.0, num / den) : 0.0;
          for (size_t k = 0; k < d[i].size(); ++k) d[i][k] = F1[i][k] + beta * d[i][k];
        }
        x[i] = x1[i];
        F[i] = F1[i];
        if (energies) energies[(size_t)i * (nsteps + 1) + step] = E[i];
      }
    }
    int worst = SGO_OK;
    for (int i = 0; i < n; ++i) {
      cands_[i].status = status[i];
      worst = std::min(worst, status[i]);
      if (pcg && params)
        for (int k = 0; k < 3; ++k) params[3 * i + k] = prm[i][k];
    }
    return worst;
  }

  template <typename T>
  void apply_h_t(const double* veff, int nbx, const double* psi, double* hpsi) {
    HostCand& c = cands_.at(0);
    if (nbx < 1 || nbx > c.nb) throw Error(SGO_EINVAL, "nb must be in [1, nbands]");
    BatchGeom g = prepare(1, kMaxHist);
    LaunchCtx L = ctx(g);
    setup_geometry<T>(L);
    std::vector<T> v(c.ntot), x((size_t)c.nb * c.Kp, (T)0);
    for (int e = 0; e < c.ntot; ++e) v[e] = (T)veff[e];
    for (int i = 0; i < nbx; ++i)
      for (int k = 0; k < c.K; ++k) x[(size_t)i * c.Kp + k] = (T)psi[(size_t)i * c.K + k];
    HIPCHK(hipMemcpy(c.d.veff_t, v.data(), c.ntot * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c.d.X, x.data(), x.size() * sizeof(T), hipMemcpyHostToDevice));
    launch_hpsi<T>(L, W_X);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    HIPCHK(hipMemcpy(x.data(), c.d.HX, x.size() * sizeof(T), hipMemcpyDeviceToHost));
    for (int i = 0; i < nbx; ++i)
      for (int k = 0; k < c.K; ++k) hpsi[(size_t)i * c.K + k] = (double)x[(size_t)i * c.Kp + k];
    c.have_psi = false;
    c.have_scf = false;
  }
  void apply_h(const double* veff, int nbx, const double* psi, double* hpsi) {
    if (!veff || !psi || !hpsi) throw Error(SGO_EINVAL, "NULL argument");
    HIPCHK(hipSetDevice(device_));
    if (prec_ == SGO_FP64) apply_h_t<double>(veff, nbx, psi, hpsi);
    else apply_h_t<float>(veff, nbx, psi, hpsi);
  }

  HostCand& cand(int i) {
    if (i < 0 || i >= (int)cands_.size()) throw Error(SGO_EINVAL, "candidate index out of range");
    return cands_[i];
  }
  int size() const { return (int)cands_.size(); }
  void require_scf(const HostCand& c) {
    if (!c.have_scf) throw Error(SGO_ESTATE, "sgo_scf has not run for this structure");
  }
  // host reads ordered on the engine's stream: on the legacy null stream
  // they would wait on every blocking stream, and fail while another batch's
  // thread captures a graph
  void get_scal(const HostCand& c, double* out) { get(c.d.scal, out, S_COUNT * 8); }
  void get(const void* src, void* dst, size_t bytes) {
    HIPCHK(hipSetDevice(device_));
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
  }
  void move_atoms(int i, const double* pos) {
    HostCand& c = cand(i);
    if (!pos) throw Error(SGO_EINVAL, "NULL positions");
    std::vector<double> old = c.pos;
    c.pos.assign(pos, pos + 3 * c.nat);
    try {
      check_distances(c);
    } catch (...) {
      c.pos = old;
      throw;
    }
    c.have_scf = false;  // warm start keeps psi
  }
  void replace(int i, const double* lat, int nat, const int* spec, const double* pos, double ecut,
               const int* fft, int nb, int occ_kind, double sigma) {
    HostCand& c = cand(i);
    HostCand n;
    fill_cand(n, lat, nat, spec, pos, ecut, fft, nb, occ_kind, sigma);
    free_cand(c);
    c = std::move(n);
  }
  void reset() {
    for (auto& c : cands_) {
      c.have_psi = false;
      c.have_scf = false;
    }
  }
  int precision() const { return prec_; }
  void set_allocator(void* (*a)(size_t, void*), void (*f)(void*, void*), void* user) {
    for (auto& c : cands_) free_cand(c);  // arenas of the previous allocator
    alloc_fn_ = a;
    free_fn_ = f;
    alloc_user_ = user;
  }

  // Input density of candidate i's last SCF iteration (the one V_eff was
  // built from), [N3][N2][N1].
  void get_input_density(int i, double* rho_in) {
    HostCand& c = cand(i);
    require_scf(c);
    get(c.d.rho_in_r, rho_in, c.ntot * 8);
  }

  // Host copy of candidate i's state (FP64); any pointer may be null.
  void get_state(int i, int* info, int* millers, double* psi, double* eig, double* occ,
                 double* rho, double* veff, sgo_energy_terms* t) {
    HostCand& c = cand(i);
    if (info) {
      const int v[10] = {c.N[0], c.N[1], c.N[2], c.ntot, c.npwh, c.nb, c.npair, c.nst, c.nsp, c.nproj};
      std::memcpy(info, v, sizeof(v));
    }
    if (millers) std::memcpy(millers, c.gmill.data(), c.gmill.size() * sizeof(int));
    if (!(psi || eig || occ || rho || veff || t)) return;
    require_scf(c);
    HIPCHK(hipSetDevice(device_));
    if (psi) {
      const size_t ts = tsize();
      std::vector<char> raw((size_t)c.nb * c.Kp * ts);
      get(c.d.X, raw.data(), raw.size());
      for (int b = 0; b < c.nb; ++b)
        for (int k = 0; k < c.K; ++k) {
          const size_t e = (size_t)b * c.Kp + k;
          psi[(size_t)b * c.K + k] = prec_ == SGO_FP64 ? ((const double*)raw.data())[e]
                                                       : (double)((const float*)raw.data())[e];
        }
    }
    if (eig) get(c.d.eps, eig, c.nb * 8);
    if (occ) get(c.d.occ, occ, c.nb * 8);
    if (rho) get(c.d.rho_out_r, rho, c.ntot * 8);
    if (veff) get(c.d.veff_r, veff, c.ntot * 8);
    if (t) {
      double s[S_COUNT];
      get(c.d.scal, s, S_COUNT * 8);
      t->total = s[S_ETOT];
      t->kinetic = s[S_EKIN];
      t->nonlocal = s[S_ENL];
      t->local = s[S_ELOC];
      t->hartree = s[S_EH];
      t->xc = s[S_EXC];
      t->ewald = s[S_EEW];
      t->entropy = s[S_ENTROPY_TERM];
      t->band = s[S_EBAND];
      t->fermi = s[S_MU];
    }
  }

 private:
  int device_, prec_, capacity_;
  hipStream_t stream_ = nullptr;
  std::vector<SpeciesHost> species_;
  SpeciesDev* d_species_ = nullptr;
  std::vector<HostCand> cands_;
  CandDesc* d_desc_ = nullptr;
  size_t desc_cap_ = 0;
  CandDesc* d_desc_act_ = nullptr;  // descriptors of the active candidates only
  size_t desc_act_cap_ = 0;
  int* d_iter_ = nullptr;             // SCF iteration counter (device)
  double* d_scal_all_ = nullptr;
  int* d_jac_done_ = nullptr;  // Jacobi convergence flags [capacity]
  int* h_jac_done_ = nullptr;      // [ncand][S_COUNT] gathered status scalars (device)
  void* (*alloc_fn_)(size_t, void*) = nullptr;  // caller's device allocator (arenas)
  void (*free_fn_)(void*, void*) = nullptr;
  void* alloc_user_ = nullptr;
  double* h_scal_all_ = nullptr;      // pinned host copy
  size_t scal_cap_ = 0;
  hipStream_t own_stream_ = nullptr;  // used for graph capture when no stream is set
  bool desc_dirty_ = true;
};

}  // namespace sgo

// ====================================================================== C-ABI
using sgo::Engine;
using sgo::Error;

struct sgo_ctx {
  Engine* eng = nullptr;
  std::string err;
  bool cell = false, atoms = false, cutoff = false;
  double lat[9];
  std::vector<int> spec;
  std::vector<double> pos;
  int nat = 0;
  double ecut = 0;
  int fft[3] = {0, 0, 0};
  int nb = 0, occ_kind = 0;
  double sigma = 0;
};
struct sgo_batch {
  Engine* eng = nullptr;
  std::string err;
  std::vector<int> status;
  std::vector<int> nat;
};

static thread_local std::string g_err;

template <typename F>
static int guard(std::string* err, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (err) *err = e.what();
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    return SGO_ENOMEM;
  } catch (const std::exception& e) {
    if (err) *err = e.what();
    g_err = e.what();
    return SGO_EDEVICE;
  }
}

extern "C" {

void sgo_default_opts(sgo_scf_opts* o) {
  if (!o) return;
  o->max_iter = 100;
  o->ncg = 3;
  o->ncg_first = 8;
  o->cg_tol = 0.0;
  o->tol_e = 1e-5;
  o->tol_rho = 1e-4;
  o->mix_alpha = 0.5;
  o->kerker_q0 = 0.8;
  o->history = 8;
  o->seed = 1;
  o->use_graph = 0;
}

const char* sgo_version(void) { return "sgo-mi355x 0.1 (gfx950)"; }

int sgo_create(sgo_ctx** out, int device, int precision) {
  if (!out) return SGO_EINVAL;
  *out = nullptr;
  return guard(nullptr, [&] {
    sgo_ctx* c = new sgo_ctx();
    try {
      c->eng = new Engine(device, precision, 1);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return SGO_OK;
  });
}

int sgo_destroy(sgo_ctx* c) {
  if (!c) return SGO_EINVAL;
  delete c->eng;
  delete c;
  return SGO_OK;
}

int sgo_set_stream(sgo_ctx* c, void* s) {
  if (!c) return SGO_EINVAL;
  c->eng->set_stream(s);
  return SGO_OK;
}

int sgo_set_species(sgo_ctx* c, int id, const sgo_species* sp) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    c->eng->set_species(id, sp);
    return SGO_OK;
  });
}

static void ctx_commit(sgo_ctx* c) {
  if (!(c->cell && c->atoms && c->cutoff)) return;
  if (c->eng->size() == 0)
    c->eng->add(c->lat, c->nat, c->spec.data(), c->pos.data(), c->ecut, c->fft, c->nb, c->occ_kind,
                c->sigma);
  else
    c->eng->replace(0, c->lat, c->nat, c->spec.data(), c->pos.data(), c->ecut, c->fft, c->nb,
                    c->occ_kind, c->sigma);
}

int sgo_set_cell(sgo_ctx* c, const double lattice[9]) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!lattice) throw Error(SGO_EINVAL, "NULL lattice");
    const double* A = lattice;
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(det) > 1e-12)) throw Error(SGO_EINVAL, "cell volume must be positive");
    std::memcpy(c->lat, lattice, sizeof(c->lat));
    c->cell = true;
    if (c->atoms && c->cutoff) ctx_commit(c);
    return SGO_OK;
  });
}

int sgo_set_atoms(sgo_ctx* c, int natoms, const int* species, const double* pos) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!c->cell) throw Error(SGO_ESTATE, "set the cell before the atoms");
    if (natoms <= 0 || !species || !pos) throw Error(SGO_EINVAL, "bad atoms");
    const bool same = c->eng->size() == 1 && natoms == c->nat &&
                      std::equal(species, species + natoms, c->spec.begin());
    if (same && c->cutoff) {
      c->eng->move_atoms(0, pos);
      c->pos.assign(pos, pos + 3 * natoms);
      return SGO_OK;
    }
    std::vector<int> os = c->spec;
    std::vector<double> op = c->pos;
    int on = c->nat;
    bool oa = c->atoms;
    c->nat = natoms;
    c->spec.assign(species, species + natoms);
    c->pos.assign(pos, pos + 3 * natoms);
    c->atoms = true;
    try {
      if (c->cutoff) ctx_commit(c);
    } catch (...) {
      c->spec = os;
      c->pos = op;
      c->nat = on;
      c->atoms = oa;
      throw;
    }
    return SGO_OK;
  });
}

int sgo_set_allocator(sgo_ctx* c, void* (*alloc)(size_t, void*), void (*dealloc)(void*, void*),
                      void* user) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if ((alloc == nullptr) != (dealloc == nullptr))
      throw Error(SGO_EINVAL, "give both allocator hooks or neither");
    c->eng->set_allocator(alloc, dealloc, user);
    return SGO_OK;
  });
}

int sgo_batch_set_allocator(sgo_batch* b, void* (*alloc)(size_t, void*),
                            void (*dealloc)(void*, void*), void* user) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if ((alloc == nullptr) != (dealloc == nullptr))
      throw Error(SGO_EINVAL, "give both allocator hooks or neither");
    b->eng->set_allocator(alloc, dealloc, user);
    return SGO_OK;
  });
}

int sgo_set_cutoff(sgo_ctx* c, double ecut, const int fft[3], int nbands, int occ_kind,
                   double sigma) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!c->cell || !c->atoms) throw Error(SGO_ESTATE, "set the cell and atoms before the cutoff");
    if (!fft) throw Error(SGO_EINVAL, "NULL fft");
    c->ecut = ecut;
    std::memcpy(c->fft, fft, sizeof(c->fft));
    c->nb = nbands;
    c->occ_kind = occ_kind;
    c->sigma = sigma;
    c->cutoff = true;
    try {
      ctx_commit(c);
    } catch (...) {
      c->cutoff = false;
      throw;
    }
    return SGO_OK;
  });
}

static sgo_scf_opts opts_or_default(const sgo_scf_opts* o) {
  sgo_scf_opts d;
  sgo_default_opts(&d);
  return o ? *o : d;
}

int sgo_scf(sgo_ctx* c, const sgo_scf_opts* opts, sgo_scf_info* info) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!(c->cell && c->atoms && c->cutoff) || c->eng->size() == 0)
      throw Error(SGO_ESTATE, "set species, cell, atoms and cutoff first");
    const sgo_scf_opts o = opts_or_default(opts);
    if (o.max_iter < 1 || o.ncg < 1 || o.ncg_first < 1 || !(o.cg_tol >= 0.0))
      throw Error(SGO_EINVAL, "bad options");
    int rc = c->eng->scf(o);
    if (info) *info = c->eng->cand(0).info;
    return rc;
  });
}

int sgo_set_kpoints(sgo_ctx* c, int nk, const double* kfrac, const double* weights) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    c->eng->set_kpoints(nk, kfrac, weights);
    return SGO_OK;
  });
}

int sgo_kpoint_eigenvalues(sgo_ctx* c, double* eig, double* occ) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!eig) throw Error(SGO_EINVAL, "NULL eig");
    c->eng->kpoint_eigenvalues(eig, occ);
    return SGO_OK;
  });
}

int sgo_energy(sgo_ctx* c, double* etot, sgo_energy_terms* t) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    double s[sgo::S_COUNT];
    c->eng->get_scal(hc, s);
    if (etot) *etot = s[sgo::S_ETOT];
    if (t) {
      t->total = s[sgo::S_ETOT];
      t->kinetic = s[sgo::S_EKIN];
      t->nonlocal = s[sgo::S_ENL];
      t->local = s[sgo::S_ELOC];
      t->hartree = s[sgo::S_EH];
      t->xc = s[sgo::S_EXC];
      t->ewald = s[sgo::S_EEW];
      t->entropy = s[sgo::S_ENTROPY_TERM];
      t->band = s[sgo::S_EBAND];
      t->fermi = s[sgo::S_MU];
    }
    return SGO_OK;
  });
}

int sgo_forces(sgo_ctx* c, double* forces) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!forces) throw Error(SGO_EINVAL, "NULL forces");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    c->eng->get(hc.d.force, forces, 3 * hc.nat * sizeof(double));
    return SGO_OK;
  });
}

int sgo_stress(sgo_ctx* c, double stress[9], double* parts) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!stress) throw Error(SGO_EINVAL, "NULL stress");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    if (c->eng->kmode()) throw Error(SGO_EINVAL, "no stress with k-point sampling");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    c->eng->stress();
    double s[63];
    c->eng->get(hc.d.stress, s, sizeof(s));
    for (int k = 0; k < 9; ++k) stress[k] = s[k];
    if (parts)
      for (int k = 0; k < 54; ++k) parts[k] = s[9 + k];
    return SGO_OK;
  });
}

int sgo_eigenvalues(sgo_ctx* c, double* eig, double* occ) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!eig) throw Error(SGO_EINVAL, "NULL eig");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    if (c->eng->kmode()) throw Error(SGO_EINVAL, "k-point sampling: use sgo_kpoint_eigenvalues");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    c->eng->get(hc.d.eps, eig, hc.nb * sizeof(double));
    if (occ) c->eng->get(hc.d.occ, occ, hc.nb * sizeof(double));
    return SGO_OK;
  });
}

int sgo_adjoint(sgo_ctx* c, double gE, double* grad_pos, double* grad_lattice) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!grad_pos) throw Error(SGO_EINVAL, "NULL grad_pos");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    std::vector<double> f(3 * hc.nat);
    c->eng->get(hc.d.force, f.data(), f.size() * sizeof(double));
    for (size_t k = 0; k < f.size(); ++k) grad_pos[k] = -gE * f[k];
    if (grad_lattice && c->eng->kmode())
      throw Error(SGO_EINVAL, "no lattice gradient with k-point sampling");
    if (grad_lattice) {
      // E(A, R) with Cartesian R held fixed: under r -> (1 + eps) r both A
      // and R move, so (dE/dA)^T A - sum_I F_I R_I^T = Omega sigma, i.e.
      // dE/dA = A^-T (Omega sigma + sum_I R_I F_I^T)  (rows of A = a_i).
      c->eng->stress();
      double s[9];
      c->eng->get(hc.d.stress, s, sizeof(s));
      double M[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double v = hc.omega * s[3 * a + b];
          for (int I = 0; I < hc.nat; ++I) v += hc.pos[3 * I + a] * f[3 * I + b];
          M[3 * a + b] = v;
        }
      // A^-T = B / (2 pi) with B the reciprocal rows (b_i . a_j = 2 pi delta_ij)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int k = 0; k < 3; ++k) v += hc.B[3 * i + k] * M[3 * k + j];
          grad_lattice[3 * i + j] = gE * v / (2.0 * sgo::kPiH);
        }
    }
    return SGO_OK;
  });
}

int sgo_reset(sgo_ctx* c) {
  if (!c) return SGO_EINVAL;
  c->eng->reset();
  return SGO_OK;
}

int sgo_basis_size(sgo_ctx* c, int* npw_half, int* nproj) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    if (npw_half) *npw_half = hc.npwh;
    if (nproj) *nproj = hc.nproj;
    return SGO_OK;
  });
}

int sgo_basis_millers(sgo_ctx* c, int* millers) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!millers) throw Error(SGO_EINVAL, "NULL millers");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    std::memcpy(millers, hc.gmill.data(), hc.gmill.size() * sizeof(int));
    return SGO_OK;
  });
}

int sgo_apply_h(sgo_ctx* c, const double* veff, int nb, const double* psi, double* hpsi) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    c->eng->apply_h(veff, nb, psi, hpsi);
    return SGO_OK;
  });
}

int sgo_get_density(sgo_ctx* c, double* rho, double* veff) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& hc = c->eng->cand(0);
    c->eng->require_scf(hc);
    if (rho) c->eng->get(hc.d.rho_out_r, rho, hc.ntot * sizeof(double));
    if (veff) c->eng->get(hc.d.veff_r, veff, hc.ntot * sizeof(double));
    return SGO_OK;
  });
}

const char* sgo_last_error(const sgo_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int sgo_profile_begin(const char* kernel) {
  if (!kernel) return SGO_EINVAL;
  std::lock_guard<std::mutex> lk(sgo::g_prof_mu);
  sgo::g_prof.on = true;
  sgo::g_prof.name = kernel;
  sgo::g_prof.used = 0;
  sgo::g_prof.cand_launches = 0;
  sgo::g_prof.cand_rows = 0;
  return SGO_OK;
}

int sgo_profile_end(int* launches, double* total_ms, long long* cand_launches,
                    long long* cand_rows, double* union_ms) {
  return guard(nullptr, [&] {
    std::lock_guard<std::mutex> lk(sgo::g_prof_mu);
    auto& P = sgo::g_prof;
    double ms = 0.0;
    std::vector<std::pair<double, double>> iv;
    for (size_t k = 0; k + 1 < P.used; k += 2) {
      HIPCHK(hipEventSynchronize(P.ev[k + 1]));
      float t = 0.f, t0 = 0.f, t1 = 0.f;
      HIPCHK(hipEventElapsedTime(&t, P.ev[k], P.ev[k + 1]));
      ms += t;
      if (union_ms) {
        HIPCHK(hipEventElapsedTime(&t0, P.ev[0], P.ev[k]));
        HIPCHK(hipEventElapsedTime(&t1, P.ev[0], P.ev[k + 1]));
        iv.emplace_back(t0, t1);
      }
    }
    if (union_ms) {
      // time during which at least one profiled launch ran (launches of
      // concurrent batches on other streams overlap)
      std::sort(iv.begin(), iv.end());
      double u = 0.0, lo = 0.0, hi = 0.0;
      bool open = false;
      for (auto& x : iv) {
        if (open && x.first <= hi) {
          hi = std::max(hi, x.second);
          continue;
        }
        if (open) u += hi - lo;
        lo = x.first;
        hi = x.second;
        open = true;
      }
      if (open) u += hi - lo;
      *union_ms = u;
    }
    if (launches) *launches = (int)(P.used / 2);
    if (total_ms) *total_ms = ms;
    if (cand_launches) *cand_launches = P.cand_launches;
    if (cand_rows) *cand_rows = P.cand_rows;
    P.on = false;
    P.used = 0;
    P.cand_launches = 0;
    P.cand_rows = 0;
    return SGO_OK;
  });
}

int sgo_subspace_solve(int device, int n, int mode, const double* S, const double* H, double* M,
                       double* eps, int reps, double* ms_per_call, long long* clocks) {
  return guard(nullptr, [&] {
    if (n < 1 || n > 640 || !S || !M || (mode != 1 && mode != 3) || (mode == 3 && (!H || !eps)))
      throw Error(SGO_EINVAL, "bad subspace_solve arguments");
    if (reps < 1) reps = 1;
    HIPCHK(hipSetDevice(device));
    sgo::configure_once(device);
    const size_t nn = (size_t)n * n;
    double *dS, *dH, *dC, *dM, *deps, *dscal, *dSsave, *dHsave;
    long long* dclk;
    HIPCHK(hipMalloc(&dS, nn * 8));
    HIPCHK(hipMalloc(&dH, nn * 8));
    HIPCHK(hipMalloc(&dC, nn * 8));
    HIPCHK(hipMalloc(&dM, nn * 8));
    HIPCHK(hipMalloc(&dSsave, nn * 8));
    HIPCHK(hipMalloc(&dHsave, nn * 8));
    HIPCHK(hipMalloc(&deps, n * 8));
    HIPCHK(hipMalloc(&dscal, sgo::S_COUNT * 8));
    HIPCHK(hipMalloc(&dclk, 8 * sizeof(long long)));
    double* dred;
    int *djac, *hjac;
    HIPCHK(hipMalloc(&dred, 2048 * 8));
    HIPCHK(hipMalloc(&djac, sizeof(int)));
    HIPCHK(hipHostMalloc((void**)&hjac, sizeof(int), hipHostMallocDefault));
    HIPCHK(hipMemset(dscal, 0, sgo::S_COUNT * 8));
    HIPCHK(hipMemcpy(dSsave, S, nn * 8, hipMemcpyHostToDevice));
    if (H) HIPCHK(hipMemcpy(dHsave, H, nn * 8, hipMemcpyHostToDevice));
    sgo::CandDesc d;
    std::memset(&d, 0, sizeof(d));
    d.nb = n;
    d.active = 1;
    d.S = dS;
    d.Hs = dH;
    d.C = dC;
    d.M = dM;
    d.eps = deps;
    d.scal = dscal;
    d.red_part = dred;
    d.dbg_clk = clocks ? dclk : nullptr;
    sgo::CandDesc* dd;
    HIPCHK(hipMalloc(&dd, sizeof(d)));
    HIPCHK(hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice));
    sgo::LaunchCtx L{};
    L.stream = nullptr;
    L.desc = dd;
    L.g.ncand = 1;
    L.g.nb_max = n;
    L.jac_done = djac;
    L.jac_done_host = hjac;
    const char* env = std::getenv("SGO_SUB_THREADS");
    L.g.sub_threads = env ? std::max(64, std::min(512, std::atoi(env) / 64 * 64)) : 512;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float total = 0.f;
    for (int r = 0; r < reps; ++r) {
      HIPCHK(hipMemcpy(dS, dSsave, nn * 8, hipMemcpyDeviceToDevice));
      if (H) HIPCHK(hipMemcpy(dH, dHsave, nn * 8, hipMemcpyDeviceToDevice));
      HIPCHK(hipEventRecord(e0, nullptr));
      sgo::launch_subspace(L, mode);
      HIPCHK(hipEventRecord(e1, nullptr));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      total += t;
    }
    double flag = 0;
    HIPCHK(hipMemcpy(M, dM, nn * 8, hipMemcpyDeviceToHost));
    if (eps && mode == 3) HIPCHK(hipMemcpy(eps, deps, n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&flag, dscal + sgo::S_ERR, 8, hipMemcpyDeviceToHost));
    if (clocks) HIPCHK(hipMemcpy(clocks, dclk, 6 * sizeof(long long), hipMemcpyDeviceToHost));
    if (ms_per_call) *ms_per_call = total / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (void* p : {(void*)dS, (void*)dH, (void*)dC, (void*)dM, (void*)deps, (void*)dscal,
                    (void*)dSsave, (void*)dHsave, (void*)dclk, (void*)dd, (void*)dred,
                    (void*)djac})
      (void)hipFree(p);
    (void)hipHostFree(hjac);
    if (flag != 0.0) throw Error(SGO_ENUMERIC, "overlap matrix is not positive definite");
    return SGO_OK;
  });
}

int sgo_subspace_solve_noalloc(int device, int n, int mode, const double* S, const double* H,
                               double* M, double* eps, int* status, void* hip_stream) {
  return guard(nullptr, [&] {
    if (!S || !M || (mode != 1 && mode != 3) || (mode == 3 && (!H || !eps)))
      throw Error(SGO_EINVAL, "bad subspace_solve_noalloc arguments");
    if (n < 1 || n > sgo::kNoAllocMaxN)
      throw Error(SGO_EINVAL, "subspace_solve_noalloc: n = " + std::to_string(n) +
                                  " is outside 1.." + std::to_string(sgo::kNoAllocMaxN) +
                                  " (the size of its fixed workspace)");
    HIPCHK(hipSetDevice(device));
    sgo::configure_once(device);
    const char* env = std::getenv("SGO_SUB_THREADS");
    const int nthr = env ? std::max(64, std::min(512, std::atoi(env) / 64 * 64)) : 512;
    const int rc = sgo::subspace_noalloc(device, n, mode, S, H, M, eps, status, SGO_ENUMERIC,
                                         (hipStream_t)hip_stream, nthr);
    if (rc != 0) throw Error(SGO_ENUMERIC, "overlap matrix is not positive definite");
    return SGO_OK;
  });
}

int sgo_set_tuning(const char* key, int value) {
  if (!key) return SGO_EINVAL;
  static const char* known[] = {"SGO_GRAM_KC", "SGO_SUB_THREADS", "SGO_SP_CHUNK",
                                "SGO_DENS_CHUNKS", "SGO_RR_SWEEPS", "SGO_PLANE_KERNEL",
                                "SGO_GEMM_KERNEL", "SGO_GRAM_KERNEL", "SGO_PCG_TRIAL",
                                "SGO_PCG_FLOOR", "SGO_JAC_GRID", "SGO_PLANE_GROUP", "SGO_COMPACT",
                                "SGO_GEMM_WAVES", "SGO_GRAM_TILE"};
  bool ok = false;
  for (const char* k : known) ok = ok || std::strcmp(k, key) == 0;
  if (!ok) return SGO_EINVAL;
  if (value <= 0) sgo::g_tuning.erase(key);
  else sgo::g_tuning[key] = value;
  return SGO_OK;
}

int sgo_get_tuning(const char* key) {
  if (!key) return SGO_EINVAL;
  auto it = sgo::g_tuning.find(key);
  return it == sgo::g_tuning.end() ? 0 : it->second;
}

int sgo_grid_info(sgo_ctx* c, int* info) {
  if (!c) return SGO_EINVAL;
  return guard(&c->err, [&] {
    if (!info) throw Error(SGO_EINVAL, "NULL info");
    if (c->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    auto& h = c->eng->cand(0);
    const int v[10] = {h.N[0], h.N[1], h.N[2], h.ntot, h.npwh, h.nb, h.npair, h.nst, h.nsp, h.nproj};
    std::memcpy(info, v, sizeof(v));
    return SGO_OK;
  });
}

// ---------------------------------------------------------------- batches
int sgo_batch_create(sgo_batch** out, int device, int precision, int capacity) {
  if (!out) return SGO_EINVAL;
  *out = nullptr;
  return guard(nullptr, [&] {
    sgo_batch* b = new sgo_batch();
    try {
      b->eng = new Engine(device, precision, capacity);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
    return SGO_OK;
  });
}

int sgo_batch_destroy(sgo_batch* b) {
  if (!b) return SGO_EINVAL;
  delete b->eng;
  delete b;
  return SGO_OK;
}

int sgo_batch_set_stream(sgo_batch* b, void* s) {
  if (!b) return SGO_EINVAL;
  b->eng->set_stream(s);
  return SGO_OK;
}

int sgo_batch_set_species(sgo_batch* b, int id, const sgo_species* sp) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    b->eng->set_species(id, sp);
    return SGO_OK;
  });
}

int sgo_batch_add(sgo_batch* b, const double lattice[9], int natoms, const int* species,
                  const double* pos, double ecut, const int fft[3], int nbands, int occ_kind,
                  double sigma, int* index_out) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    int i = b->eng->add(lattice, natoms, species, pos, ecut, fft, nbands, occ_kind, sigma);
    b->nat.push_back(natoms);
    b->status.push_back(SGO_OK);
    if (index_out) *index_out = i;
    return SGO_OK;
  });
}

int sgo_batch_set_atoms(sgo_batch* b, int i, const double* pos) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    b->eng->move_atoms(i, pos);
    return SGO_OK;
  });
}

int sgo_batch_scf(sgo_batch* b, const sgo_scf_opts* opts, double* energies, double* forces,
                  int* status) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (b->eng->size() == 0) throw Error(SGO_ESTATE, "empty batch");
    const sgo_scf_opts o = opts_or_default(opts);
    int rc = b->eng->scf(o);
    size_t off = 0;
    for (int i = 0; i < b->eng->size(); ++i) {
      auto& hc = b->eng->cand(i);
      if (energies) {
        double s[sgo::S_COUNT];
        b->eng->get_scal(hc, s);
        energies[i] = s[sgo::S_ETOT];
      }
      if (forces) b->eng->get(hc.d.force, forces + off, 3 * hc.nat * sizeof(double));
      off += 3 * hc.nat;
      if (status) status[i] = hc.status;
      b->status[i] = hc.status;
    }
    return rc;
  });
}

int sgo_batches_scf(sgo_batch* const* batches, int n, const sgo_scf_opts* opts,
                    double* energies, double* forces, int* status) {
  if (!batches || n < 1) return SGO_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (!batches[k]) return SGO_EINVAL;
    for (int j = 0; j < k; ++j)
      if (batches[j] == batches[k]) return SGO_EINVAL;
  }
  // output offsets in batch order
  std::vector<size_t> eoff(n + 1, 0), foff(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    const int m = batches[k]->eng->size();
    size_t f = 0;
    for (int i = 0; i < m; ++i) f += 3 * (size_t)batches[k]->eng->cand(i).nat;
    eoff[k + 1] = eoff[k] + m;
    foff[k + 1] = foff[k] + f;
  }
  std::vector<int> rc(n, SGO_OK);
  auto run = [&](int k) {
    rc[k] = sgo_batch_scf(batches[k], opts, energies ? energies + eoff[k] : nullptr,
                          forces ? forces + foff[k] : nullptr, status ? status + eoff[k] : nullptr);
  };
  std::vector<std::thread> pool;
  int inline_from = n;  // batches from here on run on the calling thread
  for (int k = 0; k < n; ++k) {
    try {
      pool.emplace_back(run, k);
    } catch (const std::system_error&) {
      inline_from = k;  // no thread could be started: solve the rest here
      break;
    }
  }
  for (int k = inline_from; k < n; ++k) run(k);
  for (auto& t : pool) t.join();
  // a hard error of any batch (invalid input, allocation, device or state)
  // comes first, in batch order; otherwise the per-candidate outcomes
  // combine as in sgo_batch_scf (SGO_ENUMERIC over SGO_ENOTCONV over SGO_OK)
  for (int k = 0; k < n; ++k)
    if (rc[k] != SGO_OK && rc[k] != SGO_ENOTCONV && rc[k] != SGO_ENUMERIC) return rc[k];
  int worst = SGO_OK;
  for (int k = 0; k < n; ++k) worst = std::min(worst, rc[k]);
  return worst;
}

int sgo_batch_info(sgo_batch* b, int i, sgo_scf_info* info) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (!info) throw Error(SGO_EINVAL, "NULL info");
    *info = b->eng->cand(i).info;
    return SGO_OK;
  });
}

int sgo_batch_relax_cg(sgo_batch* b, int nsteps, const sgo_scf_opts* opts, double* energies,
                       double* forces, double* positions, int* status) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (b->eng->size() == 0) throw Error(SGO_ESTATE, "empty batch");
    if (nsteps < 0) throw Error(SGO_EINVAL, "nsteps must be >= 0");
    const sgo_scf_opts o = opts_or_default(opts);
    const int rc = b->eng->relax_cg(nsteps, o, energies);
    size_t off = 0;
    for (int i = 0; i < b->eng->size(); ++i) {
      auto& hc = b->eng->cand(i);
      if (forces) b->eng->get(hc.d.force, forces + off, 3 * hc.nat * sizeof(double));
      if (positions) std::memcpy(positions + off, hc.pos.data(), 3 * hc.nat * sizeof(double));
      off += 3 * hc.nat;
      if (status) status[i] = hc.status;
    }
    return rc;
  });
}

int sgo_batch_relax_pcg(sgo_batch* b, int nsteps, int refit, const sgo_scf_opts* opts,
                        double* energies, double* forces, double* positions, double* params,
                        int* status) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (b->eng->size() == 0) throw Error(SGO_ESTATE, "empty batch");
    if (nsteps < 0 || refit < 0) throw Error(SGO_EINVAL, "nsteps and refit must be >= 0");
    const sgo_scf_opts o = opts_or_default(opts);
    const int rc = b->eng->relax_pcg(nsteps, o, energies, refit, params);
    size_t off = 0;
    for (int i = 0; i < b->eng->size(); ++i) {
      auto& hc = b->eng->cand(i);
      if (forces) b->eng->get(hc.d.force, forces + off, 3 * hc.nat * sizeof(double));
      if (positions) std::memcpy(positions + off, hc.pos.data(), 3 * hc.nat * sizeof(double));
      off += 3 * hc.nat;
      if (status) status[i] = hc.status;
    }
    return rc;
  });
}

int sgo_batch_relax_cls(sgo_batch* b, int nsteps, const sgo_scf_opts* opts, double* energies,
                        double* forces, double* positions, double* params, int* status) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (b->eng->size() == 0) throw Error(SGO_ESTATE, "empty batch");
    if (nsteps < 0) throw Error(SGO_EINVAL, "nsteps must be >= 0");
    const sgo_scf_opts o = opts_or_default(opts);
    const int rc = b->eng->relax_cls(nsteps, o, energies, params);
    size_t off = 0;
    for (int i = 0; i < b->eng->size(); ++i) {
      auto& hc = b->eng->cand(i);
      if (forces) b->eng->get(hc.d.force, forces + off, 3 * hc.nat * sizeof(double));
      if (positions) std::memcpy(positions + off, hc.pos.data(), 3 * hc.nat * sizeof(double));
      off += 3 * hc.nat;
      if (status) status[i] = hc.status;
    }
    return rc;
  });
}

int sgo_ff_guided_curve(const double lattice[9], int natoms, const double params[3],
                        const double* x0, int max_nodes, double* nodes, int* nnodes) {
  if (!lattice || natoms < 1 || !params || !x0 || !nodes || !nnodes || max_nodes < 1)
    return SGO_EINVAL;
  std::vector<double> v;
  sgo::ff::guided_curve(lattice, natoms, params, x0, 0.02, 1e-3, 200, v);
  const int K = (int)(v.size() / (3 * natoms));
  if (K > max_nodes) return SGO_EINVAL;
  std::memcpy(nodes, v.data(), v.size() * sizeof(double));
  *nnodes = K;
  return SGO_OK;
}

int sgo_ff_morse(const double lattice[9], int natoms, const double* pos, const double params[3],
                 double* energy, double* forces) {
  if (!lattice || natoms < 1 || !pos || !params) return SGO_EINVAL;
  sgo::ff::morse(lattice, natoms, pos, params, energy, forces);
  return SGO_OK;
}

int sgo_ff_hessian(const double lattice[9], int natoms, const double* pos, const double params[3],
                   double* H) {
  if (!lattice || natoms < 1 || !pos || !params || !H) return SGO_EINVAL;
  sgo::ff::morse_hessian(lattice, natoms, pos, params, H);
  return SGO_OK;
}

int sgo_ff_fit(const double lattice[9], int natoms, int nsamples, const double* pos,
               const double* forces, double params[3]) {
  if (!lattice || natoms < 2 || nsamples < 1 || !pos || !forces || !params) return SGO_EINVAL;
  sgo::ff::fit(lattice, natoms, nsamples, pos, forces, params);
  return SGO_OK;
}

int sgo_ff_preconditioner(int m, const double* H, double* P) {
  if (m < 1 || !H || !P) return SGO_EINVAL;
  sgo::ff::preconditioner(m, H, P);
  return SGO_OK;
}

int sgo_batch_get_state(sgo_batch* b, int i, int* info, int* millers, double* psi, double* eig,
                        double* occ, double* rho, double* veff, sgo_energy_terms* terms) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    b->eng->get_state(i, info, millers, psi, eig, occ, rho, veff, terms);
    return SGO_OK;
  });
}

int sgo_batch_get_input_density(sgo_batch* b, int i, double* rho_in) {
  if (!b || !rho_in) return SGO_EINVAL;
  return guard(&b->err, [&] {
    b->eng->get_input_density(i, rho_in);
    return SGO_OK;
  });
}

int sgo_batch_reset(sgo_batch* b) {
  if (!b) return SGO_EINVAL;
  b->eng->reset();
  return SGO_OK;
}

int sgo_batch_stress(sgo_batch* b, double* stress) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (!stress) throw Error(SGO_EINVAL, "NULL stress");
    if (b->eng->size() == 0) throw Error(SGO_ESTATE, "no structure");
    for (int i = 0; i < b->eng->size(); ++i) b->eng->require_scf(b->eng->cand(i));
    b->eng->stress();
    for (int i = 0; i < b->eng->size(); ++i)
      b->eng->get(b->eng->cand(i).d.stress, stress + 9 * i, 9 * sizeof(double));
    return SGO_OK;
  });
}

int sgo_batch_size(sgo_batch* b, int* n) {
  if (!b || !n) return SGO_EINVAL;
  *n = b->eng->size();
  return SGO_OK;
}

const char* sgo_batch_last_error(const sgo_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

int sgo_batch_de_generation(sgo_batch* b, const sgo_de_opts* de, const sgo_scf_opts* opts,
                            const double* parents, const double* e_parent,
                            const sgo_de_draw* draws, double* trial, int* attempt_used,
                            double* e_trial, double* survivors, double* e_survivor, int* take,
                            int* status) {
  if (!b) return SGO_EINVAL;
  return guard(&b->err, [&] {
    if (!de || !parents || !e_parent || !draws) throw Error(SGO_EINVAL, "NULL argument");
    sgo::Engine& eng = *b->eng;
    const int n = eng.size();
    if (n < 4) throw Error(SGO_EINVAL, "a generation needs at least 4 candidates");
    if ((de->mutation != SGO_DE_TRIANGLE && de->mutation != SGO_DE_CLASSIC) ||
        (de->crossover != SGO_DE_PLANE && de->crossover != SGO_DE_SPHERE) ||
        de->relax_steps < 0 || de->attempts < 1 || !(de->dmin >= 0) || !(de->sim_tol >= 0))
      throw Error(SGO_EINVAL, "invalid generation options");
    const sgo::HostCand& c0 = eng.cand(0);
    const int nat = c0.nat, nc = 3 * nat;
    for (int i = 1; i < n; ++i) {
      const sgo::HostCand& c = eng.cand(i);
      if (c.nat != nat || c.spec != c0.spec || !std::equal(c.A, c.A + 9, c0.A))
        throw Error(SGO_EINVAL, "the candidates of a generation share one species array and cell");
    }
    const int na = de->attempts;
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < na; ++a) {
        const int* r = draws[(size_t)i * na + a].r;
        for (int k = 0; k < 3; ++k)
          if (r[k] < 0 || r[k] >= n || r[k] == i || r[k] == r[(k + 1) % 3])
            throw Error(SGO_EINVAL, "donors must be distinct candidates other than the target");
      }
    double emin = e_parent[0];
    for (int i = 1; i < n; ++i) emin = std::min(emin, e_parent[i]);
    std::vector<double> f(n);
    for (int i = 0; i < n; ++i) f[i] = e_parent[i] - (de->fitness_shift ? emin : 0.0);
    auto P = [&](int i) { return parents + (size_t)i * nc; };
    std::vector<double> tr((size_t)n * nc), v(nc), child(nc);
    std::vector<int> used(n, -1);
    for (int i = 0; i < n; ++i) {
      for (int a = 0; a < na && used[i] < 0; ++a) {
        const sgo_de_draw& d = draws[(size_t)i * na + a];
        sgo::de::mutate(nc, P(d.r[0]), P(d.r[1]), P(d.r[2]), f[d.r[0]], f[d.r[1]], f[d.r[2]],
                        de->mutation == SGO_DE_CLASSIC, de->F, v.data());
        const int rc = de->crossover == SGO_DE_PLANE
                           ? sgo::de::cross_plane(nat, c0.spec.data(), v.data(), P(i), d.normal,
                                                  d.axis, child.data(), nullptr, nullptr)
                           : sgo::de::cross_sphere(nat, c0.spec.data(), v.data(), P(i), d.offset,
                                                   d.radius, child.data(), nullptr);
        if (rc == SGO_EINVAL) throw Error(SGO_EINVAL, "invalid crossover draw");
        if (rc != SGO_OK) continue;
        // below dmin (and never closer than the evaluator accepts) the child is rejected
        if (sgo::de::min_distance(c0.A, nat, child.data()) < std::max(de->dmin, 1e-3)) continue;
        bool alike = false;
        for (int j = 0; j < n && de->sim_tol > 0 && !alike; ++j)
          alike = sgo::de::similarity(c0.A, nat, child.data(), P(j)) < de->sim_tol;
        if (alike) continue;
        std::copy(child.begin(), child.end(), tr.begin() + (size_t)i * nc);
        used[i] = a;
      }
      if (used[i] < 0) std::copy(P(i), P(i) + nc, tr.begin() + (size_t)i * nc);
    }
    for (int i = 0; i < n; ++i) eng.move_atoms(i, tr.data() + (size_t)i * nc);
    const int ns = de->relax_steps;
    std::vector<double> en((size_t)n * (ns + 1));
    const sgo_scf_opts o = opts_or_default(opts);
    const int rc = eng.relax_cg(ns, o, en.data());
    int worst = SGO_OK;
    std::vector<double> keep(nc);
    for (int i = 0; i < n; ++i) {
      const sgo::HostCand& c = eng.cand(i);
      const double et = en[(size_t)i * (ns + 1) + ns];
      const int ok = (c.status == SGO_OK && et < e_parent[i]) ? 1 : 0;
      if (ok)
        std::copy(c.pos.begin(), c.pos.end(), keep.begin());
      else
        std::copy(P(i), P(i) + nc, keep.begin());
      if (trial) std::copy(tr.begin() + (size_t)i * nc, tr.begin() + (size_t)(i + 1) * nc, trial + (size_t)i * nc);
      if (attempt_used) attempt_used[i] = used[i];
      if (e_trial) e_trial[i] = et;
      if (take) take[i] = ok;
      if (status) status[i] = c.status;
      if (e_survivor) e_survivor[i] = ok ? et : e_parent[i];
      if (survivors) std::copy(keep.begin(), keep.end(), survivors + (size_t)i * nc);
      if (c.status < worst) worst = c.status;
      eng.move_atoms(i, keep.data());  // the batch keeps the survivors (warm start from the child)
    }
    (void)rc;
    return worst;
  });
}

}  // extern "C"
