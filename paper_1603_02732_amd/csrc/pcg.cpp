// Force-fitted inverse-Hessian preconditioner (Section 2.3, PCG option),
// host code.
//
// Force field: Morse pairs E = sum D [(1 - e^{-a (r - r0)})^2 - 1] (minimum
// image).  With e = e^{-a (r - r0)}: dE/dr = 2 D a (1 - e) e and
// d2E/dr2 = 2 D a^2 e (2e - 1); a pair block of the Hessian is
// E'' u u^T + (E'/r)(I - u u^T), u the unit pair vector.
// Fit: the forces are linear in D, so for each (a, r0) D is the least-squares
// optimum; (a, r0) come from a 51 x 41 grid (a from 0.5 in steps of 0.05, r0
// from 0.80 to 1.60 of the smallest sampled distance in steps of 0.02) and a
// compass search inside the same box that halves its steps 30 times.
// Preconditioner: cyclic Jacobi eigen-decomposition of the Hessian; the
// translations (|tau| <= 1e-6 max|tau|) are dropped, the other modes weighted
// by 1 / max(|tau|, floor max|tau|) (floor 0.1 by default) so that P stays
// positive semi-definite.
#include "pcg.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sgo {
namespace ff {
namespace {

struct Pair {
  int i, j;
  double d[3];  // r_i - r_j, minimum image
  double r;
};

std::vector<Pair> pairs(const double* A, int n, const double* pos) {
  std::vector<Pair> out;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      Pair p{i, j, {0, 0, 0}, INFINITY};
      double best = INFINITY;
      for (int s0 = -1; s0 <= 1; ++s0)
        for (int s1 = -1; s1 <= 1; ++s1)
          for (int s2 = -1; s2 <= 1; ++s2) {
            double d[3], r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
              d[k] = pos[3 * i + k] - pos[3 * j + k] + s0 * A[k] + s1 * A[3 + k] + s2 * A[6 + k];
              r2 += d[k] * d[k];
            }
            if (r2 < best) {
              best = r2;
              for (int k = 0; k < 3; ++k) p.d[k] = d[k];
            }
          }
      p.r = std::sqrt(best);
      out.push_back(p);
    }
  return out;
}

// forces of unit D for one geometry's pair list, accumulated into g
void unit_forces(const std::vector<Pair>& pl, double a, double r0, double* g) {
  for (const Pair& p : pl) {
    const double ex = std::exp(-a * (p.r - r0));
    const double dEdr = 2.0 * a * (1.0 - ex) * ex;
    for (int k = 0; k < 3; ++k) {
      const double c = dEdr * p.d[k] / p.r;
      g[3 * p.i + k] -= c;
      g[3 * p.j + k] += c;
    }
  }
}

// squared force error minimised over D; +inf when the optimum D is not positive
double objective(const std::vector<std::vector<Pair>>& pls, int n, const double* forces, double a,
                 double r0, double* D) {
  double gg = 0.0, gf = 0.0, ff = 0.0;
  std::vector<double> g(3 * n);
  for (size_t s = 0; s < pls.size(); ++s) {
    std::fill(g.begin(), g.end(), 0.0);
    unit_forces(pls[s], a, r0, g.data());
    const double* F = forces + s * 3 * n;
    for (int k = 0; k < 3 * n; ++k) {
      gg += g[k] * g[k];
      gf += g[k] * F[k];
      ff += F[k] * F[k];
    }
  }
  if (!(gg > 0.0)) {
    *D = 0.0;
    return INFINITY;
  }
  *D = gf / gg;
  if (!(*D > 0.0)) return INFINITY;
  return ff - gf * gf / gg;
}

// cyclic Jacobi: A (m x m, symmetric, destroyed) -> eigenvalues w, vectors V (columns)
void jacobi_eigen(int m, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  double norm = 0.0;
  for (double x : A) norm += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += 2.0 * A[(size_t)p * m + q] * A[(size_t)p * m + q];
    if (off <= 1e-30 * norm) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {  // columns p, q
          const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {  // rows p, q
          const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = c * vkp - s * vkq;
          V[(size_t)k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A[(size_t)i * m + i];
}

}  // namespace

void morse(const double* A, int n, const double* pos, const double* prm, double* energy,
           double* forces) {
  const auto pl = pairs(A, n, pos);
  double e = 0.0;
  if (forces) std::fill(forces, forces + 3 * n, 0.0);
  for (const Pair& p : pl) {
    const double ex = std::exp(-prm[1] * (p.r - prm[2]));
    e += prm[0] * ((1.0 - ex) * (1.0 - ex) - 1.0);
    if (forces) {
      const double dEdr = 2.0 * prm[0] * prm[1] * (1.0 - ex) * ex;
      for (int k = 0; k < 3; ++k) {
        const double c = dEdr * p.d[k] / p.r;
        forces[3 * p.i + k] -= c;
        forces[3 * p.j + k] += c;
      }
    }
  }
  if (energy) *energy = e;
}

void morse_hessian(const double* A, int n, const double* pos, const double* prm, double* H) {
  const int m = 3 * n;
  std::fill(H, H + (size_t)m * m, 0.0);
  for (const Pair& p : pairs(A, n, pos)) {
    const double D = prm[0], a = prm[1];
    const double ex = std::exp(-a * (p.r - prm[2]));
    const double d1 = 2.0 * D * a * (1.0 - ex) * ex;
    const double d2 = 2.0 * D * a * a * ex * (2.0 * ex - 1.0);
    double u[3];
    for (int k = 0; k < 3; ++k) u[k] = p.d[k] / p.r;
    double K[3][3];
    for (int k = 0; k < 3; ++k)
      for (int l = k; l < 3; ++l) {  // symmetric block, computed once per pair (k, l)
        const double uu = u[k] * u[l];
        K[k][l] = K[l][k] = d2 * uu + (d1 / p.r) * ((k == l ? 1.0 : 0.0) - uu);
      }
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        H[(size_t)(3 * p.i + k) * m + 3 * p.i + l] += K[k][l];
        H[(size_t)(3 * p.j + k) * m + 3 * p.j + l] += K[k][l];
        H[(size_t)(3 * p.i + k) * m + 3 * p.j + l] -= K[k][l];
        H[(size_t)(3 * p.j + k) * m + 3 * p.i + l] -= K[k][l];
      }
  }
}

void fit(const double* A, int n, int ns, const double* pos, const double* forces, double* prm) {
  std::vector<std::vector<Pair>> pls;
  double rmin = INFINITY;
  for (int s = 0; s < ns; ++s) {
    pls.push_back(pairs(A, n, pos + (size_t)s * 3 * n));
    for (const Pair& p : pls.back()) rmin = std::min(rmin, p.r);
  }
  double best = INFINITY, a = 0.0, r0 = 0.0, D = 0.0;
  for (int ia = 0; ia < 51; ++ia)
    for (int ir = 0; ir < 41; ++ir) {
      const double ta = 0.5 + 0.05 * ia, tr = rmin * (0.80 + 0.02 * ir);
      const double v = objective(pls, n, forces, ta, tr, &D);
      if (v < best) {
        best = v;
        a = ta;
        r0 = tr;
      }
    }
  if (!(best < INFINITY)) {
    prm[0] = 0.1;
    prm[1] = 1.0;
    prm[2] = rmin;
    return;
  }
  double sa = 0.05, sr = 0.02 * rmin;
  const double moves[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
  for (int h = 0; h < 30; ++h) {
    bool moved = true;
    while (moved) {
      moved = false;
      for (const auto& mv : moves) {
        const double ta = a + mv[0] * sa, tr = r0 + mv[1] * sr;
        if (!(ta >= 0.5 && ta <= 3.0 && tr >= 0.8 * rmin && tr <= 1.6 * rmin)) continue;
        const double v = objective(pls, n, forces, ta, tr, &D);
        if (v < best) {
          best = v;
          a = ta;
          r0 = tr;
          moved = true;
          break;
        }
      }
    }
    sa *= 0.5;
    sr *= 0.5;
  }
  objective(pls, n, forces, a, r0, &D);
  prm[0] = D;
  prm[1] = a;
  prm[2] = r0;
}

void guided_curve(const double* A, int n, const double* prm, const double* x0, double h,
                  double ftol, int kmax, std::vector<double>& nodes) {
  const int m = 3 * n;
  std::vector<double> x(x0, x0 + m), F(m);
  nodes.assign(x.begin(), x.end());
  for (int k = 0; k < kmax; ++k) {
    morse(A, n, x.data(), prm, nullptr, F.data());
    double fm = 0.0;
    for (int I = 0; I < n; ++I)
      fm = std::max(fm, std::sqrt(F[3 * I] * F[3 * I] + F[3 * I + 1] * F[3 * I + 1] +
                                  F[3 * I + 2] * F[3 * I + 2]));
    if (fm < ftol) break;
    for (int c = 0; c < m; ++c) x[c] += h * F[c] / fm;
    nodes.insert(nodes.end(), x.begin(), x.end());
  }
}

void preconditioner(int m, const double* H, double* P, double floor) {
  std::vector<double> Aw(H, H + (size_t)m * m), w, V;
  jacobi_eigen(m, Aw, w, V);
  double tmax = 0.0;
  for (double t : w) tmax = std::max(tmax, std::fabs(t));
  std::fill(P, P + (size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    if (std::fabs(w[j]) <= 1e-6 * tmax) continue;
    const double inv = 1.0 / std::max(std::fabs(w[j]), floor * tmax);
    for (int k = 0; k < m; ++k) {
      const double vk = V[(size_t)k * m + j] * inv;
      for (int l = 0; l < m; ++l) P[(size_t)k * m + l] += vk * V[(size_t)l * m + j];
    }
  }
}

}  // namespace ff
}  // namespace sgo
