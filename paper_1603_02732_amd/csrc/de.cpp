// Differential-evolution operators (Section 2.2), host code.
//
// mutation    Eq. 1 V = X3 + F (X1 - X2), or the triangle form of Eq. 2: V is
//             the affine combination sum_k (4/3 - 3 p_k) X_k of the three
//             donors with p_k = |f_k| / sum |f| (the printed form expanded);
// crossover   plane or sphere cut-and-splice: the child keeps P1's atoms on
//             one side of a plane through P1's centroid (outside a sphere) and
//             takes P2's on the other side (inside), P2 translated by the
//             difference of the centroids; the plane turns about an axis, and
//             P1's part of the sphere scheme is re-chosen per species, until
//             the child has P1's composition;
// checks      minimum interatomic distance and a sorted pair-distance
//             fingerprint (minimum image over the 27 neighbouring cells);
// init        random placement in the cell, a ball or a slab with a minimum
//             distance, one trial atom per three uniforms.
#include "de.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "../../include/sgo.h"

namespace sgo {
namespace de {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 at(const double* p, int j) { return {p[3 * j], p[3 * j + 1], p[3 * j + 2]}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

V3 centroid(int n, const double* p) {
  V3 c{0, 0, 0};
  for (int j = 0; j < n; ++j) c = add(c, at(p, j));
  return scale(c, 1.0 / n);
}

// the 27 lattice translations sum_i n_i a_i, n_i in {-1, 0, 1}
std::vector<V3> shifts27(const double* A) {
  std::vector<V3> s;
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j)
      for (int k = -1; k <= 1; ++k)
        s.push_back({i * A[0] + j * A[3] + k * A[6], i * A[1] + j * A[4] + k * A[7],
                     i * A[2] + j * A[5] + k * A[8]});
  return s;
}

double image_distance(V3 d, const std::vector<V3>& sh) {
  double best = INFINITY;
  for (const V3& t : sh) best = std::min(best, norm(add(d, t)));
  return best;
}

std::vector<double> pair_list(const double* A, int n, const double* p) {
  const auto sh = shifts27(A);
  std::vector<double> out;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) out.push_back(image_distance(sub(at(p, i), at(p, j)), sh));
  return out;
}

// Child slots follow P1's species array: for each species, P1's chosen atoms
// (ascending index) fill its slots first, then P2's.  `from1`/`from2` are
// ascending index lists.  Writes child positions (P2 shifted by c12) and the
// (parent, index) source pairs.
bool fill(int n, const int* species, const std::vector<int>& from1, const std::vector<int>& from2,
          const double* p1, const double* p2, V3 c12, double* child, int* source) {
  std::map<int, std::vector<std::pair<int, int>>> pool;
  for (int j : from1) pool[species[j]].push_back({0, j});
  for (int j : from2) pool[species[j]].push_back({1, j});
  std::map<int, size_t> next;
  for (int slot = 0; slot < n; ++slot) {
    auto& q = pool[species[slot]];
    size_t& k = next[species[slot]];
    if (k >= q.size()) return false;
    const auto src = q[k++];
    const V3 x = src.first == 0 ? at(p1, src.second) : add(at(p2, src.second), c12);
    child[3 * slot] = x.x;
    child[3 * slot + 1] = x.y;
    child[3 * slot + 2] = x.z;
    if (source) {
      source[2 * slot] = src.first;
      source[2 * slot + 1] = src.second;
    }
  }
  for (auto& kv : pool)
    if (next[kv.first] != kv.second.size()) return false;
  return true;
}

}  // namespace

int mutate(int ncoord, const double* x1, const double* x2, const double* x3, double f1, double f2,
           double f3, int classic, double F, double* v) {
  if (ncoord < 0 || !x1 || !x2 || !x3 || !v) return SGO_EINVAL;
  if (classic) {
    for (int k = 0; k < ncoord; ++k) v[k] = x3[k] + F * (x1[k] - x2[k]);
    return SGO_OK;
  }
  const double s = std::fabs(f1) + std::fabs(f2) + std::fabs(f3);
  double p1 = 1.0 / 3.0, p2 = 1.0 / 3.0, p3 = 1.0 / 3.0;
  if (s > 0) {
    p1 = std::fabs(f1) / s;
    p2 = std::fabs(f2) / s;
    p3 = std::fabs(f3) / s;
  }
  const double w1 = 4.0 / 3.0 - 3.0 * p1, w2 = 4.0 / 3.0 - 3.0 * p2, w3 = 4.0 / 3.0 - 3.0 * p3;
  for (int k = 0; k < ncoord; ++k) v[k] = w1 * x1[k] + w2 * x2[k] + w3 * x3[k];
  return SGO_OK;
}

int cross_plane(int n, const int* species, const double* p1, const double* p2,
                const double* normal, const double* axis, double* child, int* source,
                double* theta_out) {
  if (n <= 0 || !species || !p1 || !p2 || !normal || !axis || !child) return SGO_EINVAL;
  V3 nv{normal[0], normal[1], normal[2]};
  const double nn = norm(nv);
  if (!(nn > 0)) return SGO_EINVAL;
  nv = scale(nv, 1.0 / nn);
  V3 av{axis[0], axis[1], axis[2]};
  av = sub(av, scale(nv, dot(av, nv)));
  const double na = norm(av);
  if (!(na > 1e-12 * std::max(1.0, norm(V3{axis[0], axis[1], axis[2]})))) return SGO_EINVAL;
  av = scale(av, 1.0 / na);
  const V3 wv = cross(av, nv);  // the normal turns as n cos(t) + w sin(t)
  const V3 c1 = centroid(n, p1), c2 = centroid(n, p2);
  std::vector<V3> r1(n), r2(n);
  for (int j = 0; j < n; ++j) {
    r1[j] = sub(at(p1, j), c1);
    r2[j] = sub(at(p2, j), c2);
  }
  std::map<int, int> want;
  for (int j = 0; j < n; ++j) ++want[species[j]];
  // an atom changes side where its component along n(t) vanishes
  std::vector<double> ev;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < n; ++j) {
      const V3 r = pass == 0 ? r1[j] : r2[j];
      const double u = dot(r, nv), w = dot(r, wv);
      if (u == 0.0 && w == 0.0) continue;
      double t = std::fmod(std::atan2(-u, w), M_PI);
      if (t < 0) t += M_PI;
      ev.push_back(t);
      ev.push_back(t + M_PI);
    }
  std::sort(ev.begin(), ev.end());
  ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
  std::vector<double> cand{0.0};
  for (size_t k = 0; k < ev.size(); ++k) {
    const double hi = k + 1 < ev.size() ? ev[k + 1] : ev[0] + 2.0 * M_PI;
    cand.push_back(0.5 * (ev[k] + hi));
  }
  std::vector<int> up, down;
  for (double t : cand) {
    const V3 nt = add(scale(nv, std::cos(t)), scale(wv, std::sin(t)));
    up.clear();
    down.clear();
    for (int j = 0; j < n; ++j)
      if (dot(r1[j], nt) > 0) up.push_back(j);
    for (int j = 0; j < n; ++j)
      if (!(dot(r2[j], nt) > 0)) down.push_back(j);
    if ((int)(up.size() + down.size()) != n) continue;
    std::map<int, int> got;
    for (int j : up) ++got[species[j]];
    for (int j : down) ++got[species[j]];
    if (got != want) continue;
    if (!fill(n, species, up, down, p1, p2, sub(c1, c2), child, source)) continue;
    if (theta_out) *theta_out = t;
    return SGO_OK;
  }
  return SGO_ENUMERIC;
}

int cross_sphere(int n, const int* species, const double* p1, const double* p2,
                 const double* offset, double radius, double* child, int* source) {
  if (n <= 0 || !species || !p1 || !p2 || !offset || !child || !(radius >= 0)) return SGO_EINVAL;
  const V3 t{offset[0], offset[1], offset[2]};
  const V3 c1 = centroid(n, p1), c2 = centroid(n, p2);
  const V3 s1 = add(c1, t), s2 = add(c2, t);
  std::vector<int> in2;
  std::map<int, int> k2;
  for (int j = 0; j < n; ++j)
    if (norm(sub(at(p2, j), s2)) < radius) {
      in2.push_back(j);
      ++k2[species[j]];
    }
  std::map<int, std::vector<int>> by;
  for (int j = 0; j < n; ++j) by[species[j]].push_back(j);
  std::vector<int> keep1;
  for (auto& kv : by) {
    auto idx = kv.second;
    std::vector<double> dist(n);
    for (int j : idx) dist[j] = norm(sub(at(p1, j), s1));
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return dist[a] > dist[b]; });
    const int m = (int)idx.size() - k2[kv.first];
    keep1.insert(keep1.end(), idx.begin(), idx.begin() + m);
  }
  std::sort(keep1.begin(), keep1.end());
  if (!fill(n, species, keep1, in2, p1, p2, sub(c1, c2), child, source)) return SGO_ENUMERIC;
  return SGO_OK;
}

double min_distance(const double* A, int n, const double* p) {
  const auto d = pair_list(A, n, p);
  return d.empty() ? INFINITY : *std::min_element(d.begin(), d.end());
}

double similarity(const double* A, int n, const double* pa, const double* pb) {
  auto da = pair_list(A, n, pa), db = pair_list(A, n, pb);
  if (da.empty()) return 0.0;
  std::sort(da.begin(), da.end());
  std::sort(db.begin(), db.end());
  double s = 0.0;
  for (size_t k = 0; k < da.size(); ++k) s += std::fabs(da[k] - db[k]);
  return s / (double)da.size();
}

int init_positions(const double* A, int n, int region, const double* params, double dmin,
                   const double* u, int nu, double* pos, int* used) {
  if (!A || n < 0 || !pos || (nu > 0 && !u) || region < 0 || region > 2) return SGO_EINVAL;
  if (region > 0 && (!params || !(params[0] >= 0))) return SGO_EINVAL;
  const auto sh = shifts27(A);
  const V3 a0{A[0], A[1], A[2]}, a1{A[3], A[4], A[5]}, a2{A[6], A[7], A[8]};
  const V3 centre = scale(add(add(a0, a1), a2), 0.5);
  int placed = 0, k = 0;
  while (placed < n) {
    if (k + 3 > nu) {
      if (used) *used = k;
      return SGO_ENUMERIC;
    }
    const double a = u[k], b = u[k + 1], c = u[k + 2];
    k += 3;
    V3 x;
    if (region == 0) {
      x = add(add(scale(a0, a), scale(a1, b)), scale(a2, c));
    } else if (region == 1) {
      const double r = params[0] * std::pow(a, 1.0 / 3.0);
      const double ct = 2.0 * b - 1.0, st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
      const double ph = 2.0 * M_PI * c;
      x = add(centre, scale(V3{st * std::cos(ph), st * std::sin(ph), ct}, r));
    } else {
      const double zc = 0.5 + (2.0 * c - 1.0) * params[0] / norm(a2);
      x = add(add(scale(a0, a), scale(a1, b)), scale(a2, zc));
    }
    bool ok = true;
    for (int j = 0; j < placed && ok; ++j)
      if (image_distance(sub(x, at(pos, j)), sh) < dmin) ok = false;
    if (!ok) continue;
    pos[3 * placed] = x.x;
    pos[3 * placed + 1] = x.y;
    pos[3 * placed + 2] = x.z;
    ++placed;
  }
  if (used) *used = k;
  return SGO_OK;
}

}  // namespace de
}  // namespace sgo

extern "C" {

int sgo_de_mutate(int ncoord, const double* x1, const double* x2, const double* x3, double f1,
                  double f2, double f3, int scheme, double F, double* v) {
  if (scheme != SGO_DE_TRIANGLE && scheme != SGO_DE_CLASSIC) return SGO_EINVAL;
  return sgo::de::mutate(ncoord, x1, x2, x3, f1, f2, f3, scheme == SGO_DE_CLASSIC, F, v);
}

int sgo_de_cross_plane(int natoms, const int* species, const double* p1, const double* p2,
                       const double normal[3], const double axis[3], double* child, int* source,
                       double* theta) {
  return sgo::de::cross_plane(natoms, species, p1, p2, normal, axis, child, source, theta);
}

int sgo_de_cross_sphere(int natoms, const int* species, const double* p1, const double* p2,
                        const double offset[3], double radius, double* child, int* source) {
  return sgo::de::cross_sphere(natoms, species, p1, p2, offset, radius, child, source);
}

int sgo_de_min_distance(const double lattice[9], int natoms, const double* pos, double* dmin) {
  if (!lattice || natoms < 0 || (natoms > 0 && !pos) || !dmin) return SGO_EINVAL;
  *dmin = sgo::de::min_distance(lattice, natoms, pos);
  return SGO_OK;
}

int sgo_de_similarity(const double lattice[9], int natoms, const double* pa, const double* pb,
                      double* s) {
  if (!lattice || natoms < 0 || (natoms > 0 && (!pa || !pb)) || !s) return SGO_EINVAL;
  *s = sgo::de::similarity(lattice, natoms, pa, pb);
  return SGO_OK;
}

int sgo_de_init_positions(const double lattice[9], int natoms, int region, const double* params,
                          double dmin, const double* uniforms, int nuniform, double* pos,
                          int* used) {
  return sgo::de::init_positions(lattice, natoms, region, params, dmin, uniforms, nuniform, pos,
                                 used);
}

int sgo_de_jitter_cell(const double lattice[9], double delta, const double u[3], double out[9]) {
  if (!lattice || !u || !out || !(delta >= 0)) return SGO_EINVAL;
  for (int k = 0; k < 3; ++k) {
    const double f = 1.0 + delta * (2.0 * u[k] - 1.0);
    for (int c = 0; c < 3; ++c) out[3 * k + c] = lattice[3 * k + c] * f;
  }
  return SGO_OK;
}

int sgo_de_select(int n, const double* e_parent, const double* e_child, const int* child_status,
                  int* take) {
  if (n < 0 || (n > 0 && (!e_parent || !e_child || !take))) return SGO_EINVAL;
  for (int i = 0; i < n; ++i) {
    const bool ok = !child_status || child_status[i] == SGO_OK;
    take[i] = (ok && e_child[i] < e_parent[i]) ? 1 : 0;
  }
  return SGO_OK;
}

}  // extern "C"
