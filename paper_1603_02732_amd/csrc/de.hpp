// Differential-evolution operators of the structure search (Section 2.2),
// host code: they touch a few kilobytes of positions per generation, so they
// run on the CPU beside the batched GPU evaluator that dominates the time.
// Positions are Cartesian bohr, [natoms][3]; lattices are three row vectors.
// Every random number is an argument.  Return values are SGO_* codes.
#pragma once

namespace sgo {
namespace de {

// Eq. 2 (triangle) when classic == 0, Eq. 1 with scale F otherwise.
int mutate(int ncoord, const double* x1, const double* x2, const double* x3, double f1, double f2,
           double f3, int classic, double F, double* v);
// Plane cut-and-splice; SGO_ENUMERIC when no orientation of the plane about
// `axis` gives P1's per-species counts.
int cross_plane(int natoms, const int* species, const double* p1, const double* p2,
                const double* normal, const double* axis, double* child, int* source,
                double* theta);
int cross_sphere(int natoms, const int* species, const double* p1, const double* p2,
                 const double* offset, double radius, double* child, int* source);
// Minimum-image distance over the 27 neighbouring cells of every pair.
double min_distance(const double* lattice, int natoms, const double* pos);
double similarity(const double* lattice, int natoms, const double* pa, const double* pb);
int init_positions(const double* lattice, int natoms, int region, const double* params,
                   double dmin, const double* uniforms, int nuniform, double* pos, int* used);

}  // namespace de
}  // namespace sgo
