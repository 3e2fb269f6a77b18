// Force-fitted inverse-Hessian preconditioner for the PCG relaxation
// (Section 2.3), host code: a Morse pair force field fitted to the DFT
// forces, its Hessian, and the inverse over the modes with non-zero
// eigenvalue.  Sizes are a few hundred coordinates at most.
#pragma once

#include <vector>

namespace sgo {
namespace ff {

// params = {D, a, r0}; E = sum_{i<j} D [(1 - e^{-a (r - r0)})^2 - 1] over
// minimum-image pairs.  energy and forces (nullable) out.
void morse(const double* lattice, int natoms, const double* pos, const double* params,
           double* energy, double* forces);
// Analytic Hessian [3n][3n] of the Morse energy.
void morse_hessian(const double* lattice, int natoms, const double* pos, const double* params,
                   double* H);
// Fit of {D, a, r0} to nsamples (positions, forces) pairs, each [natoms][3].
void fit(const double* lattice, int natoms, int nsamples, const double* pos, const double* forces,
         double* params);
// Guided curve of the CLS relaxation: nodes of the steepest-descent path of
// the fitted energy from x0, x_{k+1} = x_k + h F(x_k) / max_atom |F(x_k)|,
// until max_atom |F| < ftol or kmax steps.  nodes receives (K+1) * 3n values.
void guided_curve(const double* lattice, int natoms, const double* params, const double* x0,
                  double h, double ftol, int kmax, std::vector<double>& nodes);
// P = sum over modes with |tau| > 1e-6 max|tau| of v v^T / max(|tau|, floor max|tau|).
void preconditioner(int m, const double* H, double* P, double floor = 0.1);

}  // namespace ff
}  // namespace sgo
