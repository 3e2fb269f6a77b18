"""FP64 CPU oracle for the Gamma-point plane-wave Kohn-Sham energy and forces.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
path (no kernels, headers, helpers, tables or constant generators); the two
meet only at the seeded inputs of the `workloads` package.

What it computes (the discretised Kohn-Sham functional that the paper's
energy engine minimises self-consistently, Section 2.4 and Algorithm 1):
  * full complex plane-wave sphere |G|^2/2 <= Ecut (no half-sphere packing),
  * products on the given FFT grid (aliasing is part of the definition),
  * analytic local pseudopotentials and Gaussian Kleinman-Bylander
    projectors, Perdew-Zunger LDA, Ewald ion-ion energy,
  * the self-consistent fixed point found by dense diagonalisation of H
    (iterative LOBPCG only where the dense matrix would not fit) and
    Pulay/Kerker density mixing, converged far below the parity tolerance,
  * Hellmann-Feynman forces and the fixed-basis stress.

Modules: basis, pseudo, lda, ewald, hamiltonian, scf, forces, stress.
"""
from . import basis, pseudo, lda, ewald, hamiltonian, scf, forces, stress  # noqa: F401
from .scf import run_scf  # noqa: F401
