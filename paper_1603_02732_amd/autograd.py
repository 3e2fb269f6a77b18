"""Total energy as a differentiable function of the atomic positions and,
optionally, of the cell.

`ScfEnergy.apply(positions, ctx, opts, lattice)` runs the self-consistent
solve of the structure held by `ctx` (a `Context`) at `positions` (bohr,
(natoms, 3), any torch device) and, if `lattice` is a (3, 3) tensor (rows =
lattice vectors), in that cell; it returns the free energy as a 0-d float64
tensor.  At self-consistency the energy is variational in the wavefunctions
and occupations, so no derivative through the SCF iterations is needed:
  dE/dR = -F   (Hellmann-Feynman: local structure-factor sums, nonlocal
               projector derivatives, Ewald),
  dE/dA = A^-T (Omega sigma + sum_I R_I F_I^T)  with Cartesian positions
               held fixed, from the fixed-basis stress sigma,
both evaluated by the library from the converged state (`sgo_adjoint`).  A
new cell rebuilds the plane-wave sphere for its own cutoff, so the lattice
gradient is that of the fixed-basis functional (the Miller set does not move
with an infinitesimal strain).  Autograd keeps no wavefunctions: the library
holds one set per structure and recomputes it on the next forward call.
"""
import numpy as np
import torch


class ScfEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, positions, ctx, opts=None, lattice=None):
        if lattice is not None:
            ctx.set_cell(lattice.detach().to("cpu", torch.float64).numpy())
        species = ctx.atom_species
        pos = positions.detach().to("cpu", torch.float64).numpy()
        ctx.set_atoms(species, pos)
        info = ctx.scf(opts)
        energy, _ = ctx.energy()
        if lattice is not None:
            gpos, glat = ctx.adjoint(1.0, lattice=True)
            fctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(gpos)),
                                   torch.from_numpy(np.ascontiguousarray(glat)))
        else:
            gpos = ctx.adjoint(1.0)  # dE/dR = -F
            fctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(gpos)))
        fctx.info = info
        fctx.lattice_device = None if lattice is None else lattice.device
        return torch.tensor(energy, dtype=torch.float64, device=positions.device)

    @staticmethod
    def backward(fctx, gE):
        saved = fctx.saved_tensors
        gpos = gE * saved[0].to(device=gE.device, dtype=torch.float64)
        glat = None
        if len(saved) > 1:
            glat = (gE * saved[1].to(device=gE.device, dtype=torch.float64)).to(fctx.lattice_device)
        return gpos, None, None, glat


def scf_energy(positions, ctx, opts=None, lattice=None):
    return ScfEnergy.apply(positions, ctx, opts, lattice)
