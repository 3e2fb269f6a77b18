"""Total energy as a differentiable function of the atomic positions.

`ScfEnergy.apply(positions, ctx, opts)` runs the self-consistent solve of
the structure held by `ctx` (a `Context`) at `positions` (bohr, (natoms, 3),
any torch device) and returns the free energy as a 0-d float64 tensor.  Its
backward returns gE * dE/dR: at self-consistency the energy is variational,
so dE/dR is the Hellmann-Feynman expression -F (local structure-factor sums,
nonlocal projector derivatives, Ewald), which the library evaluates from the
converged state (`sgo_adjoint`).  No derivative through the SCF iterations
is needed, and the wavefunctions are not kept by autograd: the library holds
one set per structure and recomputes them on the next forward call.
"""
import numpy as np
import torch


class ScfEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, positions, ctx, opts=None):
        species = ctx.atom_species
        pos = positions.detach().to("cpu", torch.float64).numpy()
        ctx.set_atoms(species, pos)
        info = ctx.scf(opts)
        energy, _ = ctx.energy()
        grad = ctx.adjoint(1.0)  # dE/dR = -F
        fctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(grad)))
        fctx.info = info
        return torch.tensor(energy, dtype=torch.float64, device=positions.device)

    @staticmethod
    def backward(fctx, gE):
        (g,) = fctx.saved_tensors
        return gE * g.to(device=gE.device, dtype=torch.float64), None, None


def scf_energy(positions, ctx, opts=None):
    return ScfEnergy.apply(positions, ctx, opts)
