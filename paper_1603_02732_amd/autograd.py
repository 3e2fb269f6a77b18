"""Total energy as a differentiable function of the atomic positions and,
optionally, of the cell.

`ScfEnergy.apply(positions, ctx, opts, lattice)` runs the self-consistent
solve of the structure held by `ctx` (a `Context`) at `positions` (bohr,
(natoms, 3), any torch device) and, if `lattice` is a (3, 3) tensor (rows =
lattice vectors), in that cell; it returns the free energy as a 0-d float64
tensor.  At self-consistency the energy is variational in the wavefunctions
and occupations, so no derivative through the SCF iterations is needed
(Section 2.1: the forces of each structure):
  dE/dR = -F   (Hellmann-Feynman: local structure-factor sums, nonlocal
               projector derivatives, Ewald),
  dE/dA = A^-T (Omega sigma + sum_I R_I F_I^T)  with Cartesian positions
               held fixed, from the fixed-basis stress sigma,
both evaluated by the library from a converged state (`sgo_adjoint`).  A
new cell rebuilds the plane-wave sphere for its own cutoff, so the lattice
gradient is that of the fixed-basis functional (the Miller set does not move
with an infinitesimal strain).

The adjoint runs in `backward` only, so a forward pass that no backward
follows costs one solve.  Autograd keeps no wavefunctions: the library
holds one set per structure.  If that state has changed since the forward
pass (another forward on the same context, a new cell or atoms), backward
first recomputes the wavefunctions by solving again at the saved positions
and cell, then takes the adjoint of that solve.
"""
import numpy as np
import torch


def _solve(ctx, pos, lattice, opts):
    if lattice is not None:
        ctx.set_cell(lattice)
    ctx.set_atoms(ctx.atom_species, pos)
    return ctx.scf(opts)


class ScfEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, positions, ctx, opts=None, lattice=None):
        pos = positions.detach().to("cpu", torch.float64).numpy().copy()
        lat = None if lattice is None else lattice.detach().to("cpu", torch.float64).numpy().copy()
        info = _solve(ctx, pos, lat, opts)
        energy, _ = ctx.energy()
        fctx.ctx, fctx.opts, fctx.pos, fctx.lat = ctx, opts, pos, lat
        fctx.generation = ctx.generation
        fctx.info = info
        fctx.recomputed = False
        fctx.lattice_device = None if lattice is None else lattice.device
        return torch.tensor(energy, dtype=torch.float64, device=positions.device)

    @staticmethod
    def backward(fctx, gE):
        ctx = fctx.ctx
        if ctx.generation != fctx.generation:
            # the held state is another solve's: recompute the wavefunctions
            _solve(ctx, fctx.pos, fctx.lat, fctx.opts)
            fctx.generation = ctx.generation
            fctx.recomputed = True
        g = float(gE)
        if fctx.lat is None:
            gpos = ctx.adjoint(g)  # g dE/dR = -g F
            return torch.from_numpy(np.ascontiguousarray(gpos)).to(gE.device), None, None, None
        gpos, glat = ctx.adjoint(g, lattice=True)
        return (torch.from_numpy(np.ascontiguousarray(gpos)).to(gE.device), None, None,
                torch.from_numpy(np.ascontiguousarray(glat)).to(fctx.lattice_device))


def scf_energy(positions, ctx, opts=None, lattice=None):
    return ScfEnergy.apply(positions, ctx, opts, lattice)
