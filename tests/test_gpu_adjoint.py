"""The energy as a torch.autograd.Function: its backward (the library's
Hellmann-Feynman adjoint) against central finite differences of the same
energy (h = 1e-3 bohr) and against the oracle's forces."""
import copy

import numpy as np
import pytest

from tests.gpu_helpers import say, load_golden
import workloads

pytestmark = pytest.mark.gpu


def _sheet_small():
    lat, pos = workloads.sheet_random(8, 8.0, 8.0, 10.0, 2.4, 21)
    return workloads.make_system("sheet8", lat, ["C-G"] * 8, pos, 8.0, (24, 24, 30), 20,
                                 {"kind": "fermi", "sigma": 0.01}, "fp64")


def test_autograd_matches_finite_differences_fp64():
    import torch
    import paper_1603_02732_amd as sgo
    from paper_1603_02732_amd.autograd import ScfEnergy
    s = _sheet_small()
    ctx = sgo.context_from_system(s, sgo.SGO_FP64)
    opts = sgo.default_opts(tol_e=1e-12, tol_rho=1e-9, max_iter=300)
    R = torch.tensor(np.array(s["positions"]), dtype=torch.float64, requires_grad=True)
    E = ScfEnergy.apply(R, ctx, opts)
    (g,) = torch.autograd.grad(2.5 * E, R)
    h = 1e-3
    for I, a in [(0, 0), (3, 1), (5, 2), (7, 0)]:
        e = []
        for sg in (1, -1):
            Rp = R.detach().clone()
            Rp[I, a] += sg * h
            e.append(float(ScfEnergy.apply(Rp, ctx, opts)))
        fd = 2.5 * (e[0] - e[1]) / (2 * h)
        say("atom %d axis %d: autograd %.8f  FD %.8f" % (I, a, float(g[I, a]), fd))
        assert abs(float(g[I, a]) - fd) < 1e-5


def test_backward_recomputes_a_state_the_context_no_longer_holds():
    """Two forward passes on one context, then the backward of the first:
    its solve is no longer held, so backward solves again at the saved
    positions before the adjoint; both gradients equal -F of fresh contexts
    solved at the same positions, and a backward whose state is still held
    takes the adjoint directly."""
    import torch
    import paper_1603_02732_amd as sgo
    from paper_1603_02732_amd.autograd import ScfEnergy
    s = _sheet_small()
    ctx = sgo.context_from_system(s, sgo.SGO_FP64)
    opts = sgo.default_opts(tol_e=1e-12, tol_rho=1e-9, max_iter=300)
    P1 = np.array(s["positions"])
    P2 = P1.copy()
    P2[2, 0] += 0.05
    R1 = torch.tensor(P1, dtype=torch.float64, requires_grad=True)
    R2 = torch.tensor(P2, dtype=torch.float64, requires_grad=True)
    E1 = ScfEnergy.apply(R1, ctx, opts)
    E2 = ScfEnergy.apply(R2, ctx, opts)
    (g1,) = torch.autograd.grad(E1, R1)
    assert E1.grad_fn.recomputed
    (g2,) = torch.autograd.grad(E2, R2)
    assert E2.grad_fn.recomputed  # the first backward's solve replaced it
    for P, g in ((P1, g1), (P2, g2)):
        t = dict(s)
        t["positions"] = P.tolist()
        f = sgo.context_from_system(t, sgo.SGO_FP64)
        f.scf(opts)
        dF = np.abs(g.numpy() + f.forces()).max()
        say("  recomputed backward vs fresh solve: max dF %.2e" % dF)
        assert dF < 1e-6
    E3 = ScfEnergy.apply(R2, ctx, opts)
    (g3,) = torch.autograd.grad(E3, R2)
    assert not E3.grad_fn.recomputed
    assert np.abs(g3.numpy() - g2.numpy()).max() < 1e-6


def test_autograd_fp32_sheet_matches_oracle_forces():
    import torch
    import paper_1603_02732_amd as sgo
    from paper_1603_02732_amd.autograd import ScfEnergy
    s = workloads.config_c2()
    ref = load_golden("C2", s)
    if ref is None:
        pytest.skip("C2 oracle reference not generated")
    ctx = sgo.context_from_system(s, sgo.SGO_FP32)
    opts = sgo.default_opts(tol_e=1e-8, tol_rho=1e-6, max_iter=200)
    R = torch.tensor(np.array(s["positions"]), dtype=torch.float64, requires_grad=True)
    E = ScfEnergy.apply(R, ctx, opts)
    E.backward()
    dF = np.abs(-R.grad.numpy() - np.array(ref["forces"])).max()
    say("C2 fp32 adjoint vs oracle forces: max dF %.2e, dE/atom %.2e"
        % (dF, abs(float(E) - ref["energy"]) / 24))
    assert dF < 5e-4
    assert abs(float(E) - ref["energy"]) / 24 < 1e-5


def test_autograd_lattice_gradient_matches_finite_differences():
    """dE/dA from the stress (Cartesian positions fixed) against central
    differences of the GPU energy over the cell; the step is small enough
    that no plane wave crosses the cutoff sphere (checked), so the basis of
    the strained cells is the fixed one the gradient refers to."""
    import torch
    import paper_1603_02732_amd as sgo
    from paper_1603_02732_amd.autograd import ScfEnergy
    s = workloads.tiny_system("sip", grid=(12, 12, 15))
    ctx = sgo.context_from_system(s, sgo.SGO_FP64)
    opts = sgo.default_opts(tol_e=1e-12, tol_rho=1e-10, max_iter=300)
    R = torch.tensor(np.array(s["positions"]), dtype=torch.float64, requires_grad=True)
    A = torch.tensor(np.array(s["lattice"]), dtype=torch.float64, requires_grad=True)
    E = ScfEnergy.apply(R, ctx, opts, A)
    gR, gA = torch.autograd.grad(1.5 * E, (R, A))
    npw0 = len(ctx.basis()[0])
    assert torch.allclose(gR, -1.5 * torch.from_numpy(ctx.forces()))
    h = 1e-4
    for (i, j) in [(0, 0), (0, 2), (2, 1)]:
        e = []
        for sg in (1, -1):
            Ap = A.detach().clone()
            Ap[i, j] += sg * h
            e.append(float(ScfEnergy.apply(R.detach(), ctx, opts, Ap)))
            assert len(ctx.basis()[0]) == npw0
        fd = 1.5 * (e[0] - e[1]) / (2 * h)
        say("dE/dA[%d,%d]: autograd %.9f  FD %.9f" % (i, j, float(gA[i, j]), fd))
        assert abs(float(gA[i, j]) - fd) < 2e-6
