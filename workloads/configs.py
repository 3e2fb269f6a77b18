"""The five synthetic workloads, fully explicit.

A *system* is a plain dict (JSON-serialisable):
    name, lattice (3x3 rows, bohr), species {name: params}, symbols [..],
    positions [[x,y,z], ..] (bohr), ecut (Ha), grid [N1,N2,N3], nbands,
    occupation {"kind": "fixed"} | {"kind": "fermi", "sigma": s},
    nelec, precision ("fp64" | "fp32").

Readings of underdetermined workload descriptions are recorded in "notes".
"""
import copy
import numpy as np

from .species import SPECIES
from .geometry import (diamond_cells, sheet_random, cluster_ball,
                       population_uneven, grid_rule, nbands_rule)


def make_system(name, lattice, symbols, positions, ecut, grid, nbands,
                occupation, precision="fp64", notes=""):
    lattice = np.asarray(lattice, dtype=float)
    positions = np.asarray(positions, dtype=float)
    used = sorted(set(symbols))
    species = {s: copy.deepcopy(SPECIES[s]) for s in used}
    nelec = float(sum(species[s]["Z"] for s in symbols))
    return {"name": name, "lattice": lattice.tolist(), "species": species,
            "symbols": list(symbols), "positions": positions.tolist(),
            "ecut": float(ecut), "grid": [int(g) for g in grid],
            "nbands": int(nbands), "occupation": dict(occupation),
            "nelec": nelec, "precision": precision, "notes": notes}


FIXED = {"kind": "fixed"}
FERMI = {"kind": "fermi", "sigma": 0.01}


def config_c1(seed=1, jitter=0.1):
    """Si8 diamond, a = 10.26 bohr, +-0.1 bohr seeded jitter; Ecut 8 Ha, 24^3,
    20 bands (32 electrons need 16 doubly occupied bands; 12 cannot hold them),
    Appelbaum-Hamann local potential, fixed occupations, FP64."""
    lat, pos = diamond_cells(10.26, (1, 1, 1), jitter, seed)
    return make_system("C1", lat, ["Si-AH"] * 8, pos, 8.0, (24, 24, 24), 20,
                       FIXED, "fp64", "nb=20 (16 occupied + 4)")


def config_c2(seed=2):
    """24-atom carbon sheet, 14 x 12.1 bohr in plane, c = 15 bohr, sheet at
    z = c/2; Gaussian local only; Ecut 15, 48x40x48, 56 bands, Fermi-Dirac
    sigma = 0.01 Ha, FP32 bulk."""
    lat, pos = sheet_random(24, 14.0, 12.1, 15.0, 2.4, seed)
    return make_system("C2", lat, ["C-Gloc"] * 24, pos, 15.0, (48, 40, 48), 56,
                       FERMI, "fp32", "c = 15 bohr; hard-disk MC sheet")


def config_c3(count=32, seed0=100):
    """Population of 13-atom clusters in a 24-bohr cubic box, uniform in a
    radius-5 ball, dmin 3.5; Gaussian local + s KB; Ecut 10, 48^3, 32 bands."""
    out = []
    for k in range(count):
        lat, pos = cluster_ball(13, 24.0, 5.0, 3.5, seed0 + k)
        out.append(make_system("C3-%d" % k, lat, ["C-G"] * 13, pos, 10.0,
                               (48, 48, 48), 32, FERMI, "fp32"))
    return out


def config_c4(count=64, seed0=200, ecut=15.0):
    """Uneven population of 8-40 carbon atoms in 12-22 bohr cells; grid by
    the 2^a3^b5^c rule at h <= 0.375 bohr; bands = even ceil(1.4 x occupied)
    (the random clusters carry many dangling-bond states near the Fermi
    level: with 1.2 x occupied the top band of several candidates still holds
    charge at self-consistency, and their SCF stalls)."""
    out = []
    for k, (lat, pos) in enumerate(population_uneven(count, seed0)):
        n = len(pos)
        grid = [grid_rule(lat[i, i]) for i in range(3)]
        nb = nbands_rule(2 * n, 1.4)  # 4 electrons per atom -> 2n occupied bands
        out.append(make_system("C4-%d" % k, lat, ["C-G"] * n, pos, ecut, grid,
                               nb, FERMI, "fp32"))
    return out


def config_c5(seed=5, stretch=False):
    """128-atom Si supercell of 4x2x2 conventional cells (a = 10.26 bohr,
    +-0.15 jitter), Ecut 20, 108x54x54, 282 bands, Gaussian s+p KB; the
    literal 4x4x2 box (256 atoms, 108x108x54, 564 bands) is the stretch."""
    if stretch:
        lat, pos = diamond_cells(10.26, (4, 4, 2), 0.15, seed)
        return make_system("C5s", lat, ["Si-G"] * len(pos), pos, 20.0,
                           (108, 108, 54), 564, FIXED, "fp32")
    lat, pos = diamond_cells(10.26, (4, 2, 2), 0.15, seed)
    return make_system("C5", lat, ["Si-G"] * len(pos), pos, 20.0, (108, 54, 54),
                       282, FIXED, "fp32", "128 atoms = 4x2x2 cells")


def tiny_system(kind="si", ecut=3.0, grid=(12, 12, 12), nbands=None, seed=11,
                jitter=0.1, occupation=None):
    """Small variants of the workloads that a dense FP64 diagonalisation
    handles in well under a second per SCF iteration."""
    if kind == "si":
        lat, pos = diamond_cells(10.26, (1, 1, 1), jitter, seed)
        return make_system("tiny-si", lat, ["Si-AH"] * 8, pos, ecut, grid,
                           nbands or 20, occupation or FIXED, "fp64")
    if kind == "c":
        lat, pos = cluster_ball(4, 10.0, 2.0, 2.4, seed)
        return make_system("tiny-c", lat, ["C-G"] * 4, pos, ecut, grid,
                           nbands or 10, occupation or FERMI, "fp64")
    if kind == "sip":
        lat, pos = diamond_cells(10.26, (1, 1, 1), jitter, seed)
        return make_system("tiny-sip", lat, ["Si-G"] * 8, pos, ecut, grid,
                           nbands or 20, occupation or FERMI, "fp64")
    raise ValueError(kind)


CONFIGS = {"C1": config_c1, "C2": config_c2, "C3": config_c3, "C4": config_c4,
           "C5": config_c5}
