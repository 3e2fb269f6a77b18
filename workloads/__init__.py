"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *describes* systems: lattices, atom positions, species
parameters, cutoffs, grids, band counts and occupation modes.  It contains
none of the plane-wave method's arithmetic, so the oracle and the GPU path
can both read it without sharing any part of the computation.

The shapes follow the workloads of the structure-search paper (Section 3.1:
bulk crystals, 2-D sheets and clusters, Table 1; population of candidates,
Section 2.4 last paragraph).  The species constants are project constants
(analytic pseudopotential forms), not fitted data.
"""
from .species import SPECIES
from .geometry import (diamond_cells, sheet_random, cluster_ball,
                       population_uneven, grid_rule, nbands_rule)
from .configs import (make_system, config_c1, config_c2, config_c3, config_c4,
                      config_c5, tiny_system, CONFIGS)

__all__ = ["SPECIES", "diamond_cells", "sheet_random", "cluster_ball",
           "population_uneven", "grid_rule", "nbands_rule", "make_system",
           "config_c1", "config_c2", "config_c3", "config_c4", "config_c5",
           "tiny_system", "CONFIGS"]
