"""Species parameter sets (Hartree atomic units).

local.kind == "ah":    v(r) = -(Z/r) erf(sqrt(alpha) r) + (v1 + v2 r^2) exp(-alpha r^2)
local.kind == "gauss": v(r) = -(Z/r) erf(r/(sqrt(2) rloc))
                              + exp(-r^2/(2 rloc^2)) [c1 + c2 (r/rloc)^2]
kb: list of Kleinman-Bylander channels {l, r, h}; the radial projector is a
normalised Gaussian r^l exp(-r^2/(2 r_l^2)) and h is the channel energy.
rho0_width: width (bohr) of the normalised Gaussian of charge Z used as the
starting density around each atom (same definition on both sides).

The numbers are project constants shaped after published analytic
pseudopotentials; they are inputs, and parity never depends on their values.
"""

SPECIES = {
    # Appelbaum-Hamann-form local potential for Si (bulk crystal workload).
    "Si-AH": {"Z": 4.0,
              "local": {"kind": "ah", "alpha": 0.6102, "v1": 3.042, "v2": -1.372},
              "kb": [],
              "rho0_width": 0.9052},
    # Carbon-like Gaussian-form local + one s-channel KB projector.
    "C-G": {"Z": 4.0,
            "local": {"kind": "gauss", "rloc": 0.338, "c1": -8.80, "c2": 1.34},
            "kb": [{"l": 0, "r": 0.303, "h": 9.62}],
            "rho0_width": 0.338},
    # Same local part with no projector (sheet workload uses local only).
    "C-Gloc": {"Z": 4.0,
               "local": {"kind": "gauss", "rloc": 0.338, "c1": -8.80, "c2": 1.34},
               "kb": [],
               "rho0_width": 0.338},
    # Silicon-like Gaussian-form local + s and p KB projectors (large cell).
    "Si-G": {"Z": 4.0,
             "local": {"kind": "gauss", "rloc": 0.44, "c1": -7.34, "c2": 0.0},
             "kb": [{"l": 0, "r": 0.423, "h": 5.91},
                    {"l": 1, "r": 0.484, "h": 2.73}],
             "rho0_width": 0.44},
}
