"""Fixed-basis stress (oracle): sigma_ab = (1/Omega) dF/d eps_ab at a fixed set
of Miller indices.  Filled in with the strain derivatives of each energy
term; see the function docstring."""
