"""Write the oracle's reference results for the workloads to tests/golden/.

Calls only the oracle (FP64 CPU) on the seeded inputs of `workloads`; no
value here comes from the HIP path.  Usage:
    python tests/golden/make_golden.py C1 [C2 C3 ...]
A name may end in ":cluster" to run the oracle's mixing with the weak Kerker
damping that suits a few atoms in a vacuum box (alpha 0.3, q0 0.3 bohr^-1,
up to 400 iterations); the fixed point is the same, only the path differs.
Each result is written to tests/golden/<name>.json with the total free
energy, its terms, eigenvalues, occupations and Hellmann-Feynman forces.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle.scf import run_scf  # noqa: E402
from oracle.forces import hf_forces  # noqa: E402


def golden(system, **kw):
    t0 = time.time()
    r = run_scf(system, **kw)
    F, parts = hf_forces(r)
    return {"name": system["name"], "energy": r["energy"], "terms": r["terms"],
            "eigenvalues": r["eigenvalues"].tolist(), "occupations": r["occupations"].tolist(),
            "mu": r["mu"], "forces": F.tolist(),
            "force_parts": {k: v.tolist() for k, v in parts.items()},
            "iterations": r["info"]["iterations"], "npw": int(r["setup"].npw),
            "trace": [list(t) for t in r["info"]["trace"]],
            "seconds": time.time() - t0, "system": system}


def main(names):
    for name in names:
        kw = {"tol_e": 1e-11, "tol_rho": 1e-9}
        if name.endswith(":cluster"):
            name = name[:-len(":cluster")]
            kw.update(mix_alpha=0.3, kerker_q0=0.3, maxiter=400)
        if name == "C1":
            systems = [workloads.config_c1()]
        elif name == "C2":
            systems = [workloads.config_c2()]
        elif name.startswith("C3-"):
            k = int(name[3:])
            systems = [workloads.config_c3(count=k + 1)[k]]
        elif name.startswith("C4-"):
            k = int(name[3:])
            systems = [workloads.config_c4(count=k + 1)[k]]
        elif name == "C5":
            systems = [workloads.config_c5()]
        else:
            raise SystemExit("unknown workload " + name)
        for s in systems:
            g = golden(s, **kw)
            path = os.path.join(HERE, s["name"] + ".json")
            with open(path, "w") as f:
                json.dump(g, f, indent=1)
            print("wrote", path, "E =", g["energy"], "in %.1f s" % g["seconds"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["C1"])
