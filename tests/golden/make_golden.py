"""Write the stored oracle values used by the GPU parity tests at full size.

Calls only ``oracle/`` (and the shared seeded input generators in
``workloads``).  Run from the repository root:

    python tests/golden/make_golden.py [itps_d4_chi64] [itps_d6_chi144]

Outputs (JSON, one file per workload):
* itps_d4_chi64.json   2x2 cell, d=2, D=4, chi=64, N(0,1) tensors seed 1, randomized SVD
                       p=32, q=2, sketch seed 11; Heisenberg energy per site and per
                       bond after sweeps 1, 2, 5, 10, 20, 30; corner spectra after 30.
* itps_d6_chi144.json  2x2 cell, d=2, D=6, chi=144, seed 2, p=48, q=1, sketch seed 12;
                       energies after sweeps 1 and 2 (the oracle needs minutes per sweep).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.ctmrg import Environment  # noqa: E402

WORKLOADS = {
    "itps_d4_chi64": dict(D=4, chi=64, seed=1, p=32, q=2, sketch_seed=11, record=(1, 2, 5, 10, 20, 30)),
    "itps_d6_chi144": dict(D=6, chi=144, seed=2, p=48, q=1, sketch_seed=12, record=(1, 2)),
}


def run(name):
    """Oracle energies, and the same run with inputs perturbed by 1e-13 (relative):
    their difference is the run's own sensitivity to rounding, the scale below
    which two correct FP64 implementations cannot be told apart."""
    w = WORKLOADS[name]
    A = wl.random_itps(2, 2, w["D"], 2, seed=w["seed"])
    rng = np.random.default_rng(0)
    Ap = [a * (1 + 1e-13 * rng.standard_normal(a.shape)) for a in A]
    H = wl.heisenberg_bond()
    out = dict(workload=name, params=w, cutoff=1e-12, energies={}, energies_perturbed={}, bonds={})
    t0 = time.time()
    for key, tensors in (("energies", A), ("energies_perturbed", Ap)):
        env = Environment(tensors, 2, 2, chi=w["chi"], layers=2, mode="rsvd", oversample=w["p"],
                          power_iters=w["q"], seed=w["sketch_seed"], cutoff=1e-12)
        for s in range(1, max(w["record"]) + 1):
            env.sweep()
            if s in w["record"]:
                out[key][str(s)] = ob.energy_per_site(env, H)
                if key == "energies":
                    out["bonds"][str(s)] = [[ob.expect(ob.rho_bond(env, i, dr), H) for dr in (0, 1)]
                                            for i in range(4)]
                print(name, key, "sweep", s, out[key][str(s)], "%.0fs" % (time.time() - t0), flush=True)
        if key == "energies":
            out["spectra_last"] = env.corner_spectra().tolist()
            out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        run(name)
