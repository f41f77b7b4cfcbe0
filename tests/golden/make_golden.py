"""Write the stored oracle values used by the GPU parity tests at full size.

Calls only ``oracle/`` (and the shared seeded input generators in
``workloads``).  Run from the repository root:

    python tests/golden/make_golden.py [itps_d4_chi64] [itps_d6_chi144] [move_d6_chi144]

Outputs (JSON, one file per workload):
* itps_d4_chi64.json   2x2 cell, d=2, D=4, chi=64, N(0,1) tensors seed 1, randomized SVD
                       p=32, q=2, sketch seed 11; Heisenberg energy per site and per
                       bond after sweeps 1, 2, 5, 10, 20, 30; corner spectra after 30.
* itps_d6_chi144.json  2x2 cell, d=2, D=6, chi=144, seed 2, p=48, q=1, sketch seed 12;
                       energies after sweeps 1 and 2 (the oracle needs minutes per sweep).
* move_d6_chi144.json  the same D=6, chi=144 workload, one move in each direction from a
                       random full-dimension environment (seed 21): sampled entries of
                       every renormalised corner and edge.

The energy files also hold the same runs repeated with the site tensors
perturbed by 1e-13 (relative, three seeds): their spread is the run's own
sensitivity to rounding, the scale below which two correct FP64
implementations cannot be told apart.
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

CUTOFF = 1e-12
WORKLOADS = {
    "itps_d4_chi64": dict(D=4, chi=64, seed=1, p=32, q=2, sketch_seed=11, record=(1, 2, 5, 10, 20, 30)),
    "itps_d6_chi144": dict(D=6, chi=144, seed=2, p=48, q=1, sketch_seed=12, record=(1, 2)),
}
MOVES = {
    "move_d6_chi144": dict(D=6, chi=144, seed=2, p=48, q=1, sketch_seed=12, env_seed=21, samples=256),
}
PERTURB_SEEDS = (0, 1, 2)


def run_energies(name):
    w = WORKLOADS[name]
    A = wl.random_itps(2, 2, w["D"], 2, seed=w["seed"])
    H = wl.heisenberg_bond()
    out = dict(workload=name, params=w, cutoff=CUTOFF, energies={}, energies_perturbed=[], bonds={})
    t0 = time.time()
    runs = [("energies", A)]
    for ps in PERTURB_SEEDS:
        rng = np.random.default_rng(ps)
        runs.append(("perturbed %d" % ps, [a * (1 + 1e-13 * rng.standard_normal(a.shape)) for a in A]))
    for key, tensors in runs:
        env = Environment(tensors, 2, 2, chi=w["chi"], layers=2, mode="rsvd", oversample=w["p"],
                          power_iters=w["q"], seed=w["sketch_seed"], cutoff=CUTOFF)
        energies = {}
        for s in range(1, max(w["record"]) + 1):
            env.sweep()
            if s in w["record"]:
                energies[str(s)] = ob.energy_per_site(env, H)
                if key == "energies":
                    out["bonds"][str(s)] = [[ob.expect(ob.rho_bond(env, i, dr), H) for dr in (0, 1)]
                                            for i in range(4)]
                print(name, key, "sweep", s, energies[str(s)], "%.0fs" % (time.time() - t0), flush=True)
        if key == "energies":
            out["energies"] = energies
            out["spectra_last"] = env.corner_spectra().tolist()
            out["oracle_seconds"] = time.time() - t0
        else:
            out["energies_perturbed"].append(energies)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)


def run_moves(name):
    w = MOVES[name]
    D, chi = w["D"], w["chi"]
    A = wl.random_itps(2, 2, D, 2, seed=w["seed"])
    env0 = wl.random_environment(2, 2, chi, D * D, seed=w["env_seed"])
    out = dict(workload=name, params=w, cutoff=CUTOFF, moves={})
    t0 = time.time()
    for direction, r in (("left", 0), ("up", 1), ("right", 2), ("down", 3)):
        env = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=w["p"], power_iters=w["q"],
                          seed=w["sketch_seed"], cutoff=CUTOFF)
        for i, (C, T) in enumerate(env0):
            env.C[i] = [c.copy() for c in C]
            env.T[i] = [t.copy() for t in T]
        env.left_move(r)
        rng = np.random.default_rng(99)
        rec = {}
        for i in range(4):
            for kind, k in (("C", (0 + r) % 4), ("T", (3 + r) % 4), ("C", (3 + r) % 4)):
                x = env.C[i][k] if kind == "C" else env.T[i][k]
                pos = rng.integers(0, x.size, size=w["samples"])
                rec["%s%d_site%d" % (kind, k + 1, i)] = dict(shape=list(x.shape), pos=pos.tolist(),
                                                             val=x.reshape(-1)[pos].tolist(),
                                                             fro=float(np.linalg.norm(x)))
        out["moves"][direction] = rec
        print(name, direction, "%.0fs" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS) + list(MOVES)):
        (run_energies if name in WORKLOADS else run_moves)(name)
