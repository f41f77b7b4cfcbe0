"""Write the stored oracle values used by the GPU parity tests.

Calls only ``oracle/`` (and the shared seeded input generators in
``workloads``).  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Outputs (JSON, one file per workload):
* itps_d4_chi64.json    2x2 cell, d=2, D=4, chi=64, N(0,1) tensors seed 1, randomized SVD
                        p=32, q=2, sketch seed 11, from the trivial boundary: Heisenberg
                        energy per site (and per bond) after sweeps 1, 2, 5, 10, 20, 30;
                        corner spectra after 30.
* itps_d6_chi144.json   2x2 cell, d=2, D=6, chi=144, seed 2, p=48, q=1, sketch seed 12,
                        from the trivial boundary: energies after sweeps 1, 2, 5, 10, 20, 30.
* restart_d4_chi64.json the D=4, chi=64 workload started from a random full-dimension
                        environment (seed 21): energies after each of 3 sweeps.
* tfim_converged.json   transverse-field Ising requests (mean-field state plus 0.1 N(0,1)
                        noise) at D = 2 and 3, 1x1 and 2x2 cells: energy per site and
                        <sigma_z> per site after 40 sweeps, where the energy has settled
                        to about 1e-13.
* ising_peps_2x2.json   the Ising PEPS (beta = 0.5) on a 2x2 cell with random bond
                        gauges, run to delta < 1e-11: <sigma_z sigma_z> on every bond.
* move_d6_chi144.json   the D=6, chi=144 workload, one move in each direction from a
                        random full-dimension environment (seed 21): sampled entries of
                        every renormalised corner and edge.

The energy files also hold the same runs repeated with every entry of the
site tensors moved by one unit in the last place (up or down at random, one
run per perturbation seed): their spread is the run's own sensitivity to
rounding at the level of unit roundoff, the scale below which two correct
FP64 implementations cannot be told apart.
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
from tests._util import ulp_perturbed  # noqa: E402
from oracle.ctmrg import Environment  # noqa: E402

CUTOFF = 1e-12
WORKLOADS = {
    "itps_d4_chi64": dict(D=4, chi=64, seed=1, p=32, q=2, sketch_seed=11, record=(1, 2, 5, 10, 20, 30),
                          perturb=(0, 1, 2, 3)),
    "itps_d6_chi144": dict(D=6, chi=144, seed=2, p=48, q=1, sketch_seed=12, record=(1, 2, 5, 10, 20, 30),
                           perturb=(0,)),
    "restart_d4_chi64": dict(D=4, chi=64, seed=1, p=32, q=2, sketch_seed=11, record=(1, 2, 3), env_seed=21,
                             perturb=(0, 1, 2)),
}
MOVES = {
    "move_d6_chi144": dict(D=6, chi=144, seed=2, p=48, q=1, sketch_seed=12, env_seed=21, samples=256),
}
TFIM = dict(p=16, q=1, sketch_seed=9, eps=0.1, sweeps=40, record=(20, 30, 40),
            cases=[dict(L=1, D=2, chi=16, h=2.9), dict(L=2, D=2, chi=20, h=3.1), dict(L=1, D=3, chi=24, h=2.7),
                   dict(L=2, D=3, chi=30, h=3.3)])


def run_energies(name):
    w = WORKLOADS[name]
    A = wl.random_itps(2, 2, w["D"], 2, seed=w["seed"])
    H = wl.heisenberg_bond()
    out = dict(workload=name, params=w, cutoff=CUTOFF, perturbation="1 ulp per entry of the site tensors",
               energies={}, energies_perturbed=[], bonds={})
    t0 = time.time()
    runs = [("energies", A)] + [("perturbed %d" % ps, ulp_perturbed(A, ps)) for ps in w["perturb"]]
    for key, tensors in runs:
        env = Environment(tensors, 2, 2, chi=w["chi"], layers=2, mode="rsvd", oversample=w["p"],
                          power_iters=w["q"], seed=w["sketch_seed"], cutoff=CUTOFF)
        if "env_seed" in w:
            for i, (C, T) in enumerate(wl.random_environment(2, 2, w["chi"], w["D"] ** 2, seed=w["env_seed"])):
                env.C[i] = [c.copy() for c in C]
                env.T[i] = [t.copy() for t in T]
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


def run_tfim():
    w = TFIM
    out = dict(workload="tfim_converged", params={k: v for k, v in w.items() if k != "cases"}, cutoff=CUTOFF,
               cases=[])
    t0 = time.time()
    for case in w["cases"]:
        L, D, chi, h = case["L"], case["D"], case["chi"], case["h"]
        A = wl.tfim_request_tensors(h, D, L, L, w["eps"], seed=17 + D + L)
        env = Environment(A, L, L, chi=chi, layers=2, mode="rsvd", oversample=w["p"], power_iters=w["q"],
                          seed=w["sketch_seed"], cutoff=CUTOFF)
        rec = dict(case, tensor_seed=17 + D + L, energies={})
        prev = env.corner_spectra()
        for s in range(1, w["sweeps"] + 1):
            env.sweep()
            cur = env.corner_spectra()
            delta = float(np.max(np.sum(np.abs(cur - prev), axis=1)))
            prev = cur
            if s in w["record"]:
                rec["energies"][str(s)] = ob.energy_per_site(env, wl.tfim_bond(h))
        rec["delta_last"] = delta
        rec["mz"] = [ob.expect(ob.rho_one_site(env, i), wl.SZ) for i in range(L * L)]
        out["cases"].append(rec)
        print("tfim", case, rec["energies"], "delta %.1e" % delta, "%.0fs" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "tfim_converged.json"), "w") as f:
        json.dump(out, f)


def run_ising_peps():
    beta = 0.5
    A, _ = wl.ising_peps(beta)
    tensors = wl.gauged_2x2(A, 2, seed=7)
    env = Environment(tensors, 2, 2, chi=16, layers=2, mode="rsvd", oversample=16, power_iters=2, seed=2,
                      cutoff=CUTOFF)
    n, delta, conv = env.run(400, 1e-11)
    zz = np.kron(wl.SZ, wl.SZ)
    out = dict(workload="ising_peps_2x2", beta=beta, gauge_seed=7, chi=16, p=16, q=2, sketch_seed=2, tol=1e-11,
               sweeps=n, delta=delta, converged=bool(conv),
               zz=[[ob.expect(ob.rho_bond(env, i, dr), zz) for dr in (0, 1)] for i in range(4)])
    print("ising_peps_2x2", n, delta, out["zz"], flush=True)
    with open(os.path.join(HERE, "ising_peps_2x2.json"), "w") as f:
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
    names = sys.argv[1:] or list(WORKLOADS) + list(MOVES) + ["tfim_converged", "ising_peps_2x2"]
    for name in names:
        if name in WORKLOADS:
            run_energies(name)
        elif name in MOVES:
            run_moves(name)
        elif name == "tfim_converged":
            run_tfim()
        elif name == "ising_peps_2x2":
            run_ising_peps()
        else:
            raise SystemExit("unknown workload " + name)
