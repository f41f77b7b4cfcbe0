"""Benchmark: CTMRG sweeps per second on one MI355X.

Workload (one "step" = one CTMRG sweep = left, right, up and down moves over
the whole unit cell): iTPS on a 2x2 unit cell, physical dimension 2, bond
dimension D = 6, environment dimension chi = 144, real site tensors with
seeded N(0, 1) entries divided by their max-abs entry; projectors from the
randomized SVD with oversampling p = 48 and q = 1 power iteration.

Prints one JSON line.  `roofline` is for the dominant phase (the sketch
GEMMs: products of an n x n enlarged corner with n x k panels), timed live
with HIP events on the library's stream over the timed sweeps.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload (one left move on a random full-dimension environment) and scales
it to sweeps per second.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402

PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "f16split": 2.5e15}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "sketch_gemm_d6_chi144_traffic.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2112_13184_amd", "csrc", "gemm.hip")


def counted_traffic():
    """HBM bytes per sketch-GEMM launch (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy of known size) from the committed counter summary, or None when
    the summary is missing or was taken on another version of the GEMM source."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    return rec["hbm_bytes_per_launch"] if rec.get("gemm_source_sha256") == src else None
METRIC = "CTMRG sweeps/s + MFMA util at D=6 chi=144; solves/s and p99 latency"


def flops_per_sweep(D, chi, d, p, q, Lx=2, Ly=2):
    """Algorithmic flops of one sweep (single-layer contractions, randomized SVD)."""
    Db = D * D
    n = chi * Db
    k = min(chi + p, n)
    ncut = 4 * Lx * Ly
    corner = chi ** 3 * Db + chi ** 3 * Db * Db + 2 * chi ** 2 * Db * Db * D * D * d
    sketch = (10 + 8 * q) * n * n * k
    renorm = 2 * chi ** 3 * Db * Db + 2 * chi ** 2 * Db * Db * D * D * d
    return 2.0 * (4 * ncut * corner + ncut * sketch + ncut * renorm)


def oracle_threads():
    """Threads for the oracle: the job's CPU share (OMP_NUM_THREADS where the
    host sets it), else every core."""
    env = os.environ.get("OMP_NUM_THREADS")
    return max(1, int(env)) if env and env.isdigit() else (os.cpu_count() or 1)


def cpu_baseline(D, chi, p, q, seed):
    """Oracle time for one left move (a quarter sweep) of the headline
    workload on a random full-dimension environment."""
    from threadpoolctl import threadpool_limits

    from oracle.ctmrg import Environment
    cores = oracle_threads()
    A = wl.random_itps(2, 2, D, 2, seed=seed)
    env = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=p, power_iters=q, seed=7)
    rng = np.random.default_rng(3)
    for i in range(4):
        env.C[i] = [rng.standard_normal((chi, chi)) for _ in range(4)]
        env.T[i] = [rng.standard_normal((chi, chi, D * D)) for _ in range(4)]
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        env.left_move(0)
        dt = time.perf_counter() - t0
    return dict(value=1.0 / (4.0 * dt), unit="sweeps/s", cores=cores, host_cpu_count=os.cpu_count(),
                kind="oracle",
                sample=f"one left move (1/4 sweep) of the 2x2 D={D} chi={chi} workload on a random "
                       f"full-dimension environment, NumPy/OpenBLAS FP64 on {cores} threads, {dt:.1f} s; scaled x4")


def cpu_baseline_extra(serving_res, serving_reqs, rate_hz, n_sample=6):
    """The rest of the CPU baseline on the same host threads: oracle sweeps/s
    of the D=4, chi=64 workload (randomized SVD p=32, q=2, and the exact SVD),
    one sweep each from the trivial boundary; and the serving stream processed
    FIFO one solve at a time, estimated from a sample of requests (one oracle
    sweep each, times the sweeps that request takes to converge), replayed on
    the same arrival trace for p50 / p99."""
    from threadpoolctl import threadpool_limits

    from oracle.ctmrg import Environment
    cores = oracle_threads()
    out = {"cores": cores, "host_cpu_count": os.cpu_count(), "kind": "oracle"}
    A = wl.random_itps(2, 2, 4, 2, seed=1)
    with threadpool_limits(limits=cores):
        for mode in ("rsvd", "dense"):
            env = Environment(A, 2, 2, chi=64, layers=2, mode=mode, oversample=32, power_iters=2, seed=11)
            env.sweep()   # the first sweep grows the environment; time the second
            t0 = time.perf_counter()
            env.sweep()
            out[f"d4_chi64_{mode}_sweeps_per_s"] = 1.0 / (time.perf_counter() - t0)
        if serving_res is not None:
            rng = np.random.default_rng(0)
            idx = sorted(rng.choice(len(serving_reqs), size=min(n_sample, len(serving_reqs)), replace=False))
            per_sweep = []
            for i in idx:
                r = serving_reqs[i]
                env = Environment(r["A"], r["Lx"], r["Ly"], chi=r["chi"], layers=2, mode="rsvd", oversample=16,
                                  power_iters=1, seed=3)
                env.sweep()
                t0 = time.perf_counter()
                env.sweep()
                per_sweep.append(time.perf_counter() - t0)
            # service time of every request: a sweep costs about c L^2 n^2 k
            # (4 L^2 cuts, sketch products of n x n corners with n x k
            # panels, n = chi D^2, k = chi + 16), c the median over the sample,
            # times the sweeps the request takes
            work = lambda r: r["Lx"] ** 2 * float(r["chi"] * r["D"] ** 2) ** 2 * (r["chi"] + 16)
            c_med = float(np.median([t / work(serving_reqs[i]) for t, i in zip(per_sweep, idx)]))
            svc = [c_med * work(r) * max(res["sweeps"], 1) for r, res in zip(serving_reqs, serving_res)]
            t, lat = 0.0, []
            for r, s in zip(serving_reqs, svc):
                t = max(t, r["arrival"]) + s
                lat.append(t - r["arrival"])
            out["serving_fifo_estimate"] = {
                "requests": len(serving_reqs), "sampled": [int(i) for i in idx],
                "sampled_sweep_s": per_sweep, "solves_per_s": len(svc) / sum(svc),
                "arrival_rate_hz": rate_hz, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "model": "service time = c L^2 (chi D^2)^2 (chi + 16) x the request's sweep count on the GPU "
                         "run, c the median over the sampled oracle sweeps; FIFO on the open-loop arrival trace"}
    return out


def run_sweeps(lib, A, D, chi, d, p, q, prec, warmup, steps, timing=2, seed=12):
    """warmup untimed sweeps, then `steps` timed sweeps through ctm_sweep
    (the four moves and the stop rule's corner spectra of every sweep);
    returns (seconds, phase timings, energy per site after warmup + steps
    sweeps, cut counts).  timing 2 records HIP events around the sketch
    products only (one pair per four products), 1 around every phase (its
    events add about 10 us of idle stream per pair, so that pass is for the
    phase breakdown, not for the rate)."""
    import torch
    ctx = lib.Ctm(A, 2, 2, D, chi, d=d, prec=prec, rsvd_oversample=p, rsvd_power_iters=q, seed=seed)
    if warmup:
        ctx.ctm_sweep(warmup, 0.0)
    torch.cuda.synchronize()
    ctx.ctm_timing_enable(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, _, _ = ctx.ctm_sweep(steps, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert n == steps
    phases = ctx.ctm_timing_read()
    ctx.ctm_timing_enable(False)
    H = wl.heisenberg_bond()
    energy = sum(ctx.ctm_expect_2site(i, dr, H) for i in range(4) for dr in (0, 1)) / 4
    cuts = ctx.ctm_cut_stats()
    del ctx
    return dt, phases, energy, cuts


def sketch_rate(phases):
    sk = phases["sketch_gemm"]
    return sk["flops"] / (sk["ms"] * 1e-3) if sk["ms"] > 0 else 0.0


def copy_calibration():
    """Plain device-to-device copies of a known size (1 GiB, 5 times), for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    x.uniform_()
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": x.numel() * 8, "launches": 5}))


def serving_requests(n, seed=4, rate_hz=None):
    out = []
    for r in wl.serving_stream(n=n, seed=seed, rate_hz=rate_hz, eps=0.1):
        A = wl.tfim_request_tensors(r["h"], r["D"], r["Lx"], r["Ly"], 0.1, r["tensor_seed"])
        out.append(dict(r, A=A, op=wl.tfim_bond(r["h"])))
    return out


def scan_requests(n, D=3, chi=32, L=2, seed=5):
    """A transverse-field scan at one shape: h evenly over [2.5, 3.5]."""
    out = []
    for i in range(n):
        h = 2.5 + i / max(n - 1, 1)
        A = wl.tfim_request_tensors(h, D, L, L, 0.1, seed * 1000 + i)
        out.append(dict(index=i, h=h, D=D, chi=chi, Lx=L, Ly=L, arrival=0.0, A=A, op=wl.tfim_bond(h)))
    return out


def scan_bench(lib, n, max_active, budget_gb, p=16, q=1, tol=1e-10, max_sweeps=40):
    """Closed-loop throughput of a one-shape scan, grouped (same-shape requests
    share a context and its launches) and with one request per admission."""
    out = {"requests": n, "shape": "2x2 D=3 chi=32", "max_active": max_active}
    for label, mx in (("grouped", max_active), ("one_per_admission", None)):
        qu = lib.Queue(int(budget_gb * (1 << 30)), max_active)
        reqs = scan_requests(n)
        t0 = time.perf_counter()
        res = []
        if mx is None:   # submit the next request only when a slot is free: no grouping possible
            pending = list(reqs)
            inflight = []
            while pending or inflight:
                while pending and len(inflight) < max_active:
                    r = pending.pop(0)
                    inflight.append(qu.submit(r["A"], 2, 2, r["D"], r["chi"], r["op"], tol=tol, max_sweeps=max_sweeps,
                                              rsvd_oversample=p, rsvd_power_iters=q, seed=3)[1])
                st, rr = qu.wait(inflight.pop(0), -1)
                res.append(rr)
        else:
            tickets = [qu.submit(r["A"], 2, 2, r["D"], r["chi"], r["op"], tol=tol, max_sweeps=max_sweeps,
                                 rsvd_oversample=p, rsvd_power_iters=q, seed=3)[1] for r in reqs]
            res = [qu.wait(t, -1)[1] for t in tickets]
        dt = time.perf_counter() - t0
        qu.destroy()
        out[label] = {"solves_per_s": n / dt, "energies": [float(r.energy_per_site) for r in res]}
        print(f"scan ({label}): {n} done, {dt:.1f} s", file=sys.stderr, flush=True)
    diff = max(abs(a - b) for a, b in zip(out["grouped"].pop("energies"), out["one_per_admission"].pop("energies")))
    out["max_energy_diff_grouped_vs_single"] = diff
    return out


def serving_bench(lib, n, max_active, budget_gb, p=16, q=1, tol=1e-10, max_sweeps=40, loads=(0.8,)):
    """The mixed TFIM stream through the serving queue: a closed loop (all
    requests at t = 0) gives the capacity; open loops replay Poisson arrivals
    at the given fractions of that capacity for p50 / p99 latency (arrival to
    done).  Every request also measures <sigma_z> on each site."""
    budget = int(budget_gb * (1 << 30))

    def run(reqs, label):
        qu = lib.Queue(budget, max_active)
        tickets = []
        t0 = time.perf_counter()
        timed = label != "closed"
        for r in reqs:
            if timed:
                dt = r["arrival"] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            st, t = qu.submit(r["A"], r["Lx"], r["Ly"], r["D"], r["chi"], r["op"], tol=tol,
                              max_sweeps=max_sweeps, tag=r["index"], rsvd_oversample=p, rsvd_power_iters=q,
                              seed=3, obs=[wl.SZ])
            if st != 0:
                raise RuntimeError(f"submit failed with status {st}")
            tickets.append(t)
        res = []
        for i, t in enumerate(tickets):
            st, r = qu.wait(t, -1)
            if st != 0:
                raise RuntimeError(f"request failed with status {st}")
            res.append(r)
            if (i + 1) % 64 == 0 or i + 1 == len(tickets):
                print(f"serving ({label}): {i + 1}/{len(tickets)} done, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        qu.destroy()
        first = min(r.t_submit_ns for r in res)
        last = max(r.t_done_ns for r in res)
        lat = np.array([(r.t_done_ns - r.t_submit_ns) * 1e-6 for r in res])
        conv = int(sum(r.converged for r in res))
        return dict(solves_per_s=len(res) / ((last - first) * 1e-9), p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), mean_sweeps=float(np.mean([r.sweeps for r in res])),
                    converged=conv, converged_fraction=conv / len(res), wall_s=time.perf_counter() - t0,
                    energies=[float(r.energy_per_site) for r in res], sweeps=[int(r.sweeps) for r in res])

    reqs = serving_requests(n)
    closed = run(reqs, "closed")
    out = {"requests": n, "max_active": max_active, "budget_gb": budget_gb, "rsvd_p": p, "rsvd_q": q,
           "tol": tol, "max_sweeps": max_sweeps}
    energies, sweeps = closed.pop("energies"), closed.pop("sweeps")
    out["closed_loop"] = closed
    for load in loads:
        rate = load * closed["solves_per_s"]
        opened = run(serving_requests(n, rate_hz=rate), f"open {load}x")
        # the same request gives the same energy in every run
        same = float(np.max(np.abs(np.array(energies) - np.array(opened.pop("energies")))))
        opened.pop("sweeps")
        out[f"open_loop_{load}x"] = dict(opened, arrival_rate_hz=rate, max_energy_diff_vs_closed=same)
    return out, reqs, sweeps


def d4_bench(lib, sweeps=30, warm=2):
    """D = 4, chi = 64 (2x2 cell, p = 32, q = 2, sketch seed 11, tensors of
    seed 1): sweeps/s over the sweeps after the first `warm`, the sketch
    GEMMs' fraction of the FP64 peak, and the energy per site after all
    sweeps against the oracle's stored run of the same sweeps."""
    A = wl.random_itps(2, 2, 4, 2, seed=1)
    dt, ph, e, cuts = run_sweeps(lib, A, 4, 64, 2, 32, 2, "f64", warm, sweeps - warm, seed=11)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "itps_d4_chi64.json")) as f:
        ref = json.load(f)["energies"][str(sweeps)]
    r = sketch_rate(ph)
    print(f"D=4 chi=64 f64: {(sweeps - warm) / dt:.2f} sweeps/s", file=sys.stderr, flush=True)
    return {"workload": "itps_2x2_d2_D4_chi64", "rsvd_p": 32, "rsvd_q": 2, "sweeps": sweeps,
            "timed_sweeps": sweeps - warm, "sweeps_per_s": (sweeps - warm) / dt, "sketch_tflops": r / 1e12,
            "sketch_frac_of_peak": r / PEAK["f64"], "energy_per_site": e, "oracle_energy_per_site": ref,
            "abs_energy_diff_vs_oracle": abs(e - ref),
            "cuts": dict(zip(("identity", "rsvd_batched", "fallback"), cuts))}


def big_bench(lib, sweeps, D=8, chi=256, p=64, q=1, seed=3, warm=2):
    """D = 8, chi = 256 (2x2 cell): `sweeps` sweeps from the trivial boundary
    in FP64 and in split FP16; sweeps/s over the sweeps after the first
    `warm` (the environment has reached chi by then), the sketch GEMMs'
    fraction of each precision's peak, and the energy difference after all
    sweeps."""
    A = wl.random_itps(2, 2, D, 2, seed=seed)
    out = {"workload": f"itps_2x2_d2_D{D}_chi{chi}", "D": D, "chi": chi, "rsvd_p": p, "rsvd_q": q,
           "sweeps": sweeps, "timed_sweeps": sweeps - warm}
    energies = {}
    for prec in ("f64", "f16split"):
        dt, ph, e, cuts = run_sweeps(lib, A, D, chi, 2, p, q, prec, warm, sweeps - warm)
        r = sketch_rate(ph)
        energies[prec] = e
        out[prec] = {"sweeps_per_s": (sweeps - warm) / dt, "sketch_tflops": r / 1e12,
                     "sketch_frac_of_peak": r / PEAK[prec], "energy_per_site": e,
                     "cuts": dict(zip(("identity", "rsvd_batched", "fallback"), cuts))}
        print(f"D={D} chi={chi} {prec}: {(sweeps - warm) / dt:.3f} sweeps/s", file=sys.stderr, flush=True)
    out["f16split"]["abs_energy_diff_vs_f64"] = abs(energies["f16split"] - energies["f64"])
    out["f16split"]["sketch_passes"] = "3 MFMA passes per product (hi hi, hi lo, lo hi); the fraction counts the algorithmic flops once"
    return out


def ex1_bond(h):
    """The paper's transverse-field Ising example (Sec. 6.1) in spin units,
    J_z = -1: -Sz Sz - (h/4)(Sx 1 + 1 Sx), the field split over the four bonds
    of a site."""
    Sz, Sx = 0.5 * wl.SZ, 0.5 * wl.SX
    return -np.kron(Sz, Sz) - 0.25 * h * (np.kron(Sx, wl.ID2) + np.kron(wl.ID2, Sx))


def su_flops_per_update(D, d):
    """Algorithmic FP64 flops of one bond update of the reduced simple update:
    Householder QR of the two D^3 x Dd tensors, the gated core, an SVD of the
    m x m core with both vector sets (LAPACK count 21 m^3) and the two
    products Q U, Q V."""
    R, C = D ** 3, D * d
    k = min(R, C)
    m = k * d
    qr = 2 * 2 * C * C * (R - C / 3.0)
    core = 2 * k * k * d * d * D + 2 * m * m * d * d
    svd = 21.0 * m ** 3
    rec = 2 * 4.0 * R * C * k
    return qr + core + svd + rec


def su_problem_inputs(hs, D, noise=1e-3, seed=2):
    """Polarised product state (+z) plus noise on every entry, unit weights,
    the spin-unit Ising bond of each field on every bond of the 2x2 cell."""
    N = 4
    rng = np.random.default_rng(seed)
    G0 = [g + noise * rng.standard_normal(g.shape) for g in wl.product_itps([np.array([1.0, 0.0])] * N, D)]
    B = len(hs)
    gam = np.broadcast_to(np.stack(G0)[None], (B, N) + G0[0].shape).copy()
    lam = np.ones((B, N, 2, D))
    H = np.stack([np.stack([np.stack([ex1_bond(h), ex1_bond(h)]) for _ in range(N)]) for h in hs])
    return G0, gam, lam, H


def su_bench(lib, B=256, D=4, steps=1000, tau=0.01, cpu=True, cplx=False):
    """Simple-update imaginary-time evolution of a field scan: B fields of the
    spin-unit transverse-field Ising model in [0, 2.5], 2x2 cell, D, tau, the
    given Trotter steps, all problems in one batch.  Device time from the
    library's HIP events around its launches."""
    hs = np.linspace(0.0, 2.5, B)
    _, gam, lam, H = su_problem_inputs(hs, D)
    warm = lib.SimpleUpdate(gam, lam, 2, 2, D, complex_tensors=cplx)
    warm.set_hamiltonians(H, tau)
    warm.run(10)
    warm.free()
    s = lib.SimpleUpdate(gam, lam, 2, 2, D, complex_tensors=cplx)
    s.set_hamiltonians(H, tau)
    t0 = time.perf_counter()
    s.run(steps)
    wall = time.perf_counter() - t0
    gpu_ms, launches, updates = s.stats()
    e, _ = s.mfe_energy()
    s.free()
    f = su_flops_per_update(D, 2)
    rate = updates / (gpu_ms / 1e3)
    out = {"workload": f"su_tfim_scan_2x2_D{D}_B{B}" + ("_complex" if cplx else ""), "problems": B, "D": D,
           "d": 2, "tau": tau, "arithmetic": "complex FP64" if cplx else "FP64",
           "trotter_steps": steps, "bond_updates": updates, "gpu_ms": gpu_ms, "wall_s": wall,
           "bond_updates_per_s": rate, "launches": launches,
           "roofline": {"bound": "alu", "achieved": rate * f / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                        "frac": rate * f / 78.6e12, "flops_per_bond_update": f,
                        "kernel": "k_su_run (one workgroup per problem, every bond in order)",
                        "flops_counted": "real flops of the real algorithm" + ("; complex arithmetic does about "
                                                                             "four times as many" if cplx else "")},
           "mfe_energy_per_site": {"h_min": float(e[0]), "h_max": float(e[-1])}}
    if cpu:
        from threadpoolctl import threadpool_limits

        from oracle import simple_update as osu
        cores = oracle_threads()
        G0, _, _, _ = su_problem_inputs(hs[:1], D)
        ones = [np.ones(D) for _ in range(4)]
        Hp = [[H[B // 2, i, 0], H[B // 2, i, 1]] for i in range(4)]
        n_cpu = 250
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            osu.simple_update(G0, ones, ones, Hp, tau, 2, 2, n_cpu)
            dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_cpu * 8 / dt, "unit": "bond updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"{n_cpu} Trotter steps (8 bonds each) of one D={D} problem of the scan, "
                                         f"full SVD of the two-site matrix, NumPy/OpenBLAS FP64, {dt:.1f} s"}
    print(f"simple update D={D}{' complex' if cplx else ''}: {rate:.3g} bond updates/s ({gpu_ms:.1f} ms for {updates} updates)",
          file=sys.stderr, flush=True)
    return out


def ex1_scan(lib, fields=32, D=2, steps=1000, tau=0.01, chi=10, sweeps=10):
    """The paper's transverse-field Ising example end to end (Sec. 6.1:
    simple updates 1000, tau 0.01, D 2, chi 10, 10 CTMRG sweeps): simple
    update of every field in one batch, the iTPS of each handed to a CTMRG
    context in device memory, <S^z> and <S^x> averaged over the cell."""
    import torch
    hs = np.linspace(0.0, 2.5, fields)
    _, gam, lam, H = su_problem_inputs(hs, D)
    t0 = time.perf_counter()
    s = lib.SimpleUpdate(gam, lam, 2, 2, D)
    s.set_hamiltonians(H, tau)
    s.run(steps)
    buf = torch.empty(fields * 4 * D ** 4 * 2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.get_itps(device_ptr=buf.data_ptr())
    s.free()
    t_su = time.perf_counter() - t0
    sz, sx, es = [], [], []
    per = 4 * D ** 4 * 2
    for b in range(fields):
        ctx = lib.Ctm(None, 2, 2, D, chi=chi, device_ptr=buf.data_ptr() + 8 * b * per)
        ctx.ctm_sweep(sweeps, 1e-10)
        sz.append(float(np.mean([abs(ctx.ctm_expect_1site(i, 0.5 * wl.SZ)) for i in range(4)])))
        sx.append(float(np.mean([ctx.ctm_expect_1site(i, 0.5 * wl.SX) for i in range(4)])))
        es.append(float(np.mean([ctx.ctm_expect_2site(i, dr, ex1_bond(hs[b])) for i in range(4) for dr in (0, 1)]) * 2))
        ctx.ctm_free()
    wall = time.perf_counter() - t0
    print(f"transverse-field Ising scan: {fields} fields in {wall:.1f} s", file=sys.stderr, flush=True)
    # the same CTMRG solves through the serving queue, which runs same-shape
    # requests as replicas of one context (the simple update's device output
    # copied at submit)
    t1 = time.perf_counter()
    q = lib.Queue(16 << 30, 8)
    tickets = []
    for b in range(fields):
        st, tk = q.submit(None, 2, 2, D, chi, ex1_bond(hs[b]), tol=1e-10, max_sweeps=sweeps,
                          device_ptr=buf.data_ptr() + 8 * b * per, obs=[0.5 * wl.SZ, 0.5 * wl.SX], tag=b)
        assert st == 0, st
        tickets.append(tk)
    qsz, qsx, qes = [], [], []
    for tk in tickets:
        st, r = q.wait(tk)
        assert st == 0 and r.status == 0, (st, r.status)
        qsz.append(float(np.mean(np.abs(r.observable(0, 4)))))
        qsx.append(float(np.mean(r.observable(1, 4))))
        qes.append(float(r.energy_per_site))
    q.destroy()
    t_queue = time.perf_counter() - t1
    diff = max(max(abs(a - b) for a, b in zip(es, qes)), max(abs(a - b) for a, b in zip(sz, qsz)),
               max(abs(a - b) for a, b in zip(sx, qsx)))
    print(f"transverse-field Ising scan, CTMRG through the queue: {t_queue:.2f} s "
          f"(one context per field: {wall - t_su:.2f} s), max difference {diff:.1e}", file=sys.stderr, flush=True)
    return {"workload": f"ex1_tfim_scan_2x2_D{D}_chi{chi}", "fields": fields, "su_steps": steps, "tau": tau,
            "ctm_sweeps": sweeps, "h": [float(h) for h in hs], "abs_sz": sz, "sx": sx, "energy_per_site": es,
            "su_wall_s": t_su, "wall_s": wall, "ctm_queue_wall_s": t_queue,
            "ctm_sequential_wall_s": wall - t_su, "queue_max_abs_diff": diff}


def fu_bench(lib, D=4, chi=32, p=32, h=1.5, su_steps=500, fu_steps=3, tau=0.01, als_iters=5, env_sweeps=1,
             cpu=True):
    """The paper's optimisation pipeline on one problem (Sec. 2.3): simple
    updates, the iTPS handed to a CTMRG context and converged, then full-update
    Trotter steps (each bond with its CTMRG environment, env_sweeps sweeps
    after each bond).  Reports the time per full-update step and the CTMRG
    energy per site before and after."""
    import torch
    hs = np.array([h])
    _, gam, lam, H = su_problem_inputs(hs, D)
    s = lib.SimpleUpdate(gam, lam, 2, 2, D)
    s.set_hamiltonians(H, tau)
    s.run(su_steps)
    buf = torch.empty(4 * D ** 4 * 2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.get_itps(device_ptr=buf.data_ptr())
    A0 = s.get_itps()[0]
    s.free()
    Hb = ex1_bond(h)
    Hfu = np.asarray([[Hb, Hb] for _ in range(4)])
    ctx = lib.Ctm(None, 2, 2, D, chi=chi, device_ptr=buf.data_ptr(), rsvd_oversample=p)
    ctx.ctm_sweep(30, 1e-10)
    e_su = sum(ctx.ctm_expect_2site(i, dr, Hb) for i in range(4) for dr in (0, 1)) / 4
    t0 = time.perf_counter()
    ctx.ctm_sweep(1, 0.0)
    t_sweep = time.perf_counter() - t0
    ctx.ctm_fu_step(Hfu, tau, als_iters=als_iters, env_sweeps=env_sweeps)      # warm-up step
    t0 = time.perf_counter()
    for _ in range(fu_steps):
        ctx.ctm_fu_step(Hfu, tau, als_iters=als_iters, env_sweeps=env_sweeps)
    dt = (time.perf_counter() - t0) / fu_steps
    ctx.ctm_sweep(30, 1e-10)
    e_fu = sum(ctx.ctm_expect_2site(i, dr, Hb) for i in range(4) for dr in (0, 1)) / 4
    ctx.ctm_free()
    out = {"workload": f"fu_tfim_2x2_D{D}_chi{chi}_h{h}", "D": D, "chi": chi, "rsvd_p": p, "h": h, "tau": tau,
           "su_steps_before": su_steps, "fu_steps_timed": fu_steps, "als_iters": als_iters,
           "env_sweeps_per_bond": env_sweeps, "ms_per_fu_step": 1e3 * dt,
           "bond_updates_per_s": 8.0 / dt, "ms_per_env_sweep": 1e3 * t_sweep,
           "env_share": 8 * env_sweeps * t_sweep / dt,
           "energy_per_site_su": e_su, "energy_per_site_after_fu": e_fu}
    if cpu:
        from threadpoolctl import threadpool_limits

        from oracle import full_update as ofu
        from oracle.ctmrg import Environment
        cores = oracle_threads()
        from oracle.simple_update import gate as ogate
        with threadpool_limits(limits=cores):
            env = Environment([np.array(a) for a in A0], 2, 2, chi=chi, oversample=p)
            for _ in range(3):
                env.sweep()
            t0 = time.perf_counter()
            ofu.bond_update(env, 0, 0, ogate(Hb, tau), als_iters)
            t_bond = time.perf_counter() - t0
            t0 = time.perf_counter()
            env.sweep()
            t_env = time.perf_counter() - t0
        step = 8 * (t_bond + env_sweeps * t_env)
        out["cpu_baseline"] = {"value": 8.0 / step, "unit": "bond updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"one full-update bond update ({t_bond:.1f} s) and one CTMRG sweep "
                                         f"({t_env:.1f} s) of the same D={D}, chi={chi} workload, NumPy/OpenBLAS "
                                         f"FP64; a Trotter step is 8 of each"}
    print(f"full update D={D} chi={chi}: {1e3 * dt:.0f} ms per Trotter step", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="f64", choices=sorted(PEAK))
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=144)
    ap.add_argument("--p", type=int, default=48)
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the comparison runs in the other precisions")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies (counter calibration)")
    ap.add_argument("--serving", type=int, default=512, metavar="N",
                    help="also run the first N requests of the mixed TFIM serving stream (512 = all, 0 = none)")
    ap.add_argument("--loads", default="0.8",
                    help="open-loop arrival rates as fractions of the closed-loop capacity (comma list)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving stream")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--big-sweeps", type=int, default=20,
                    help="sweeps of the D=8, chi=256 comparison of split FP16 with FP64 (0 = skip)")
    ap.add_argument("--su", type=int, default=1, help="simple-update and field-scan sections (0 = skip)")
    ap.add_argument("--su-only", action="store_true", help="run only the simple-update sections")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2112_13184_amd as lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    lib.load()
    loads = tuple(float(x) for x in args.loads.split(",") if x)
    if args.serving_only:
        sv, _, _ = serving_bench(lib, args.serving or 512, args.max_active, args.budget_gb, loads=loads)
        print(json.dumps({"serving": sv}), flush=True)
        return
    if args.su_only:
        out = {"simple_update": su_bench(lib, cpu=not args.no_cpu_baseline),
               "simple_update_d2": su_bench(lib, D=2, cpu=False),
               "simple_update_b1024": su_bench(lib, B=1024, steps=400, cpu=False),
               "simple_update_complex": su_bench(lib, cpu=False, cplx=True), "ex1_scan": ex1_scan(lib),
               "full_update": fu_bench(lib, cpu=not args.no_cpu_baseline)}
        print(json.dumps(out), flush=True)
        return
    D, chi, d, p, q = args.D, args.chi, 2, args.p, args.q
    A = wl.random_itps(2, 2, D, d, seed=2)
    dt, phases, energy, cuts = run_sweeps(lib, A, D, chi, d, p, q, args.prec, args.warmup, args.steps)
    # the phase breakdown from a second pass with every phase timed
    _, all_phases, _, _ = run_sweeps(lib, A, D, chi, d, p, q, args.prec, args.warmup, args.steps, timing=1)
    n, k = chi * D * D, min(chi + p, chi * D * D)   # one launch: 2 cuts, corner n x n, panel n x k
    sweeps_per_s = args.steps / dt
    sk = phases["sketch_gemm"]
    achieved = sketch_rate(phases)
    alg = flops_per_sweep(D, chi, d, p, q)
    out = {
        "metric": METRIC,
        "value": sweeps_per_s,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"itps_2x2_d2_D{D}_chi{chi}", "Lx": 2, "Ly": 2, "d": d, "D": D,
                   "chi": chi, "rsvd_p": p, "rsvd_q": q, "precision": args.prec, "tensor_seed": 2},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[args.prec] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[args.prec],
                     # the counters were taken on the default workload only
                     "traffic": counted_traffic() if (args.prec == "f64" and (D, chi, p, q) == (6, 144, 48, 1))
                     else None,
                     "kernel": "sketch GEMMs (n x k panel times n x n corner)",
                     "alg_bytes_per_launch": 8.0 * 2 * (n * n + 2 * n * k),
                     "launches": sk["launches"], "avg_launch_ms": sk["ms"] / max(sk["launches"], 1),
                     "flops_per_launch": sk["flops"] / max(sk["launches"], 1)},
        "whole_sweep": {"alg_tflop": alg / 1e12, "achieved_tflops": alg * sweeps_per_s / 1e12,
                        "frac_of_peak": alg * sweeps_per_s / PEAK[args.prec]},
        "phases_ms_per_sweep": {k: v["ms"] / args.steps for k, v in all_phases.items()},
        "phases_note": "a separate pass of the same sweeps with every phase timed (its events add idle gaps); "
                       "value and roofline come from the pass that times the sketch products only",
        "energy_per_site": energy,
        "cuts": dict(zip(("identity", "rsvd_batched", "fallback"), cuts)),
    }
    if not args.no_precisions:
        # the same workload and sweep count in every precision: throughput,
        # sketch-GEMM MFMA fraction of that precision's peak, and the energy
        # difference to this run (the FP64 path is matched to the oracle move
        # by move at this size)
        cmp = {}
        for prec in ("f64", "f32", "f16split", "bf16"):
            if prec == args.prec:
                continue
            dtp, php, ep, _ = run_sweeps(lib, A, D, chi, d, p, q, prec, args.warmup, args.steps)
            r = sketch_rate(php)
            cmp[prec] = {"sweeps_per_s": args.steps / dtp, "sketch_tflops": r / 1e12,
                         "sketch_frac_of_peak": r / PEAK[prec], "peak_tflops": PEAK[prec] / 1e12,
                         "energy_per_site": ep, "abs_energy_diff": abs(ep - energy)}
        out["precisions"] = cmp
    if args.big_sweeps:
        out["d4_chi64"] = d4_bench(lib)
        out["d8_chi256"] = big_bench(lib, args.big_sweeps)
    if args.su:
        out["simple_update"] = su_bench(lib, cpu=not args.no_cpu_baseline)
        out["simple_update_complex"] = su_bench(lib, cpu=False, cplx=True)
        # 1024 fields: four problems per CU, the throughput of a saturated GPU
        out["simple_update_b1024"] = su_bench(lib, B=1024, steps=400, cpu=False)
        out["ex1_scan"] = ex1_scan(lib)
        # the oracle's full-update bond update takes about a minute: its CPU leg
        # runs with --su-only
        out["full_update"] = fu_bench(lib, cpu=False)
    sv_reqs = sv_sweeps = None
    if args.serving:
        out["serving"], sv_reqs, sv_sweeps = serving_bench(lib, args.serving, args.max_active, args.budget_gb,
                                                           loads=loads)
        out["serving_scan"] = scan_bench(lib, 16, args.max_active, args.budget_gb)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(D, chi, p, q, seed=2)
        rate = out["serving"][f"open_loop_{loads[0]}x"]["arrival_rate_hz"] if sv_reqs and loads else None
        arrivals = serving_requests(len(sv_reqs), rate_hz=rate) if sv_reqs and rate else sv_reqs
        out["cpu_baseline_more"] = cpu_baseline_extra(
            [{"sweeps": n} for n in sv_sweeps] if sv_sweeps else None, arrivals, rate)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
