"""The serving queue (continuous batching of CTMRG solves on one GPU), through
the C ABI: results alone and in a mix, closed forms through the queue, HBM
budget admission, cancellation, and the footprint bound."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import observables as ob
from oracle.ctmrg import Environment
from paper_2112_13184_amd import _binding as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


def _requests(n, seed=4, eps=0.1, chi_max=40, D_max=3):
    reqs = []
    for r in wl.serving_stream(n=n, seed=seed, eps=eps):
        D = 2 + (r["D"] - 2) % (D_max - 1)
        chi = 16 + (r["chi"] - 16) % (chi_max - 15)
        A = wl.tfim_request_tensors(r["h"], D, r["Lx"], r["Ly"], eps, r["tensor_seed"])
        reqs.append(dict(A=A, h=r["h"], D=D, chi=chi, Lx=r["Lx"], Ly=r["Ly"]))
    return reqs


def _submit(q, r, tag, max_sweeps=12, **kw):
    return q.submit(r["A"], r["Lx"], r["Ly"], r["D"], r["chi"], wl.tfim_bond(r["h"]), tol=1e-10,
                    max_sweeps=max_sweeps, tag=tag, rsvd_oversample=16, rsvd_power_iters=1, seed=3,
                    obs=[wl.SZ], **kw)


def _mz(res, r):
    return list(res.observable(0, r["Lx"] * r["Ly"]))


def test_results_alone_equal_results_in_mix(lib):
    """Every solve owns its context and stream, so running it alone (one at a
    time) or among others gives the same numbers (bitwise, as the kernels are
    deterministic); the stated tolerance 1e-10 is asserted, equality
    reported."""
    reqs = _requests(10)
    alone = []
    q1 = lib.Queue(64 << 30, 1)
    for i, r in enumerate(reqs):
        st, t = _submit(q1, r, i)
        assert st == B.CTM_OK
        st, res = q1.wait(t, 120000)
        assert st == B.CTM_OK, st
        alone.append((res.energy_per_site, res.sweeps, _mz(res, r)))
    q1.destroy()
    q = lib.Queue(64 << 30, 6)
    tickets = []
    for i, r in enumerate(reqs):
        st, t = _submit(q, r, i)
        assert st == B.CTM_OK
        tickets.append(t)
    mixed = []
    overlap = 0
    spans = []
    for i, t in enumerate(tickets):
        st, res = q.wait(t, 120000)
        assert st == B.CTM_OK, st
        assert res.tag == i
        mixed.append((res.energy_per_site, res.sweeps, _mz(res, reqs[i])))
        spans.append((res.t_admit_ns, res.t_done_ns))
    q.destroy()
    for (ea, sa, ma), (em, sm, mm) in zip(alone, mixed):
        assert sa == sm
        assert abs(ea - em) <= 1e-10
        assert np.max(np.abs(np.array(ma) - np.array(mm))) <= 1e-10
    # the mix really ran concurrently
    for i in range(len(spans)):
        for j in range(i + 1, len(spans)):
            overlap += spans[i][0] < spans[j][1] and spans[j][0] < spans[i][1]
    assert overlap > 0
    print("bitwise equal:", all(a == m for a, m in zip(alone, mixed)), "overlapping pairs:", overlap)


def test_mean_field_states_through_queue(lib):
    """eps = 0: exact product states, energy = the TFIM mean-field closed form."""
    q = lib.Queue(16 << 30, 4)
    hs = [2.6, 3.0, 3.4]
    tickets = []
    for i, h in enumerate(hs):
        A = wl.tfim_request_tensors(h, 3, 2, 2, 0.0, seed=i)
        st, t = q.submit(A, 2, 2, 3, 20, wl.tfim_bond(h), tol=1e-12, max_sweeps=6, tag=i,
                         rsvd_oversample=8, rsvd_power_iters=1, seed=1)
        assert st == B.CTM_OK
        tickets.append(t)
    for h, t in zip(hs, tickets):
        st, res = q.wait(t, 60000)
        assert st == B.CTM_OK
        _, e_mf = wl.tfim_mean_field(h)
        assert abs(res.energy_per_site - e_mf) < 1e-12
    q.destroy()


def test_queue_matches_oracle(lib):
    """The converged transverse-field Ising requests of the stored oracle runs
    (D = 2 and 3, 1x1 and 2x2 cells, 40 sweeps), submitted together: energy
    per site and <sigma_z> against the oracle, 1e-10 (tests/golden/
    tfim_converged.json, written by make_golden.py from the oracle alone)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tfim_converged.json")))
    w = g["params"]
    q = lib.Queue(16 << 30, 4)
    tickets = []
    for i, c in enumerate(g["cases"]):
        A = wl.tfim_request_tensors(c["h"], c["D"], c["L"], c["L"], w["eps"], seed=c["tensor_seed"])
        st, t = q.submit(A, c["L"], c["L"], c["D"], c["chi"], wl.tfim_bond(c["h"]), tol=0.0,
                         max_sweeps=w["sweeps"], tag=i, rsvd_oversample=w["p"], rsvd_power_iters=w["q"],
                         seed=w["sketch_seed"], svd_rel_cutoff=g["cutoff"], obs=[wl.SZ])
        assert st == B.CTM_OK
        tickets.append(t)
    for c, t in zip(g["cases"], tickets):
        st, res = q.wait(t, 120000)
        assert st == B.CTM_OK and res.sweeps == w["sweeps"]
        de = abs(res.energy_per_site - c["energies"][str(w["sweeps"])])
        dmz = max(abs(res.obs[0][i] - c["mz"][i]) for i in range(c["L"] ** 2))
        print(f"queue, tfim L={c['L']} D={c['D']} chi={c['chi']}: |dE| = {de:.2e}, max |d mz| = {dmz:.2e}")
        assert de < 1e-10 and dmz < 1e-10
    q.destroy()


def test_budget_admission_and_cancel(lib):
    reqs = _requests(4, seed=5)
    fp = [B.ctm_footprint_bytes(B.make_config(r["Lx"], r["Ly"], r["D"], r["chi"], rsvd_oversample=16))
          for r in reqs]
    # a budget that holds the largest request but not two of them
    budget = max(fp) + min(fp) // 2
    q = lib.Queue(budget, 4)
    tickets = []
    for i, r in enumerate(reqs):
        st, t = _submit(q, r, i)
        assert st == B.CTM_OK
        tickets.append(t)
    spans = []
    for t in tickets:
        st, res = q.wait(t, 120000)
        assert st == B.CTM_OK
        spans.append((res.t_admit_ns, res.t_done_ns))
    # no two solves whose summed footprints exceed the budget ran together
    for i in range(len(spans)):
        for j in range(i + 1, len(spans)):
            if fp[i] + fp[j] > budget:
                assert not (spans[i][0] < spans[j][1] and spans[j][0] < spans[i][1]), (i, j)
    # larger than the whole budget: rejected at once
    A5 = wl.tfim_request_tensors(3.0, 5, 2, 2, 0.1, seed=6)
    st, _ = q.submit(A5, 2, 2, 5, 200, wl.tfim_bond(3.0))
    assert st == B.CTM_ETOOBIG
    q.destroy()
    # cancellation of pending requests behind a running one
    q = lib.Queue(64 << 30, 1)
    ts = [_submit(q, r, i, max_sweeps=30)[1] for i, r in enumerate(reqs)]
    assert q.cancel(ts[-1]) == B.CTM_OK
    st, res = q.wait(ts[-1], 60000)
    assert st == B.CTM_ECANCELED
    st, res = q.wait(ts[0], 120000)
    assert st == B.CTM_OK
    q.destroy()


def _device_free_bytes():
    """hipMemGetInfo of the HIP runtime the library itself uses (torch's: the
    binding loads torch before the library)."""
    import torch
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    return free


@pytest.mark.parametrize("D,chi,L", [(2, 16, 1), (3, 40, 2), (5, 100, 2), (6, 144, 2)])
def test_footprint_bounds_device_memory(lib, D, chi, L):
    """ctm_footprint_bytes (the admission size) bounds the device memory a
    context holds after sweeps and the energy evaluation."""
    # one-time runtime set-up (code objects, library kernels) is not per context
    warm = lib.Ctm(wl.random_itps(1, 1, 2, 2, seed=1), 1, 1, 2, 8, rsvd_oversample=8)
    warm.ctm_move("left")
    warm.ctm_expect_2site(0, 0, wl.heisenberg_bond())
    warm.ctm_expect_1site(0, wl.SZ)
    del warm
    free0 = _device_free_bytes()
    A = wl.random_itps(L, L, D, 2, seed=1)
    ctx = lib.Ctm(A, L, L, D, chi, rsvd_oversample=16, rsvd_power_iters=1, seed=1)
    for dname in ("left", "right", "up", "down"):
        ctx.ctm_move(dname)
    H = wl.heisenberg_bond()
    for i in range(L * L):
        ctx.ctm_expect_2site(i, 0, H)
        ctx.ctm_expect_2site(i, 1, H)
        ctx.ctm_expect_1site(i, wl.SZ)
    free1 = _device_free_bytes()
    used = free0 - free1
    fp = B.ctm_footprint_bytes(B.make_config(L, L, D, chi, rsvd_oversample=16))
    print(f"D={D} chi={chi} {L}x{L}: used {used / 2**20:.1f} MiB, footprint {fp / 2**20:.1f} MiB")
    assert used <= fp
    del ctx


def test_same_shape_requests_run_as_one_group(lib):
    """A transverse-field scan at one shape (2x2, D=3, chi=24) plus two other
    shapes: submitted together, the same-shape requests are admitted as one
    group (one context, their cuts batched into the same launches) and give
    the same results as when each runs alone."""
    hs = [2.6, 2.8, 3.0, 3.2, 3.4]
    reqs = [dict(A=wl.tfim_request_tensors(h, 3, 2, 2, 0.1, seed=40 + i), h=h, D=3, chi=24, Lx=2, Ly=2)
            for i, h in enumerate(hs)]
    reqs += _requests(2, seed=41)
    alone = []
    q1 = lib.Queue(64 << 30, 1)
    for i, r in enumerate(reqs):
        st, t = _submit(q1, r, i, max_sweeps=8 + i)
        assert st == B.CTM_OK
        st, res = q1.wait(t, 120000)
        assert st == B.CTM_OK, st
        alone.append((res.energy_per_site, res.sweeps, _mz(res, r)))
    q1.destroy()
    # one slot: a request of another shape runs first, so that the scan is
    # pending as a whole when the slot frees up
    q = lib.Queue(64 << 30, 1)
    order = [len(hs)] + list(range(len(hs))) + [len(hs) + 1]
    tickets = {i: _submit(q, reqs[i], i, max_sweeps=8 + i)[1] for i in order}
    grouped, admits, dones = [], [], []
    for i in range(len(reqs)):
        st, res = q.wait(tickets[i], 120000)
        assert st == B.CTM_OK, st
        grouped.append((res.energy_per_site, res.sweeps, _mz(res, reqs[i])))
        admits.append(res.t_admit_ns)
        dones.append(res.t_done_ns)
    q.destroy()
    # the scan shares one admission (one group); different caps per request,
    # and each result is published when its own solve ends
    assert len(set(admits[:len(hs)])) == 1 and admits[len(hs)] < admits[0]
    assert all(dones[i] < dones[i + 1] for i in range(len(hs) - 1)), dones[:len(hs)]
    for (ea, sa, ma), (eg, sg, mg) in zip(alone, grouped):
        assert sa == sg
        assert abs(ea - eg) <= 1e-10
        assert np.max(np.abs(np.array(ma) - np.array(mg))) <= 1e-10
    print("bitwise equal:", all(a == g for a, g in zip(alone, grouped)))


def test_pending_request_joins_running_group(lib):
    """Nine requests of one shape with one worker: eight form a group (the
    largest group), the ninth waits and starts in the slot of the first solve
    to finish, at a sweep boundary, while the others are still running.  Every
    result equals the request run alone (bitwise expected, 1e-10 asserted)."""
    hs = [2.5 + 0.1 * i for i in range(9)]
    reqs = [dict(A=wl.tfim_request_tensors(h, 2, 2, 2, 0.1, seed=60 + i), h=h, D=2, chi=16, Lx=2, Ly=2)
            for i, h in enumerate(hs)]
    caps = [3] + [10] * 8
    alone = []
    q1 = lib.Queue(64 << 30, 1)
    for i, r in enumerate(reqs):
        st, t = _submit(q1, r, i, max_sweeps=caps[i])
        st, res = q1.wait(t, 120000)
        assert st == B.CTM_OK, st
        alone.append((res.energy_per_site, res.sweeps, _mz(res, r)))
    q1.destroy()
    q = lib.Queue(64 << 30, 1)
    # a request of another shape occupies the worker first, so that the nine
    # are all pending when it frees up
    blocker = _requests(1, seed=61, chi_max=30, D_max=3)[0]
    blocker.update(Lx=1, Ly=1, A=blocker["A"][:1], chi=30)
    tb = _submit(q, blocker, 99, max_sweeps=8)[1]
    tickets = [_submit(q, r, i, max_sweeps=caps[i])[1] for i, r in enumerate(reqs)]
    out = [q.wait(t, 120000) for t in tickets]
    assert q.wait(tb, 120000)[0] == B.CTM_OK
    q.destroy()
    for st, _ in out:
        assert st == B.CTM_OK
    res = [r for _, r in out]
    admit0 = res[0].t_admit_ns
    assert all(r.t_admit_ns == admit0 for r in res[:8])
    # the ninth joined the running group: after the first solve was published
    # and before the other seven ended
    assert res[0].t_done_ns <= res[8].t_admit_ns < min(r.t_done_ns for r in res[1:8])
    for i, r in enumerate(res):
        e, n, m = r.energy_per_site, r.sweeps, _mz(r, reqs[i])
        assert n == alone[i][1]
        assert abs(e - alone[i][0]) <= 1e-10
        assert np.max(np.abs(np.array(m) - np.array(alone[i][2]))) <= 1e-10
    print("bitwise equal:", all((r.energy_per_site, r.sweeps, _mz(r, reqs[i])) == alone[i] for i, r in enumerate(res)))


def test_numerical_failure_is_isolated_in_group(lib):
    """A request whose tensors are all zero (every cut loses all its singular
    values) grouped with valid requests of the same shape: it ends with
    CTM_ENUMERIC, the others finish with the results they have alone.  NaN
    tensors are rejected at submit."""
    hs = [2.7, 3.0, 3.3]
    reqs = [dict(A=wl.tfim_request_tensors(h, 2, 2, 2, 0.1, seed=80 + i), h=h, D=2, chi=16, Lx=2, Ly=2)
            for i, h in enumerate(hs)]
    bad = dict(reqs[0], A=[np.zeros_like(a) for a in reqs[0]["A"]])
    alone = []
    q1 = lib.Queue(64 << 30, 1)
    for i, r in enumerate(reqs):
        st, t = _submit(q1, r, i, max_sweeps=10)
        st, res = q1.wait(t, 120000)
        assert st == B.CTM_OK, st
        alone.append((res.energy_per_site, res.sweeps, _mz(res, r)))
    q1.destroy()
    q = lib.Queue(64 << 30, 1)
    blocker = _requests(1, seed=61, chi_max=30, D_max=3)[0]
    blocker.update(Lx=1, Ly=1, A=blocker["A"][:1], chi=30)
    tb = _submit(q, blocker, 99, max_sweeps=8)[1]
    order = [reqs[0], bad, reqs[1], reqs[2]]
    tickets = [_submit(q, r, i, max_sweeps=10)[1] for i, r in enumerate(order)]
    out = [q.wait(t, 120000) for t in tickets]
    assert q.wait(tb, 120000)[0] == B.CTM_OK
    nan = dict(reqs[0], A=[a.copy() for a in reqs[0]["A"]])
    nan["A"][1][0, 0, 0, 0, 0] = np.nan
    st_nan, _ = _submit(q, nan, 9)
    q.destroy()
    assert st_nan == B.CTM_ENUMERIC
    assert out[1][0] == B.CTM_ENUMERIC
    assert len({r.t_admit_ns for _, r in out}) == 1   # one group
    for (st, res), ref, r in zip([out[0], out[2], out[3]], alone, reqs):
        assert st == B.CTM_OK
        assert res.sweeps == ref[1] and abs(res.energy_per_site - ref[0]) <= 1e-10
        assert np.max(np.abs(np.array(_mz(res, r)) - np.array(ref[2]))) <= 1e-10


def test_device_tensors_and_caller_stream(lib):
    """Site tensors in device memory (a torch tensor) read on the caller's
    stream (torch's current stream), through ctm_init (ctm_config.stream) and
    through the queue (ctm_queue_create's stream): bitwise the results of the
    host-memory inputs."""
    import torch
    r = _requests(1, seed=12, chi_max=24, D_max=3)[0]
    N = r["Lx"] * r["Ly"]
    host = np.concatenate([a.reshape(-1) for a in r["A"]])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dev = torch.from_numpy(host).to("cuda", non_blocking=False) * 1.0   # produced on `stream`
        sptr = stream.cuda_stream
        kw = dict(rsvd_oversample=16, rsvd_power_iters=1, seed=3)
        c_host = lib.Ctm(r["A"], r["Lx"], r["Ly"], r["D"], r["chi"], **kw)
        c_dev = lib.Ctm(None, r["Lx"], r["Ly"], r["D"], r["chi"], device_ptr=dev.data_ptr(), stream=sptr, **kw)
        H = wl.tfim_bond(r["h"])
        vals = []
        for c in (c_host, c_dev):
            c.ctm_sweep(6, 0.0)
            vals.append([c.ctm_expect_2site(i, dr, H) for i in range(N) for dr in (0, 1)]
                        + [c.ctm_expect_1site(i, wl.SZ) for i in range(N)])
        assert vals[0] == vals[1]
        c_dev.ctm_free()
        q = lib.Queue(16 << 30, 2, stream=sptr)
        st1, t1 = _submit(q, r, 0, max_sweeps=6)
        st2, t2 = _submit(q, r, 1, max_sweeps=6, device_ptr=dev.data_ptr())
        assert st1 == B.CTM_OK and st2 == B.CTM_OK
        (s1, a), (s2, b) = q.wait(t1, 60000), q.wait(t2, 60000)
        q.destroy()
    stream.synchronize()
    assert s1 == B.CTM_OK and s2 == B.CTM_OK
    assert a.energy_per_site == b.energy_per_site and _mz(a, r) == _mz(b, r)
