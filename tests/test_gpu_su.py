"""Simple update and mean-field environment: HIP library (C ABI) against the FP64 oracle.

Both sides are FP64 and take the same seeded inputs; the GPU reduces each bond
by QR and takes a Jacobi SVD of the small core, the oracle takes LAPACK's SVD
of the full two-site matrix, so results agree to rounding amplified by the
gaps of the kept spectrum.  Bounds:
* bond weights: 1e-10 absolute (they are singular values of unit-norm
  spectra);
* site tensors compared with the full weight on every leg (indices of a zero
  weight carry nothing and are arbitrary on both sides): 1e-9 relative to the
  largest entry;
* mean-field density matrices and energies: 1e-10 absolute; 1e-12 when both
  sides contract the same stored state.
Where the spectrum is degenerate by symmetry (product states, the Heisenberg
model) only the weights and the observables are compared.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import closed_forms as cf
from oracle import simple_update as su

pytestmark = pytest.mark.gpu

SZ, SX = wl.SZ, wl.SX


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


def ex1_bond(h):
    """The paper's transverse-field Ising example in spin units, J_z = -1:
    -Sz Sz - (h/4)(Sx 1 + 1 Sx), the field split over the four bonds of a site."""
    Sz, Sx = 0.5 * SZ, 0.5 * SX
    return -np.kron(Sz, Sz) - 0.25 * h * (np.kron(Sx, wl.ID2) + np.kron(wl.ID2, Sx))


def uniform_H(op, N):
    return [[op, op] for _ in range(N)]


def run_both(lib, G0, lh0, lv0, H, tau, Lx, Ly, D, d, nsteps):
    """One problem through the GPU and the oracle; returns both states."""
    N = Lx * Ly
    lam = np.stack([np.stack([lh0[s], lv0[s]]) for s in range(N)])
    s = lib.SimpleUpdate(np.stack(G0)[None], lam[None], Lx, Ly, D, d=d)
    s.set_hamiltonians(np.asarray(H)[None], tau)
    s.run(nsteps)
    g, lm = s.get()
    e_gpu, be_gpu = s.mfe_energy()
    r1, r2 = s.mfe()
    s.free()
    Go, lho, lvo = su.simple_update(G0, lh0, lv0, H, tau, Lx, Ly, nsteps)
    gpu = dict(G=list(g[0]), lh=[lm[0, i, 0] for i in range(N)], lv=[lm[0, i, 1] for i in range(N)],
               e=e_gpu[0], r1=r1[0], r2=r2[0])
    orc = dict(G=Go, lh=lho, lv=lvo, e=su.mfe_energy(Go, lho, lvo, Lx, Ly, H))
    return gpu, orc


def compare(gpu, orc, Lx, Ly, tensors=True, tag=""):
    N = Lx * Ly
    dl = max(float(np.abs(gpu["lh"][i] - orc["lh"][i]).max()) for i in range(N))
    dl = max(dl, max(float(np.abs(gpu["lv"][i] - orc["lv"][i]).max()) for i in range(N)))
    de = abs(gpu["e"] - orc["e"])
    msg = f"{tag}: weights {dl:.2e}, energy {de:.2e}"
    if tensors:
        Wg = su.weighted(gpu["G"], gpu["lh"], gpu["lv"], Lx, Ly)
        Wo = su.weighted(orc["G"], orc["lh"], orc["lv"], Lx, Ly)
        dg = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(Wg, Wo))
        msg += f", weighted tensors {dg:.2e}"
    print(msg)
    assert dl < 1e-10, msg
    assert de < 1e-10, msg
    if tensors:
        assert dg < 1e-9, msg


@pytest.mark.parametrize("D", [2, 3, 4])
def test_random_state_tfim_parity(lib, D):
    Lx = Ly = 2
    N = 4
    G0 = wl.random_itps(Lx, Ly, D, 2, seed=10 + D)
    ones = [np.ones(D) for _ in range(N)]
    H = uniform_H(wl.tfim_bond(3.0), N)
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.01, Lx, Ly, D, 2, 20)
    compare(gpu, orc, Lx, Ly, tag=f"D={D}")


def test_ragged_cell_and_batch(lib):
    """A 3x2 cell (odd width, six sites) and a batch of three problems with
    their own tensors, Hamiltonians and tau."""
    Lx, Ly, D, d = 3, 2, 3, 2
    N = Lx * Ly
    hs, taus = [2.0, 3.0, 4.0], [0.02, 0.01, 0.005]
    G0s = [wl.random_itps(Lx, Ly, D, d, seed=40 + b) for b in range(3)]
    rng = np.random.default_rng(7)
    lam0 = rng.uniform(0.2, 1.0, size=(3, N, 2, D))
    Hs = [uniform_H(wl.tfim_bond(h), N) for h in hs]
    s = lib.SimpleUpdate(np.stack([np.stack(g) for g in G0s]), lam0, Lx, Ly, D, d=d)
    s.set_hamiltonians(np.asarray(Hs), np.asarray(taus))
    s.run(12)
    g, lm = s.get()
    e, _ = s.mfe_energy()
    s.free()
    for b in range(3):
        lh0 = [lam0[b, i, 0] for i in range(N)]
        lv0 = [lam0[b, i, 1] for i in range(N)]
        Go, lho, lvo = su.simple_update(G0s[b], lh0, lv0, Hs[b], taus[b], Lx, Ly, 12)
        gpu = dict(G=list(g[b]), lh=[lm[b, i, 0] for i in range(N)], lv=[lm[b, i, 1] for i in range(N)], e=e[b])
        orc = dict(G=Go, lh=lho, lv=lvo, e=su.mfe_energy(Go, lho, lvo, Lx, Ly, Hs[b]))
        compare(gpu, orc, Lx, Ly, tag=f"problem {b}")


def test_spin_one_general_hamiltonian(lib):
    """d = 3 with a random symmetric bond Hamiltonian per bond (and per direction)."""
    Lx = Ly = 2
    N, D, d = 4, 2, 3
    rng = np.random.default_rng(21)
    H = []
    for _ in range(N):
        row = []
        for _ in range(2):
            X = rng.standard_normal((9, 9))
            row.append(0.5 * (X + X.T))
        H.append(row)
    G0 = wl.random_itps(Lx, Ly, D, d, seed=5)
    ones = [np.ones(D) for _ in range(N)]
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.02, Lx, Ly, D, d, 10)
    compare(gpu, orc, Lx, Ly, tag="d=3")


@pytest.mark.parametrize("D", [2, 3])
def test_product_state_tfim(lib, D):
    """From the polarised product state (rank-deficient first updates, exact
    zero weights for D = 3): weights and energies."""
    Lx = Ly = 2
    N = 4
    G0 = wl.product_itps([np.array([1.0, 0.0])] * N, D)
    ones = [np.ones(D) for _ in range(N)]
    H = uniform_H(ex1_bond(1.2), N)
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.01, Lx, Ly, D, 2, 50)
    compare(gpu, orc, Lx, Ly, tensors=False, tag=f"product D={D}")


def test_heisenberg_from_noisy_neel(lib):
    Lx = Ly = 2
    N, D = 4, 3
    rng = np.random.default_rng(3)
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    G0 = wl.product_itps([up, dn, dn, up], D)
    G0 = [g + 0.05 * rng.standard_normal(g.shape) for g in G0]
    ones = [np.ones(D) for _ in range(N)]
    H = uniform_H(wl.heisenberg_bond(), N)
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.02, Lx, Ly, D, 2, 30)
    compare(gpu, orc, Lx, Ly, tensors=False, tag="heisenberg")
    assert gpu["e"] < -0.5          # below the Neel energy: quantum fluctuations


def test_d1_reaches_mean_field(lib):
    """D = 1 (one row per reduced tensor): the oracle's pinned limit."""
    Lx = Ly = 2
    N, h = 4, 2.0
    G0 = wl.product_itps([np.array([1.0, 0.0])] * N, 1)
    ones = [np.ones(1) for _ in range(N)]
    H = uniform_H(wl.tfim_bond(h), N)
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.01, Lx, Ly, 1, 2, 800)
    compare(gpu, orc, Lx, Ly, tensors=False, tag="D=1")
    _, emf = wl.tfim_mean_field(h)
    assert abs(gpu["e"] - emf) < 1e-4


def test_largest_shape_d8(lib):
    """D = 8, d = 2: 512 x 16 reduced tensors, the largest LDS class."""
    Lx = Ly = 2
    N, D = 4, 8
    G0 = wl.random_itps(Lx, Ly, D, 2, seed=8)
    ones = [np.ones(D) for _ in range(N)]
    H = uniform_H(wl.tfim_bond(3.0), N)
    gpu, orc = run_both(lib, G0, ones, ones, H, 0.01, Lx, Ly, D, 2, 1)
    compare(gpu, orc, Lx, Ly, tag="D=8")


def test_zero_steps_and_zero_tau(lib):
    """nsteps = 0 leaves the state as given; tau = 0 (identity gates) still
    truncates and re-gauges every bond, as the oracle does."""
    Lx = Ly = 2
    N, D = 4, 2
    G0 = wl.random_itps(Lx, Ly, D, 2, seed=31)
    rng = np.random.default_rng(31)
    lam0 = rng.uniform(0.3, 1.0, size=(N, 2, D))
    s = lib.SimpleUpdate(np.stack(G0)[None], lam0[None], Lx, Ly, D)
    s.set_hamiltonians(np.asarray(uniform_H(wl.tfim_bond(3.0), N))[None], 0.0)
    s.run(0)
    g, lm = s.get()
    assert np.array_equal(g[0], np.stack(G0)) and np.array_equal(lm[0], lam0)
    s.free()
    lh0 = [lam0[i, 0] for i in range(N)]
    lv0 = [lam0[i, 1] for i in range(N)]
    gpu, orc = run_both(lib, G0, lh0, lv0, uniform_H(wl.tfim_bond(3.0), N), 0.0, Lx, Ly, D, 2, 3)
    compare(gpu, orc, Lx, Ly, tag="tau=0")


def test_mfe_of_a_given_state(lib):
    """The mean-field contraction alone: same stored state (random tensors,
    random weights) on both sides, every density matrix and the energy."""
    Lx, Ly, D, d = 2, 3, 3, 2
    N = Lx * Ly
    G0 = wl.random_itps(Lx, Ly, D, d, seed=77)
    rng = np.random.default_rng(77)
    lam0 = rng.uniform(0.1, 1.0, size=(N, 2, D))
    lh0 = [lam0[i, 0] for i in range(N)]
    lv0 = [lam0[i, 1] for i in range(N)]
    H = [[wl.tfim_bond(2.5), wl.heisenberg_bond()] for _ in range(N)]
    s = lib.SimpleUpdate(np.stack(G0)[None], lam0[None], Lx, Ly, D, d=d)
    s.set_hamiltonians(np.asarray(H)[None], 0.01)
    r1, r2 = s.mfe()
    onsite = 0.3 * SZ
    e, be = s.mfe_energy(onsite=onsite)
    s.free()
    for i in range(N):
        ro = su.mfe_rho_site(G0, lh0, lv0, Lx, Ly, i)
        assert np.abs(r1[0, i] - ro / np.trace(ro)).max() < 1e-12
        for direction in (0, 1):
            ro = su.mfe_rho_bond(G0, lh0, lv0, Lx, Ly, i, direction)
            assert np.abs(r2[0, i, direction] - ro / np.trace(ro)).max() < 1e-12
            assert abs(be[0, i, direction] - su.expect(ro, H[i][direction])) < 1e-12
    eo = su.mfe_energy(G0, lh0, lv0, Lx, Ly, H, onsite=onsite)
    assert abs(e[0] - eo) < 1e-12


def test_commuting_gates_feed_ctmrg_to_onsager(lib):
    """End to end on the GPU: commuting Ising gates from |+x> (exact, bond
    dimension 2), the iTPS handed to the CTMRG library through device memory,
    <sz sz> against Onsager at beta = 2 N tau."""
    import torch
    Lx = Ly = 2
    N, D, tau, n = 4, 2, 0.05, 3
    G0 = wl.product_itps([np.array([1.0, 1.0]) / math.sqrt(2)] * N, D)
    ones = np.ones((1, N, 2, D))
    s = lib.SimpleUpdate(np.stack(G0)[None], ones, Lx, Ly, D)
    s.set_hamiltonians(np.asarray(uniform_H(-np.kron(SZ, SZ), N))[None], tau)
    s.run(n)
    buf = torch.empty(N * D ** 4 * 2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.get_itps(device_ptr=buf.data_ptr())
    A = s.get_itps()[0]
    s.free()
    ctx = lib.Ctm(None, Lx, Ly, D, chi=24, device_ptr=buf.data_ptr())
    ctx.ctm_sweep(40, 1e-13)
    ref = cf.nn_correlator(2 * n * tau)
    for i in range(N):
        for direction in (0, 1):
            v = ctx.ctm_expect_2site(i, direction, np.kron(SZ, SZ))
            assert abs(v - ref) < 1e-10, (i, direction, v, ref)
    ctx.ctm_free()
    assert np.array_equal(buf.cpu().numpy().reshape(A.shape), A)


def test_full_size_scan_sampled(lib):
    """The benchmark's launch configuration (256 problems, D = 4, 2x2 cell,
    the paper's transverse-field Ising example over a field scan, tau = 0.01)
    for 100 steps; two problems against the oracle, every problem checked for
    normalised, sorted, non-negative weights and finite energies."""
    Lx = Ly = 2
    N, D, B, n = 4, 4, 256, 100
    hs = np.linspace(0.0, 2.5, B)
    G0 = wl.product_itps([np.array([1.0, 0.0])] * N, D)
    rng = np.random.default_rng(2)
    G0 = [g + 1e-3 * rng.standard_normal(g.shape) for g in G0]
    gam = np.broadcast_to(np.stack(G0)[None], (B, N) + G0[0].shape).copy()
    lam = np.ones((B, N, 2, D))
    H = np.stack([np.asarray(uniform_H(ex1_bond(h), N)) for h in hs])
    s = lib.SimpleUpdate(gam, lam, Lx, Ly, D)
    s.set_hamiltonians(H, 0.01)
    s.run(n)
    g, lm = s.get()
    e, _ = s.mfe_energy()
    s.free()
    assert np.all(np.isfinite(e))
    assert np.all(lm >= 0) and np.all(np.diff(lm, axis=-1) <= 0)
    assert np.abs(np.sum(lm * lm, axis=-1) - 1).max() < 1e-12
    for b in (37, 201):
        ones = [np.ones(D) for _ in range(N)]
        Go, lho, lvo = su.simple_update(G0, ones, ones, list(H[b]), 0.01, Lx, Ly, n)
        gpu = dict(G=list(g[b]), lh=[lm[b, i, 0] for i in range(N)], lv=[lm[b, i, 1] for i in range(N)], e=e[b])
        orc = dict(G=Go, lh=lho, lv=lvo, e=su.mfe_energy(Go, lho, lvo, Lx, Ly, list(H[b])))
        compare(gpu, orc, Lx, Ly, tag=f"scan problem {b} (h = {hs[b]:.3f})")


def test_invalid_arguments(lib):
    from paper_2112_13184_amd._binding import CTM_EINVAL, CTM_ENUMERIC, CtmError
    G = np.zeros((1, 2, 2, 2, 2, 2, 2))
    lam = np.ones((1, 2, 2, 2))
    with pytest.raises(CtmError) as ex:
        lib.SimpleUpdate(G, lam, 2, 1, 2)               # Ly = 1: a bond would join a tensor to itself
    assert ex.value.status == CTM_EINVAL
    G8 = np.zeros((1, 4) + (8,) * 4 + (3,))
    with pytest.raises(CtmError) as ex:
        lib.SimpleUpdate(G8, np.ones((1, 4, 2, 8)), 2, 2, 8, d=3)   # core of 72 columns
    assert ex.value.status == CTM_EINVAL
    G0 = np.stack(wl.random_itps(2, 2, 2, 2, seed=1))[None]
    s = lib.SimpleUpdate(G0, np.ones((1, 4, 2, 2)), 2, 2, 2)
    with pytest.raises(CtmError) as ex:
        s.run(1)                                        # no Hamiltonians yet
    assert ex.value.status == CTM_EINVAL
    Hbad = np.asarray(uniform_H(wl.tfim_bond(3.0), 4))[None].copy()
    Hbad[0, 1, 0, 2, 2] = np.nan
    with pytest.raises(CtmError) as ex:
        s.set_hamiltonians(Hbad, 0.01)
    assert ex.value.status == CTM_EINVAL
    s.free()
    z = lib.SimpleUpdate(np.zeros_like(G0), np.ones((1, 4, 2, 2)), 2, 2, 2)
    z.set_hamiltonians(np.asarray(uniform_H(wl.tfim_bond(3.0), 4))[None], 0.01)
    with pytest.raises(CtmError) as ex:
        z.run(1)                                        # a zero state has no singular values
    assert ex.value.status == CTM_ENUMERIC
    z.free()


def test_field_scan_pipeline_trends_and_ctmrg_parity(lib):
    """The paper's transverse-field Ising example end to end on the GPU
    (simple update, iTPS into CTMRG in device memory): |<S^z>| = 1/2 at h = 0
    and falls monotonically with h while <S^x> rises, both saturating; the
    GPU CTMRG observables of one field match the oracle CTMRG run on the same
    simple-update tensors."""
    import torch
    from oracle import observables as ob
    from oracle.ctmrg import Environment
    hs = np.array([0.0, 0.6, 1.2, 1.5, 1.8, 2.5])
    B, D, chi = len(hs), 2, 10
    rng = np.random.default_rng(2)
    G0 = [g + 1e-3 * rng.standard_normal(g.shape) for g in wl.product_itps([np.array([1.0, 0.0])] * 4, D)]
    gam = np.broadcast_to(np.stack(G0)[None], (B, 4) + G0[0].shape).copy()
    H = np.stack([np.asarray(uniform_H(ex1_bond(h), 4)) for h in hs])
    s = lib.SimpleUpdate(gam, np.ones((B, 4, 2, D)), 2, 2, D)
    s.set_hamiltonians(H, 0.01)
    s.run(600)
    per = 4 * D ** 4 * 2
    buf = torch.empty(B * per, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.get_itps(device_ptr=buf.data_ptr())
    A = s.get_itps()
    s.free()
    sz, sx = [], []
    for b in range(B):
        ctx = lib.Ctm(None, 2, 2, D, chi=chi, device_ptr=buf.data_ptr() + 8 * b * per, rsvd_oversample=32)
        ctx.ctm_sweep(10, 0.0)
        sz.append(np.mean([abs(ctx.ctm_expect_1site(i, 0.5 * SZ)) for i in range(4)]))
        sx.append(np.mean([ctx.ctm_expect_1site(i, 0.5 * SX) for i in range(4)]))
        if b == 3:
            env = Environment([np.array(a) for a in A[b]], 2, 2, chi=chi, oversample=32)
            for _ in range(10):
                env.sweep()
            for i in range(4):
                ro = ob.rho_one_site(env, i)
                assert abs(ctx.ctm_expect_1site(i, 0.5 * SX) - ob.expect(ro, 0.5 * SX)) < 1e-10
                assert abs(ctx.ctm_expect_1site(i, 0.5 * SZ) - ob.expect(ro, 0.5 * SZ)) < 1e-10
        ctx.ctm_free()
    print("h", hs, "|Sz|", np.round(sz, 4), "Sx", np.round(sx, 4))
    assert abs(sz[0] - 0.5) < 1e-6 and abs(sx[0]) < 1e-3
    assert all(a > b for a, b in zip(sz, sz[1:]))
    assert all(a < b for a, b in zip(sx, sx[1:]))
    assert sz[-1] < 0.02 and sx[-1] > 0.45


SY = np.array([[0.0, -1.0j], [1.0j, 0.0]])


def _complex_problem(D, seed, d=2):
    rng = np.random.default_rng(seed)
    G0 = [(rng.standard_normal((D,) * 4 + (d,)) + 1j * rng.standard_normal((D,) * 4 + (d,))) for _ in range(4)]
    G0 = [g / np.abs(g).max() for g in G0]
    H = []
    for _ in range(4):
        row = []
        for _ in range(2):
            X = rng.standard_normal((d * d, d * d)) + 1j * rng.standard_normal((d * d, d * d))
            row.append(0.5 * (X + X.conj().T))
        H.append(row)
    return G0, H


@pytest.mark.parametrize("D", [2, 3])
def test_complex_random_state_parity(lib, D):
    """Complex tensors and a random complex Hermitian Hamiltonian per bond:
    weights, tensors (with the full weights) and energies against the
    oracle."""
    Lx = Ly = 2
    N = 4
    G0, H = _complex_problem(D, 50 + D)
    ones = [np.ones(D) for _ in range(N)]
    lam = np.ones((1, N, 2, D))
    s = lib.SimpleUpdate(np.stack(G0)[None], lam, Lx, Ly, D, complex_tensors=True)
    s.set_hamiltonians(np.asarray(H)[None], 0.02)
    s.run(10)
    g, lm = s.get()
    e, _ = s.mfe_energy()
    r1, r2 = s.mfe()
    s.free()
    Go, lho, lvo = su.simple_update(G0, ones, ones, H, 0.02, Lx, Ly, 10)
    gpu = dict(G=list(g[0]), lh=[lm[0, i, 0] for i in range(N)], lv=[lm[0, i, 1] for i in range(N)], e=e[0])
    orc = dict(G=Go, lh=lho, lv=lvo, e=su.mfe_energy(Go, lho, lvo, Lx, Ly, H))
    compare(gpu, orc, Lx, Ly, tag=f"complex D={D}")
    for i in range(N):
        ro = su.mfe_rho_site(Go, lho, lvo, Lx, Ly, i)
        assert np.abs(r1[0, i] - ro / np.trace(ro)).max() < 1e-10
        rb = su.mfe_rho_bond(Go, lho, lvo, Lx, Ly, i, 1)
        assert np.abs(r2[0, i, 1] - rb / np.trace(rb)).max() < 1e-10


def test_complex_field_along_y(lib):
    h, tau, n = 0.9, 0.05, 8
    Hy = -0.25 * h * (np.kron(SY, wl.ID2) + np.kron(wl.ID2, SY))
    G0 = np.stack(wl.product_itps([np.array([1.0, 0.0])] * 4, 2)).astype(complex)
    s = lib.SimpleUpdate(G0[None], np.ones((1, 4, 2, 2)), 2, 2, 2, complex_tensors=True)
    s.set_hamiltonians(np.asarray(uniform_H(Hy, 4))[None], tau)
    s.run(n)
    r1, _ = s.mfe()
    s.free()
    for i in range(4):
        assert abs(np.real(np.trace(r1[0, i] @ SY)) - math.tanh(2 * n * tau * h)) < 1e-12   # sum rho[in][out] O[out][in]


def test_complex_local_unitary_rotation_matches_the_real_problem(lib):
    """The local-unitary pin of the oracle, on the GPU: a real problem and its
    rotation by U_s = diag(1, exp(i phi_s)) give the same weights and energies."""
    Lx = Ly = 2
    N, D = 4, 2
    A = wl.random_itps(Lx, Ly, D, 2, seed=13)
    Hb = wl.tfim_bond(2.5)
    H = uniform_H(Hb, N)
    lam = np.ones((1, N, 2, D))
    sr = lib.SimpleUpdate(np.stack(A)[None], lam, Lx, Ly, D)
    sr.set_hamiltonians(np.asarray(H)[None], 0.02)
    sr.run(15)
    _, lmr = sr.get()
    er, _ = sr.mfe_energy()
    sr.free()
    Us = [np.diag([1.0, np.exp(1j * p)]) for p in (0.3, 1.1, -0.7, 2.0)]
    Ac = np.stack([np.einsum("PQ,lurdQ->lurdP", Us[s], A[s]) for s in range(N)])
    Hc = []
    for s in range(N):
        row = []
        for direction in (0, 1):
            i, _, j, _ = su.bond(Lx, Ly, s, direction)
            UU = np.kron(Us[i], Us[j])
            row.append(UU @ Hb @ UU.conj().T)
        Hc.append(row)
    sc = lib.SimpleUpdate(Ac[None], lam, Lx, Ly, D, complex_tensors=True)
    sc.set_hamiltonians(np.asarray(Hc)[None], 0.02)
    sc.run(15)
    _, lmc = sc.get()
    ec, _ = sc.mfe_energy()
    sc.free()
    assert np.abs(lmc - lmr).max() < 1e-12
    assert abs(ec[0] - er[0]) < 1e-12


def test_complex_mode_on_real_data_equals_the_real_path(lib):
    Lx = Ly = 2
    N, D = 4, 3
    A = np.stack(wl.random_itps(Lx, Ly, D, 2, seed=23))
    H = np.asarray(uniform_H(wl.tfim_bond(3.0), N))
    lam = np.ones((1, N, 2, D))
    out = []
    for cplx in (False, True):
        s = lib.SimpleUpdate(A[None], lam, Lx, Ly, D, complex_tensors=cplx)
        s.set_hamiltonians(H[None], 0.01)
        s.run(10)
        g, lm = s.get()
        e, _ = s.mfe_energy()
        s.free()
        out.append((g, lm, e))
    assert np.abs(out[1][1] - out[0][1]).max() < 1e-13
    assert abs(out[1][2][0] - out[0][2][0]) < 1e-13
    assert np.abs(out[1][0].imag).max() < 1e-13
    w = [su.weighted(list(o[0][0]), [o[1][0, i, 0] for i in range(N)], [o[1][0, i, 1] for i in range(N)], Lx, Ly)
         for o in out]
    assert max(float(np.abs(a - b).max()) for a, b in zip(w[0], w[1])) < 1e-11
