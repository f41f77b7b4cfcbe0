"""Full update: HIP library (C ABI) against the FP64 oracle.

Both sides hold the same tensors and an environment built by the same number
of CTMRG sweeps; the sketch of the randomized SVD covers every cut
(k = chi + p >= chi D^2), so the environment does not depend on the random
numbers.  The GPU takes rocSOLVER's QR, SVD and symmetric eigensolver and
MFMA GEMMs, the oracle LAPACK through NumPy, so results agree to rounding
amplified by the conditioning of the ALS solves and of the CTMRG
truncation.  Bounds: tensors (sign-fixed, max-abs normalised) 1e-8 relative
to the largest entry; energies 1e-9.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as wl
from oracle import closed_forms as cf
from oracle import full_update as fu
from oracle import observables as ob
from oracle.ctmrg import Environment

pytestmark = pytest.mark.gpu

LX = LY = 2
N = LX * LY
SZ = wl.SZ


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


def both(lib, A, D, chi, p, sweeps):
    ctx = lib.Ctm(A, LX, LY, D, chi=chi, rsvd_oversample=p)
    ctx.ctm_sweep(sweeps, 0.0)
    env = Environment([np.array(a) for a in A], LX, LY, chi=chi, oversample=p)
    for _ in range(sweeps):
        env.sweep()
    return ctx, env


def energy(env, Hb):
    return ob.energy_per_site(env, Hb)


def gpu_energy(ctx, Hb):
    return sum(ctx.ctm_expect_2site(i, dr, Hb) for i in range(N) for dr in (0, 1)) / N


@pytest.mark.parametrize("direction_first", [True])
def test_one_step_random_state_parity(lib, direction_first):
    D, chi, p = 2, 8, 32
    A = wl.random_itps(LX, LY, D, 2, seed=12)
    ctx, env = both(lib, A, D, chi, p, 8)
    Hb = wl.tfim_bond(3.0)
    H = [[Hb, Hb] for _ in range(N)]
    ctx.ctm_fu_step(np.asarray(H), 0.05, als_iters=3, env_sweeps=1)
    fu.full_update_step(env, H, 0.05, als_iters=3, env_sweeps=1)
    G = ctx.ctm_get_tensors()
    dt = max(float(np.abs(G[i] - env.A[i]).max() / np.abs(env.A[i]).max()) for i in range(N))
    e_gpu, e_orc = gpu_energy(ctx, Hb), energy(env, Hb)
    print(f"tensors {dt:.2e}, energy {abs(e_gpu - e_orc):.2e}")
    ctx.ctm_free()
    assert dt < 1e-8
    assert abs(e_gpu - e_orc) < 1e-9


def test_two_steps_heisenberg_parity(lib):
    D, chi, p = 2, 8, 32
    rng = np.random.default_rng(6)
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    A = [a + 0.1 * rng.standard_normal(a.shape) for a in wl.product_itps([up, dn, dn, up], D)]
    ctx, env = both(lib, A, D, chi, p, 6)
    Hb = wl.heisenberg_bond()
    H = [[Hb, Hb] for _ in range(N)]
    for _ in range(2):
        ctx.ctm_fu_step(np.asarray(H), 0.05, als_iters=2, env_sweeps=1)
        fu.full_update_step(env, H, 0.05, als_iters=2, env_sweeps=1)
    G = ctx.ctm_get_tensors()
    dt = max(float(np.abs(G[i] - env.A[i]).max() / np.abs(env.A[i]).max()) for i in range(N))
    e_gpu, e_orc = gpu_energy(ctx, Hb), energy(env, Hb)
    print(f"tensors {dt:.2e}, energy {abs(e_gpu - e_orc):.2e}, energy {e_gpu:.6f}")
    ctx.ctm_free()
    assert dt < 1e-8
    assert abs(e_gpu - e_orc) < 1e-9


def test_spin_one_odd_order_parity(lib):
    """d = 3, D = 3: the ALS normal matrices have odd order r D = 27 (the
    padded path of the one-workgroup eigensolver), the bond environment order
    r^2 = 81 (rocSOLVER's).  A random symmetric two-site Hamiltonian, one step
    against the oracle; the sketch covers every cut (k = chi + p >= chi D^2)."""
    D, d, chi, p = 3, 3, 12, 96
    A = wl.random_itps(LX, LY, D, d, seed=21)
    ctx = lib.Ctm(A, LX, LY, D, chi=chi, d=d, rsvd_oversample=p)
    ctx.ctm_sweep(4, 0.0)
    env = Environment([np.array(a) for a in A], LX, LY, chi=chi, oversample=p)
    for _ in range(4):
        env.sweep()
    rng = np.random.default_rng(4)
    Hd = rng.standard_normal((d * d, d * d))
    Hd = Hd + Hd.T
    H = [[Hd, Hd] for _ in range(N)]
    ctx.ctm_fu_step(np.asarray(H), 0.02, als_iters=2, env_sweeps=1)
    fu.full_update_step(env, H, 0.02, als_iters=2, env_sweeps=1)
    G = ctx.ctm_get_tensors()
    dt = max(float(np.abs(G[i] - env.A[i]).max() / np.abs(env.A[i]).max()) for i in range(N))
    e_gpu, e_orc = gpu_energy(ctx, Hd), energy(env, Hd)
    print(f"tensors {dt:.2e}, energy {abs(e_gpu - e_orc):.2e}")
    ctx.ctm_free()
    assert dt < 1e-8
    assert abs(e_gpu - e_orc) < 1e-9


def test_commuting_ising_gates_reach_onsager(lib):
    D, chi, p = 2, 16, 48
    tau, n = 0.05, 3
    Hz = -np.kron(SZ, SZ)
    A = wl.product_itps([np.array([1.0, 1.0]) / math.sqrt(2)] * N, D)
    ctx = lib.Ctm(A, LX, LY, D, chi=chi, rsvd_oversample=p)
    ctx.ctm_sweep(2, 0.0)
    for _ in range(n):
        ctx.ctm_fu_step(np.asarray([[Hz, Hz]] * N), tau, als_iters=3, env_sweeps=2)
    ctx.ctm_sweep(25, 0.0)
    ref = cf.nn_correlator(2 * n * tau)
    for i in range(N):
        for dr in (0, 1):
            v = ctx.ctm_expect_2site(i, dr, np.kron(SZ, SZ))
            assert abs(v - ref) < 1e-9, (i, dr, v, ref)
    ctx.ctm_free()


def test_isolated_dimers_follow_the_exact_evolution(lib):
    rng = np.random.default_rng(5)
    Hd = rng.standard_normal((4, 4))
    Hd = Hd + Hd.T
    phis = [rng.standard_normal(2) for _ in range(N)]
    tau, n = 0.03, 4
    Z = np.zeros((4, 4))
    H = np.asarray([[Hd if s in (0, 2) else Z, Z] for s in range(N)])
    ctx = lib.Ctm(wl.product_itps(phis, 2), LX, LY, 2, chi=8, rsvd_oversample=32)
    ctx.ctm_sweep(2, 0.0)
    for _ in range(n):
        ctx.ctm_fu_step(H, tau, als_iters=2, env_sweeps=1)
    ctx.ctm_sweep(5, 0.0)
    for s in (0, 2):
        psi = expm(-n * tau * Hd) @ np.kron(phis[s], phis[s + 1])
        psi = psi / np.linalg.norm(psi)
        rho = ctx.ctm_rho_2site(s, 0)
        assert np.abs(rho - np.outer(psi, psi)).max() < 1e-12
    ctx.ctm_free()


def test_invalid_arguments(lib):
    from paper_2112_13184_amd._binding import CTM_EINVAL, CtmError
    A = wl.random_itps(LX, LY, 2, 2, seed=1)
    H = np.asarray([[wl.tfim_bond(3.0)] * 2] * N)
    ctx = lib.Ctm(A, LX, LY, 2, chi=8, prec="bf16")
    with pytest.raises(CtmError) as ex:
        ctx.ctm_fu_step(H, 0.01)
    assert ex.value.status == CTM_EINVAL
    ctx.ctm_free()
    A1 = wl.random_itps(1, 2, 2, 2, seed=1)
    ctx = lib.Ctm(A1, 1, 2, 2, chi=8)
    with pytest.raises(CtmError) as ex:
        ctx.ctm_fu_step(np.asarray([[wl.tfim_bond(3.0)] * 2] * 2), 0.01)
    assert ex.value.status == CTM_EINVAL
    ctx.ctm_free()
    ctx = lib.Ctm(A, LX, LY, 2, chi=8)
    Hbad = H.copy()
    Hbad[0, 0, 1, 1] = np.nan
    with pytest.raises(CtmError) as ex:
        ctx.ctm_fu_step(Hbad, 0.01)
    assert ex.value.status == CTM_EINVAL
    with pytest.raises(CtmError) as ex:
        ctx.ctm_fu_step(H, -0.01)
    assert ex.value.status == CTM_EINVAL
    ctx.ctm_free()
