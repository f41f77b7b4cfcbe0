"""GPU (HIP, through the C ABI) against the FP64 CPU oracle on the same seeded inputs.

Tolerances (FP64 everywhere on both sides; only summation order differs):
* single contractions (enlarged corner): 1e-12 relative to the largest entry;
* projectors and one move: 1e-8 relative (the projector divides by
  sqrt(sigma_i) down to the cutoff, which amplifies rounding by up to
  sqrt(sigma_0 / sigma_chi));
* energies and other observables of runs whose answer is fixed to that level
  (converged transverse-field Ising requests, the gauged Ising PEPS, product
  states, classical Ising): 1e-10 absolute;
* energies after a fixed number of sweeps from the trivial boundary of random
  tensors: 1e-10, unless the oracle itself moves by more than that when every
  entry of its input tensors is moved by one unit in the last place.  Such a
  run amplifies rounding through near-degenerate truncations (several results
  are then correct); the bound becomes 10x that measured one-ulp spread, and
  every such test prints |GPU - oracle|, the spread and their ratio.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import closed_forms as cf
from oracle import observables as ob
from oracle.ctmrg import Environment, enlarged_corner, projectors
from oracle.philox import stream_id
from tests._util import inject, load_state, pad_to, random_env, rel_err, ulp_perturbed

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


# --------------------------------------------------------------------------
# single building blocks on an injected environment
# --------------------------------------------------------------------------
# D = 2, 3, 4: the one-tile absorption; D = 5: two tiles; D = 6: three
@pytest.mark.parametrize("layers,D,chi", [(2, 3, 13), (2, 2, 20), (2, 4, 9), (2, 5, 7), (2, 6, 5), (1, 3, 21)])
def test_enlarged_corner_parity(lib, layers, D, chi):
    d = 2 if layers == 2 else 1
    Db = D * D if layers == 2 else D
    if layers == 2:
        A = wl.random_itps(2, 2, D, d, seed=5)
    else:
        A = wl.random_classical(2, 2, D, seed=5, positive=False)
    ctx = lib.Ctm(A, 2, 2, D, chi, d=d, layers=layers, rsvd_oversample=8)
    ora = Environment(A, 2, 2, chi=chi, layers=layers)
    env = random_env(2, 2, chi, Db, seed=7)
    inject(ora, ctx, env)
    for site in range(4):
        for j in range(4):
            G = ctx.ctm_enlarged_corner(j, site)
            ref = ora.corner(site, j)
            assert rel_err(G, ref) < 1e-12, (site, j)


def test_d8_chi256_enlarged_corner_blocks(lib):
    """The D=8, chi=256 configuration (double-layer bond 64, n = 16384), the
    largest shape of the fused absorption kernel (four tiles per pair, one
    wave per SIMD): sampled blocks of two corners (3 next-leg indices by 3
    prev-leg indices, all ket/bra pairs of each) against the oracle's
    definition (Sec. 2.2) evaluated on the same slices, 1e-12 relative."""
    D, chi = 8, 256
    Db = D * D
    A = wl.random_itps(2, 2, D, 2, seed=3)
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=64, rsvd_power_iters=1, seed=12)
    ora = Environment(A, 2, 2, chi=chi, layers=2)
    inject(ora, ctx, random_env(2, 2, chi, Db, seed=9))
    rng = np.random.default_rng(0)
    for site, j in ((0, 0), (3, 2)):
        G = ctx.ctm_enlarged_corner(j, site)
        assert G.shape == (chi * Db, chi * Db)
        cn = np.sort(rng.choice(chi, 3, replace=False))
        cp = np.sort(rng.choice(chi, 3, replace=False))
        C, Tn, Tp = ora.C[site][j], ora.T[site][j], ora.T[site][(j - 1) % 4]
        ref = enlarged_corner(C, Tn[:, cn, :], Tp[cp, :, :], ora.site(site, j), 2)
        rows = (cn[:, None] * Db + np.arange(Db)).reshape(-1)
        cols = (cp[:, None] * Db + np.arange(Db)).reshape(-1)
        assert rel_err(G[np.ix_(rows, cols)], ref) < 1e-12, (site, j)
        del G


@pytest.mark.parametrize("mode", ["rsvd", "dense", "householder"])
def test_projectors_parity(lib, mode):
    """Projectors of every cut of every move direction on an injected random
    environment: the batched path (Cholesky QR + Jacobi), the exact SVD of the
    formed cluster matrix, and the Householder QR + library SVD path that a
    cut takes when k > 320 or the batched factorisation fails (forced here
    through projector_path)."""
    D, chi, p, q, seed = 2, 10, 6, 2, 21
    A = wl.random_itps(2, 2, D, 2, seed=6)
    kw = dict(rsvd_oversample=(-1 if mode == "dense" else p), rsvd_power_iters=q, seed=seed,
              projector_path=("householder" if mode == "householder" else "auto"))
    ctx = lib.Ctm(A, 2, 2, D, chi, **kw)
    omode = "dense" if mode == "dense" else "rsvd"
    ora = Environment(A, 2, 2, chi=chi, layers=2, mode=omode, oversample=p, power_iters=q, seed=seed)
    inject(ora, ctx, random_env(2, 2, chi, D * D, seed=8))
    Db = D * D
    for direction, r in (("left", 0), ("up", 1), ("right", 2), ("down", 3)):
        for x in range(2):
            for y in range(2):
                P, Pt, k = ctx.ctm_projectors(direction, x, y)
                from oracle.ctmrg import view_site
                vs = lambda a, b: view_site(2, 2, r, a, b)
                G_ul = ora.corner(vs(x, y), (0 + r) % 4)
                G_ur = ora.corner(vs(x + 1, y), (1 + r) % 4)
                G_lr = ora.corner(vs(x + 1, y - 1), (2 + r) % 4)
                G_ll = ora.corner(vs(x, y - 1), (3 + r) % 4)
                Pr, Ptr = projectors(G_ur, G_ul, G_ll, G_lr, chi, 1e-12, omode, p, q, seed,
                                     stream_id(0, x, y), G_lr.shape[1] // Db, Db)
                scale = np.max(np.abs(Ptr @ Pr))
                assert np.max(np.abs(Pt @ P - Ptr @ Pr)) / scale < 1e-8
                assert rel_err(P, Pr) < 1e-8 and rel_err(Pt, Ptr) < 1e-8
                assert k == chi
    # every cut went through the path under test
    assert ctx.ctm_cut_stats()[1 if mode == "rsvd" else 2] == 16


def test_graded_cut_after_growth(lib):
    """Cuts whose kept singular values fall to ~1e-9 of the largest (the state
    after one sweep from the trivial boundary, D=2, chi=16): the projected
    product H_u Pt P H_d^T must keep every direction above the cutoff, and one
    move must give the oracle's energy."""
    D, chi = 2, 16
    A = wl.random_itps(2, 2, D, 2, seed=14)
    ora = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=8, power_iters=1, seed=5)
    ora.sweep()
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=8, rsvd_power_iters=1, seed=5)
    load_state(ctx, ora)
    from oracle.ctmrg import view_site
    Db = D * D
    for x in range(2):
        for y in range(2):
            vs = lambda a, b: view_site(2, 2, 0, a, b)
            G_ul, G_ur = ora.corner(vs(x, y), 0), ora.corner(vs(x + 1, y), 1)
            G_lr, G_ll = ora.corner(vs(x + 1, y - 1), 2), ora.corner(vs(x, y - 1), 3)
            na = G_ul.shape[1]
            if na <= chi:
                continue
            H_u, H_dT = G_ur @ G_ul, G_ll @ G_lr
            Pr, Ptr = projectors(G_ur, G_ul, G_ll, G_lr, chi, 1e-12, "rsvd", 8, 1, 5, stream_id(0, x, y),
                                 G_lr.shape[1] // Db, Db)
            P, Pt, _ = ctx.ctm_projectors("left", x, y)
            nc = na // Db
            P = P.reshape(chi, chi, Db)[:, :nc, :].reshape(chi, na)
            Pt = Pt.reshape(chi, Db, chi)[:nc].reshape(na, chi)
            ref = H_u @ Ptr @ Pr @ H_dT
            got = H_u @ Pt @ P @ H_dT
            assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref)), (x, y)
    assert ctx.ctm_cut_stats()[1] > 0 and ctx.ctm_cut_stats()[2] == 0
    H = wl.heisenberg_bond()
    ctx.ctm_move("left")
    ora.left_move(0)
    assert abs(_gpu_energy(ctx, H, 4) - ob.energy_per_site(ora, H)) < 1e-10


@pytest.mark.parametrize("direction,r", [("left", 0), ("up", 1), ("right", 2), ("down", 3)])
def test_one_move_parity(lib, direction, r):
    D, chi = 2, 9
    A = wl.random_itps(2, 2, D, 2, seed=9)
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=6, rsvd_power_iters=2, seed=3)
    ora = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=6, power_iters=2, seed=3)
    inject(ora, ctx, random_env(2, 2, chi, D * D, seed=10))
    ctx.ctm_move(direction)
    ora.left_move(r)
    assert ctx.ctm_cut_stats() == (0, 4, 0)
    for i in range(4):
        C, T, _ = ctx.ctm_get_env(i)
        for k in range(4):
            assert rel_err(C[k], ora.C[i][k]) < 1e-8, (i, k)
            assert rel_err(T[k], ora.T[i][k]) < 1e-8, (i, k)


@pytest.mark.parametrize("D,chi,p,path", [(2, 9, 6, "householder"), (2, 300, 32, "auto")])
def test_one_move_householder_path(lib, D, chi, p, path):
    """One left move through the Householder QR + library SVD projectors:
    forced by projector_path at a small shape, and taken by itself at
    k = chi + p = 332 > 320, beyond the batched factorisation.  Every
    renormalised tensor against the oracle's move, 1e-8 as for the batched
    path."""
    q = 1
    A = wl.random_itps(2, 2, D, 2, seed=9)
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=p, rsvd_power_iters=q, seed=3, projector_path=path)
    ora = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=p, power_iters=q, seed=3)
    inject(ora, ctx, random_env(2, 2, chi, D * D, seed=10))
    ctx.ctm_move("left")
    ora.left_move(0)
    assert ctx.ctm_cut_stats() == (0, 0, 4)
    for i in range(4):
        C, T, _ = ctx.ctm_get_env(i)
        for k in range(4):
            assert rel_err(C[k], ora.C[i][k]) < 1e-8, (i, k)
            assert rel_err(T[k], ora.T[i][k]) < 1e-8, (i, k)


def test_one_move_batched_corner_chunks(lib):
    """One left move at D = 4, chi = 144 (n = 2304) from a random
    full-dimension environment: n^2 is large enough that a batched corner
    launch takes 6 of the 8 corners of a column (two launches per column,
    each corner with its own scratch), the column update runs as one batched
    launch over both cuts.  Every renormalised tensor against the oracle's
    move, 1e-8 as for the small one-move test."""
    D, chi, p, q = 4, 144, 32, 1
    A = wl.random_itps(2, 2, D, 2, seed=9)
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=p, rsvd_power_iters=q, seed=3)
    ora = Environment(A, 2, 2, chi=chi, layers=2, mode="rsvd", oversample=p, power_iters=q, seed=3)
    inject(ora, ctx, random_env(2, 2, chi, D * D, seed=10))
    ctx.ctm_move("left")
    ora.left_move(0)
    assert ctx.ctm_cut_stats() == (0, 4, 0)
    for i in range(4):
        C, T, _ = ctx.ctm_get_env(i)
        for k in range(4):
            assert rel_err(C[k], ora.C[i][k]) < 1e-8, (i, k)
            assert rel_err(T[k], ora.T[i][k]) < 1e-8, (i, k)


# --------------------------------------------------------------------------
# whole runs from the trivial environment
# --------------------------------------------------------------------------
def _gpu_energy(ctx, H, N):
    e = 0.0
    for i in range(N):
        e += ctx.ctm_expect_2site(i, 0, H) + ctx.ctm_expect_2site(i, 1, H)
    return e / N


def _oracle_run(A, Lx, Ly, chi, sweeps):
    env = Environment(A, Lx, Ly, chi=chi, layers=2, mode="rsvd", oversample=8, power_iters=1, seed=5)
    for _ in range(sweeps):
        env.sweep()
    return env


def _spectra(Cs, chi):
    out = []
    for C in Cs:
        s = np.linalg.svd(pad_to(C, (chi, chi)), compute_uv=False)
        out.append(s / s.sum())
    return np.array(out)


def _bound(diff, spread, what):
    """1e-10, or 10x the oracle's one-ulp spread where that is larger; prints both."""
    tol = max(1e-10, 10.0 * spread)
    print(f"{what}: |gpu - oracle| = {diff:.2e}, one-ulp spread {spread:.2e}, ratio {diff / max(spread, 1e-300):.2f}, "
          f"bound {tol:.1e}")
    return tol


# (Lx, Ly, D, chi, tensor seed): random tensors from the trivial boundary,
# 6 sweeps.  The oracle's spread under one-ulp input perturbations (four
# seeds) is measured in the test; the GPU differs from the oracle by about
# that spread (ratio <= 2 on these runs).
@pytest.mark.parametrize("Lx,Ly,D,chi,seed", [(2, 2, 2, 16, 14), (1, 1, 2, 8, 14), (2, 1, 3, 17, 3),
                                              (2, 2, 3, 18, 14)])
def test_sweeps_energy_and_spectra(lib, Lx, Ly, D, chi, seed):
    sweeps = 6
    A = wl.random_itps(Lx, Ly, D, 2, seed=seed)
    ctx = lib.Ctm(A, Lx, Ly, D, chi, rsvd_oversample=8, rsvd_power_iters=1, seed=5)
    for _ in range(sweeps):
        for dname in ("left", "right", "up", "down"):
            ctx.ctm_move(dname)
    assert ctx.ctm_cut_stats()[2] == 0
    ora = _oracle_run(A, Lx, Ly, chi, sweeps)
    perturbed = [_oracle_run(ulp_perturbed(A, ps), Lx, Ly, chi, sweeps) for ps in range(4)]
    H = wl.heisenberg_bond()
    N = Lx * Ly
    e_ora = ob.energy_per_site(ora, H)
    sens_e = max(abs(e_ora - ob.energy_per_site(o, H)) for o in perturbed)
    diff = abs(_gpu_energy(ctx, H, N) - e_ora)
    assert diff < _bound(diff, sens_e, "energy per site")
    for i in range(N):
        C, T, dims = ctx.ctm_get_env(i)
        s_gpu, s_ora = _spectra(C, chi), _spectra(ora.C[i], chi)
        sens_s = max(np.max(np.abs(s_ora - _spectra(o.C[i], chi))) for o in perturbed)
        ds = np.max(np.abs(s_gpu - s_ora))
        assert ds < _bound(ds, sens_s, f"corner spectra, site {i}")
        rho = ctx.ctm_rho_1site(i)
        ref = ob.rho_one_site(ora, i)
        ref = ref / np.trace(ref)
        sens_r = max(np.max(np.abs(ref - ob.rho_one_site(o, i) / np.trace(ob.rho_one_site(o, i))))
                     for o in perturbed)
        dr = np.max(np.abs(rho - ref))
        assert dr < _bound(dr, sens_r, f"rho, site {i}")


def _tfim_golden():
    return _golden("tfim_converged")


@pytest.mark.parametrize("case", range(4))
def test_tfim_converged_matches_oracle(lib, case):
    """Transverse-field Ising states (mean-field state plus noise, D = 2 and 3,
    1x1 and 2x2 cells) after 40 sweeps, where both the oracle's and the GPU's
    energies have settled to about 1e-13: energy per site and <sigma_z> of
    every site against the stored oracle run, 1e-10."""
    g = _tfim_golden()
    w, c = g["params"], g["cases"][case]
    L, D, chi, h = c["L"], c["D"], c["chi"], c["h"]
    A = wl.tfim_request_tensors(h, D, L, L, w["eps"], seed=c["tensor_seed"])
    ctx = lib.Ctm(A, L, L, D, chi, rsvd_oversample=w["p"], rsvd_power_iters=w["q"], seed=w["sketch_seed"],
                  svd_rel_cutoff=g["cutoff"])
    n, delta, _ = ctx.ctm_sweep(w["sweeps"], 0.0)
    assert n == w["sweeps"] and ctx.ctm_cut_stats()[2] == 0
    e = _gpu_energy(ctx, wl.tfim_bond(h), L * L)
    ref = c["energies"][str(w["sweeps"])]
    dmz = max(abs(ctx.ctm_expect_1site(i, wl.SZ) - c["mz"][i]) for i in range(L * L))
    print(f"tfim L={L} D={D} chi={chi}: |dE| = {abs(e - ref):.2e}, max |d mz| = {dmz:.2e}, "
          f"delta gpu {delta:.1e} / oracle {c['delta_last']:.1e}")
    assert abs(e - ref) < 1e-10
    assert dmz < 1e-10


def test_ising_peps_gauged_2x2_matches_oracle(lib):
    """The Ising PEPS with a random gauge on every bond of a 2x2 cell (four
    different site tensors, the same state): run to delta < 1e-11 on both
    sides; <sigma_z sigma_z> on all eight bonds against the oracle, 1e-10, and
    against Onsager's nearest-neighbour correlator, 1e-9 (finite chi)."""
    g = _golden("ising_peps_2x2")
    A, _ = wl.ising_peps(g["beta"])
    ctx = lib.Ctm(wl.gauged_2x2(A, 2, seed=g["gauge_seed"]), 2, 2, 2, g["chi"], rsvd_oversample=g["p"],
                  rsvd_power_iters=g["q"], seed=g["sketch_seed"])
    n, delta, conv = ctx.ctm_sweep(400, g["tol"])
    assert conv, delta
    zz = np.kron(wl.SZ, wl.SZ)
    worst = 0.0
    for i in range(4):
        for dr in (0, 1):
            v = ctx.ctm_expect_2site(i, dr, zz)
            worst = max(worst, abs(v - g["zz"][i][dr]))
            assert abs(v - cf.nn_correlator(g["beta"])) < 1e-9
    print(f"gauged Ising PEPS: sweeps gpu {n} / oracle {g['sweeps']}, max |d zz| = {worst:.2e}")
    assert worst < 1e-10


@pytest.mark.parametrize("chi", [24, 130, 330])
def test_sweep_delta_is_the_corner_spectra_change(lib, chi):
    """The stop rule's measure (Sec. 2.2 convergence of the corner spectra):
    a sweep reports the largest, over corners, of sum |s_new - s_old| of the
    normalised singular values of each corner.  Checked against NumPy's SVD of
    the corners read back before and after the sweep; chi = 24 takes the
    one-workgroup Jacobi, chi = 130 the batched value-only Jacobi, chi = 330
    the library SVD."""
    A = wl.random_itps(2, 2, 3, 2, seed=11)
    ctx = lib.Ctm(A, 2, 2, 3, chi, rsvd_oversample=16, rsvd_power_iters=1, seed=3)
    for _ in range(2):
        ctx.ctm_sweep(1, 0.0)

    def spectra_all():
        return np.concatenate([_spectra(ctx.ctm_get_env(i)[0], chi) for i in range(4)])

    before = spectra_all()
    n, delta, _ = ctx.ctm_sweep(1, 0.0)
    after = spectra_all()
    ref = np.max(np.sum(np.abs(after - before), axis=1))
    assert n == 1
    assert ref > 1e-8
    assert abs(delta - ref) <= 1e-12 + 1e-9 * ref, (delta, ref)


def test_classical_ising_closed_forms(lib):
    beta = 0.5
    a, b, w = wl.ising_classical(beta)
    ctx = lib.Ctm([a], 1, 1, 2, 16, layers=1, boundary=w, rsvd_oversample=16, rsvd_power_iters=2, seed=5)
    n, delta, conv = ctx.ctm_sweep(400, 1e-12)
    assert conv, delta
    f = -ctx.ctm_log_kappa() / beta
    m = ctx.ctm_impurity(0, b)
    assert abs(f - (-cf.onsager_lnz(beta) / beta)) < 1e-8
    assert abs(m - cf.yang_magnetization(beta)) < 1e-5
    ora = Environment([a], 1, 1, chi=16, layers=1, boundary=w, mode="rsvd", oversample=16,
                      power_iters=2, seed=5)
    ora.run(400, 1e-12)
    assert abs(m - ob.impurity_ratio(ora, 0, b)) < 1e-10
    assert abs(ctx.ctm_log_kappa() - ob.log_kappa(ora)) < 1e-10


def test_ising_peps_closed_forms(lib):
    beta = 0.5
    A, wp = wl.ising_peps(beta)
    ctx = lib.Ctm([A], 1, 1, 2, 16, boundary=wp, rsvd_oversample=16, rsvd_power_iters=2, seed=2)
    ctx.ctm_sweep(400, 1e-11)
    zz = np.kron(wl.SZ, wl.SZ)
    assert abs(ctx.ctm_expect_2site(0, 0, zz) - cf.nn_correlator(beta)) < 1e-9
    assert abs(ctx.ctm_expect_2site(0, 1, zz) - cf.nn_correlator(beta)) < 1e-9
    assert abs(ctx.ctm_expect_1site(0, wl.SZ) - cf.yang_magnetization(beta)) < 1e-9
    assert abs(ctx.ctm_log_kappa() - cf.onsager_lnz(beta)) < 1e-10


@pytest.mark.parametrize("D", [1, 4])
def test_product_state_exact(lib, D):
    rng = np.random.default_rng(8)
    phis = [rng.standard_normal(2) for _ in range(4)]
    A = wl.product_itps(phis, D=D)
    ctx = lib.Ctm(A, 2, 2, D, 8, rsvd_oversample=8, seed=1)
    ctx.ctm_sweep(3, 1e-14)
    for i in range(4):
        for op in (wl.SX, wl.SZ):
            exact = phis[i] @ op @ phis[i] / (phis[i] @ phis[i])
            assert abs(ctx.ctm_expect_1site(i, op) - exact) < 1e-13


def test_tfim_mean_field_energy(lib):
    h = 2.9
    phi, e_mf = wl.tfim_mean_field(h)
    A = wl.product_itps([phi], D=2)
    ctx = lib.Ctm(A, 1, 1, 2, 8, rsvd_oversample=8, seed=1)
    ctx.ctm_sweep(3, 1e-14)
    assert abs(_gpu_energy(ctx, wl.tfim_bond(h), 1) - e_mf) < 1e-12


# --------------------------------------------------------------------------
# full sizes against stored oracle values (tests/golden/make_golden.py)
# --------------------------------------------------------------------------
def _golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    return json.load(open(path))


@pytest.mark.parametrize("name", ["itps_d4_chi64", "itps_d6_chi144", "restart_d4_chi64"])
def test_full_size_against_stored_oracle(lib, name):
    """Full-size runs against the stored oracle energies after the recorded
    sweeps, from the trivial boundary (itps_*) or from a random full-dimension
    environment (restart_*).  Each is gated at 1e-10, or at 10x the stored
    one-ulp spread of the oracle where the run amplifies rounding beyond that
    (printed with the measured difference)."""
    g = _golden(name)
    w = g["params"]
    A = wl.random_itps(2, 2, w["D"], 2, seed=w["seed"])
    ctx = lib.Ctm(A, 2, 2, w["D"], w["chi"], rsvd_oversample=w["p"], rsvd_power_iters=w["q"],
                  seed=w["sketch_seed"], svd_rel_cutoff=g["cutoff"])
    if "env_seed" in w:
        for i, (C, T) in enumerate(wl.random_environment(2, 2, w["chi"], w["D"] ** 2, seed=w["env_seed"])):
            ctx.ctm_set_env(i, C, T)
    H = wl.heisenberg_bond()
    last = max(int(s) for s in g["energies"])
    for s in range(1, last + 1):
        for dname in ("left", "right", "up", "down"):
            ctx.ctm_move(dname)
        if str(s) in g["energies"]:
            e = _gpu_energy(ctx, H, 4)
            ref = g["energies"][str(s)]
            sens = max(abs(ref - p[str(s)]) for p in g["energies_perturbed"])
            assert abs(e - ref) < _bound(abs(e - ref), sens, f"{name} sweep {s}"), (s, e, ref, sens)
    assert ctx.ctm_cut_stats()[2] == 0


@pytest.mark.parametrize("direction", ["left", "up", "right", "down"])
def test_full_size_one_move(lib, direction):
    """One move of the D=6, chi=144 workload (the benchmark's configuration)
    from a random full-dimension environment, against sampled entries of the
    oracle's renormalised tensors (max-abs normalised): 1e-8, as for the
    small one-move test."""
    g = _golden("move_d6_chi144")
    w = g["params"]
    D, chi = w["D"], w["chi"]
    A = wl.random_itps(2, 2, D, 2, seed=w["seed"])
    ctx = lib.Ctm(A, 2, 2, D, chi, rsvd_oversample=w["p"], rsvd_power_iters=w["q"], seed=w["sketch_seed"],
                  svd_rel_cutoff=g["cutoff"])
    for i, (C, T) in enumerate(wl.random_environment(2, 2, chi, D * D, seed=w["env_seed"])):
        ctx.ctm_set_env(i, C, T)
    ctx.ctm_move(direction)
    assert ctx.ctm_cut_stats() == (0, 4, 0)
    for key, rec in g["moves"][direction].items():
        kind, rest = key[0], key[1:]
        k = int(rest.split("_")[0]) - 1
        i = int(rest.split("site")[1])
        C, T, _ = ctx.ctm_get_env(i)
        x = C[k] if kind == "C" else T[k]
        assert list(x.shape) == rec["shape"]
        got = x.reshape(-1)[np.asarray(rec["pos"])]
        assert np.max(np.abs(got - np.asarray(rec["val"]))) < 1e-8, key
        assert abs(np.linalg.norm(x) - rec["fro"]) < 1e-8 * rec["fro"], key


def test_timing_modes(lib):
    """ctm_timing_enable: 1 times every phase, 2 the sketch products only (four
    products per pair of events), 0 stops; other values are rejected.  The
    sweeps give the same energy whichever mode is on."""
    from paper_2112_13184_amd._binding import CTM_EINVAL, CtmError
    A = wl.random_itps(2, 2, 3, 2, seed=7)
    H = wl.heisenberg_bond()
    energies, counts = [], []
    for mode in (0, 1, 2):
        ctx = lib.Ctm(A, 2, 2, 3, 24, rsvd_oversample=16, seed=4)
        ctx.ctm_sweep(2, 0.0)
        ctx.ctm_timing_enable(mode)
        ctx.ctm_sweep(2, 0.0)
        ph = ctx.ctm_timing_read()
        energies.append(sum(ctx.ctm_expect_2site(i, dr, H) for i in range(4) for dr in (0, 1)))
        counts.append({k: v["launches"] for k, v in ph.items()})
        if mode == 2:
            sk = ph["sketch_gemm"]
            assert sk["ms"] > 0 and sk["flops"] > 0
        with pytest.raises(CtmError) as ex:
            ctx.ctm_timing_enable(3)
        assert ex.value.status == CTM_EINVAL
        ctx.ctm_free()
    assert energies[0] == energies[1] == energies[2]
    assert all(v == 0 for v in counts[0].values())
    assert all(v > 0 for v in counts[1].values()), counts[1]
    assert counts[2]["sketch_gemm"] == counts[1]["sketch_gemm"] > 0
    assert all(v == 0 for k, v in counts[2].items() if k != "sketch_gemm"), counts[2]
