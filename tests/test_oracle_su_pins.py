"""Pins of the simple-update and mean-field-environment oracle (CPU only).

Each evolution below has an answer fixed by something other than the oracle:
a closed form, Onsager's solution through the (separately pinned) CTMRG
oracle, an exact two-site evolution by the matrix exponential, or the
mean-field solution of a product state.  Between them they fail on a wrong
leg or neighbour, a gate applied to the wrong pair of indices, a weight not
absorbed or not divided out, the wrong power of the weights in the mean-field
environment, or a wrong Trotter sign.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as wl
from oracle import closed_forms as cf
from oracle import observables as ob
from oracle import simple_update as su
from oracle.ctmrg import Environment

LX = LY = 2
N = LX * LY
ZERO4 = np.zeros((4, 4))


def _start(phis, D):
    return wl.product_itps(phis, D), [np.ones(D) for _ in range(N)], [np.ones(D) for _ in range(N)]


def test_field_only_evolution_is_a_rotation():
    """H = -(h/4)(sx 1 + 1 sx) on every bond: each site sees exp(tau h sx) per
    step, so |up> becomes cosh(a)|up> + sinh(a)|down>, a = N tau h, and
    <sx> = tanh(2a); the state stays a product (second weight zero)."""
    h, tau, n = 1.3, 0.05, 10
    Hf = -0.25 * h * (np.kron(wl.SX, wl.ID2) + np.kron(wl.ID2, wl.SX))
    G, lh, lv = _start([np.array([1.0, 0.0])] * N, 2)
    G, lh, lv = su.simple_update(G, lh, lv, [[Hf, Hf]] * N, tau, LX, LY, n)
    for s in range(N):
        sx = su.expect(su.mfe_rho_site(G, lh, lv, LX, LY, s), wl.SX)
        assert abs(sx - math.tanh(2 * n * tau * h)) < 1e-13
        assert lh[s][1] < 1e-14 and lv[s][1] < 1e-14


def test_commuting_ising_gates_reach_onsager():
    """H = -sz sz from |+x>: the gates commute (Trotter is exact) and the
    evolved state exp(N tau sum sz sz)|+x> has bond dimension 2, so D = 3
    truncates nothing (third weight zero) and the state is exact.  Its norm is
    the Ising partition function at beta = 2 N tau, so every bond's <sz sz>
    is Onsager's nearest-neighbour correlator."""
    tau, n = 0.05, 3
    Hz = -np.kron(wl.SZ, wl.SZ)
    G, lh, lv = _start([np.array([1.0, 1.0]) / math.sqrt(2)] * N, 3)
    G, lh, lv = su.simple_update(G, lh, lv, [[Hz, Hz]] * N, tau, LX, LY, n)
    for s in range(N):
        assert lh[s][2] < 1e-14 and lv[s][2] < 1e-14
    A = [a[:2, :2, :2, :2, :] for a in su.to_itps(G, lh, lv, LX, LY)]
    env = Environment(A, LX, LY, chi=24)
    for _ in range(30):
        env.sweep()
    ref = cf.nn_correlator(2 * n * tau)
    for s in range(N):
        for direction in (0, 1):
            assert abs(ob.expect(ob.rho_bond(env, s, direction), -Hz) - ref) < 1e-10


def test_horizontal_gates_only_make_decoupled_chains():
    """Gates on the horizontal bonds only: independent Ising chains with
    <sz sz> = tanh(2 N tau) along x and zero along y (CTMRG oracle), and the
    mean-field environment of a chain of such bonds gives the same x value."""
    tau, n = 0.05, 4
    Hz = -np.kron(wl.SZ, wl.SZ)
    G, lh, lv = _start([np.array([1.0, 1.0]) / math.sqrt(2)] * N, 2)
    G, lh, lv = su.simple_update(G, lh, lv, [[Hz, ZERO4]] * N, tau, LX, LY, n)
    env = Environment(su.to_itps(G, lh, lv, LX, LY), LX, LY, chi=16)
    for _ in range(20):
        env.sweep()
    ref = math.tanh(2 * n * tau)
    for s in range(N):
        assert abs(ob.expect(ob.rho_bond(env, s, 0), -Hz) - ref) < 1e-12
        assert abs(ob.expect(ob.rho_bond(env, s, 1), -Hz)) < 1e-12
        assert abs(su.expect(su.mfe_rho_bond(G, lh, lv, LX, LY, s, 0), -Hz) - ref) < 1e-12


def test_isolated_dimers_follow_the_exact_two_site_evolution():
    """A general symmetric gate on the horizontal bonds of sites 0 and 2 only,
    from a random product state: each dimer evolves as
    psi = expm(-N tau H) (phi_i x phi_j), which has Schmidt rank <= 2 = D, and
    its environment is trivial, so the mean-field bond and site density
    matrices are exact."""
    rng = np.random.default_rng(5)
    Hd = rng.standard_normal((4, 4))
    Hd = Hd + Hd.T
    phis = [rng.standard_normal(2) for _ in range(N)]
    tau, n = 0.03, 7
    H = [[Hd if s in (0, 2) else ZERO4, ZERO4] for s in range(N)]
    G, lh, lv = _start(phis, 2)
    G, lh, lv = su.simple_update(G, lh, lv, H, tau, LX, LY, n)
    for s in (0, 2):
        psi = expm(-n * tau * Hd) @ np.kron(phis[s], phis[s + 1])
        psi = psi / np.linalg.norm(psi)
        rho = su.mfe_rho_bond(G, lh, lv, LX, LY, s, 0)
        assert np.abs(rho / np.trace(rho) - np.outer(psi, psi)).max() < 1e-13
        P = psi.reshape(2, 2)
        r1 = su.mfe_rho_site(G, lh, lv, LX, LY, s)
        assert np.abs(r1 / np.trace(r1) - P @ P.T).max() < 1e-13
        r2 = su.mfe_rho_site(G, lh, lv, LX, LY, s + 1)
        assert np.abs(r2 / np.trace(r2) - P.T @ P).max() < 1e-13
        # the weights are the Schmidt values of the dimer
        sv = np.linalg.svd(P, compute_uv=False)
        assert np.abs(lh[s] - sv).max() < 1e-13


def test_d1_tfim_approaches_the_mean_field_energy():
    """D = 1 keeps product states: the evolution is projected imaginary-time
    evolution, whose fixed point is the mean-field state up to O(tau^2) in the
    energy; two step sizes and a Richardson step pin the limit."""
    h = 2.0
    Hb = wl.tfim_bond(h)
    _, emf = wl.tfim_mean_field(h)
    es = []
    for tau, n in ((0.02, 1500), (0.01, 3000)):
        G, lh, lv = _start([np.array([1.0, 0.0])] * N, 1)
        G, lh, lv = su.simple_update(G, lh, lv, [[Hb, Hb]] * N, tau, LX, LY, n)
        es.append(su.mfe_energy(G, lh, lv, LX, LY, [[Hb, Hb]] * N))
    assert 0 < es[0] - emf < 2e-5 and 0 < es[1] - emf < 5e-6
    assert abs((4 * es[1] - es[0]) / 3 - emf) < 2e-7


def test_d1_heisenberg_reaches_the_neel_energy():
    """D = 1, S = 1/2 antiferromagnet on the 2x2 cell from random product
    states: the projected evolution ends in a Neel state, -1/4 per bond, -1/2
    per site (a fixed point of every gate's rank-1 truncation)."""
    rng = np.random.default_rng(11)
    Hh = wl.heisenberg_bond()
    G, lh, lv = _start([rng.standard_normal(2) for _ in range(N)], 1)
    G, lh, lv = su.simple_update(G, lh, lv, [[Hh, Hh]] * N, 0.05, LX, LY, 600)
    assert abs(su.mfe_energy(G, lh, lv, LX, LY, [[Hh, Hh]] * N) + 0.5) < 1e-10


@pytest.mark.parametrize("D", [2, 3])
def test_weights_are_normalised_sorted_and_gauge_fixed(D):
    """Invariants of every bond update: weights non-negative, descending, unit
    2-norm; the sign rule leaves the first near-largest entry of each kept left
    vector positive."""
    A = wl.random_itps(LX, LY, D, 2, seed=3)
    lh = [np.ones(D) for _ in range(N)]
    lv = [np.ones(D) for _ in range(N)]
    Hb = wl.tfim_bond(3.0)
    G, lh, lv = su.simple_update(A, lh, lv, [[Hb, Hb]] * N, 0.05, LX, LY, 3)
    for w in lh + lv:
        assert np.all(w >= 0) and np.all(np.diff(w) <= 0) and abs(np.sum(w * w) - 1) < 1e-13
    # the last bond of a step is the vertical bond of site 3 (leg u of site 3)
    s = 3
    wi = su.leg_weights(lh, lv, LX, LY, s)
    B = su._scale_legs(G[s], wi, skip=1)                      # outer weights back on
    B = B.transpose(0, 2, 3, 4, 1).reshape(-1, D)             # rows (a, p), columns k
    for k in range(D):
        col = B[:, k]
        m = np.abs(col).max()
        first = int(np.argmax(np.abs(col) >= (1 - su.SIGN_TOL) * m))
        assert col[first] > 0


SY = np.array([[0.0, -1.0j], [1.0j, 0.0]])


def test_complex_field_along_y_is_a_rotation():
    """H = -(h/4)(sy 1 + 1 sy) (complex): exp(tau h sy) per step on each site
    takes |up> to cosh(a)|up> + i sinh(a)|down>, a = N tau h, so
    <sy> = tanh(2a); the state stays a product."""
    h, tau, n = 0.9, 0.05, 8
    Hy = -0.25 * h * (np.kron(SY, wl.ID2) + np.kron(wl.ID2, SY))
    G, lh, lv = _start([np.array([1.0, 0.0])] * N, 2)
    G, lh, lv = su.simple_update(G, lh, lv, [[Hy, Hy]] * N, tau, LX, LY, n)
    assert np.iscomplexobj(G[0])
    for s in range(N):
        rho = su.mfe_rho_site(G, lh, lv, LX, LY, s)
        assert abs(su.expect(rho, SY) - math.tanh(2 * n * tau * h)) < 1e-13
        assert abs(su.expect(rho, wl.SX)) < 1e-13
        assert lh[s][1] < 1e-14 and lv[s][1] < 1e-14


def test_local_unitary_rotation_of_a_real_problem():
    """Rotating every site's physical index by U_s = diag(1, exp(i phi_s))
    (tensors U_s A_s, bond Hamiltonians (U_i x U_j) H (U_i x U_j)^H, complex)
    gives the same evolution: weights and mean-field energies equal those of
    the real problem.  A conjugate missing or misplaced anywhere breaks it."""
    D = 2
    A = wl.random_itps(LX, LY, D, 2, seed=13)
    ones = [np.ones(D) for _ in range(N)]
    Hb = wl.tfim_bond(2.5)
    H = [[Hb, Hb] for _ in range(N)]
    Gr, lhr, lvr = su.simple_update(A, ones, ones, H, 0.02, LX, LY, 15)
    phis = [0.3, 1.1, -0.7, 2.0]
    Us = [np.diag([1.0, np.exp(1j * p)]) for p in phis]
    Ac = [np.einsum("PQ,lurdQ->lurdP", Us[s], A[s]) for s in range(N)]
    Hc = []
    for s in range(N):
        row = []
        for direction in (0, 1):
            i, _, j, _ = su.bond(LX, LY, s, direction)
            UU = np.kron(Us[i], Us[j])
            row.append(UU @ Hb @ UU.conj().T)
        Hc.append(row)
    Gc, lhc, lvc = su.simple_update(Ac, ones, ones, Hc, 0.02, LX, LY, 15)
    for s in range(N):
        assert np.abs(lhc[s] - lhr[s]).max() < 1e-12 and np.abs(lvc[s] - lvr[s]).max() < 1e-12
    assert abs(su.mfe_energy(Gc, lhc, lvc, LX, LY, Hc) - su.mfe_energy(Gr, lhr, lvr, LX, LY, H)) < 1e-12


def test_complex_dimers_follow_the_exact_two_site_evolution():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    Hd = X + X.conj().T
    phis = [rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(N)]
    tau, n = 0.03, 6
    H = [[Hd if s in (0, 2) else ZERO4, ZERO4] for s in range(N)]
    G = [np.zeros((2, 2, 2, 2, 2), dtype=complex) for _ in range(N)]
    for s in range(N):
        G[s][0, 0, 0, 0, :] = phis[s]
    ones = [np.ones(2) for _ in range(N)]
    G, lh, lv = su.simple_update(G, ones, ones, H, tau, LX, LY, n)
    for s in (0, 2):
        psi = expm(-n * tau * Hd) @ np.kron(phis[s], phis[s + 1])
        psi = psi / np.linalg.norm(psi)
        rho = su.mfe_rho_bond(G, lh, lv, LX, LY, s, 0)
        assert np.abs(rho / np.trace(rho) - np.outer(psi, psi.conj())).max() < 1e-13
