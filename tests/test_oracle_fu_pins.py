"""Pins of the full-update oracle (CPU only).

* The bond environment N, contracted with the untruncated pair a_i a_j,
  gives the bond density matrix of the CTMRG observables module (itself
  pinned to Onsager, brute force and product states): a wrong embedding,
  rotation or index order of N fails it.
* Each ALS half step solves its quadratic subproblem: the directly
  evaluated cost is stationary in the updated factor (central differences),
  and the cost never increases.  A wrong pairing of indices in R or S fails.
* Commuting Ising gates from |+x> are exact at D = 2 (Onsager's correlator);
  isolated dimers follow the two-site matrix exponential.
"""
import math

import numpy as np
from scipy.linalg import expm

import workloads as wl
from oracle import closed_forms as cf
from oracle import full_update as fu
from oracle import observables as ob
from oracle import simple_update as su
from oracle.ctmrg import Environment

LX = LY = 2
N = LX * LY
ZERO4 = np.zeros((4, 4))


def _converged(A, chi=16, sweeps=15):
    env = Environment([np.array(a) for a in A], LX, LY, chi=chi, oversample=32)
    for _ in range(sweeps):
        env.sweep()
    return env


def test_bond_environment_reproduces_the_bond_density_matrix():
    env = _converged(wl.random_itps(LX, LY, 2, 2, seed=4))
    for s in range(N):
        for direction in (0, 1):
            i, li, j, lj = su.bond(LX, LY, s, direction)
            D, d = 2, 2
            Xi, ai = fu.reduce_site(env.A[i], li)
            Xj, aj = fu.reduce_site(env.A[j], lj)
            Nm = fu.bond_environment(env, s, direction, fu.embed(Xi, li, D), fu.embed(Xj, lj, D))
            ident = np.eye(d * d)
            Th = fu.gated_core(ai, aj, ident, D, d)          # identity gate: the pair itself
            ri, rj = Xi.shape[1], Xj.shape[1]
            T4 = Th.reshape(ri, d, rj, d)
            rho = np.einsum("xyXY,xpyq,XPYQ->pqPQ", Nm.reshape(ri, rj, ri, rj), T4, T4).reshape(d * d, d * d)
            ref = ob.rho_bond(env, s, direction)
            assert np.abs(rho / np.trace(rho) - ref / np.trace(ref)).max() < 1e-12


def test_als_half_steps_are_exact_and_the_cost_decreases():
    env = _converged(wl.random_itps(LX, LY, 2, 2, seed=9))
    D, d = 2, 2
    g = su.gate(wl.tfim_bond(3.0), 0.2)
    s, direction = 1, 1
    i, li, j, lj = su.bond(LX, LY, s, direction)
    Xi, ai = fu.reduce_site(env.A[i], li)
    Xj, aj = fu.reduce_site(env.A[j], lj)
    Nm = fu.positive_part(fu.bond_environment(env, s, direction, fu.embed(Xi, li, D), fu.embed(Xj, lj, D)))
    Th = fu.gated_core(ai, aj, g, D, d)
    bi, bj = fu.svd_start(Th, D)
    hist = [fu.cost(bi, bj, Nm, Th, d)]
    for it in range(6):
        bi = fu.als_left(bj, Nm, Th, d, D)
        for factor in ("i",):
            h = 1e-6 * np.abs(bi).max()
            grad = np.zeros_like(bi)
            for idx in np.ndindex(bi.shape):
                e = np.zeros_like(bi)
                e[idx] = h
                grad[idx] = (fu.cost(bi + e, bj, Nm, Th, d) - fu.cost(bi - e, bj, Nm, Th, d)) / (2 * h)
            assert np.abs(grad).max() < 1e-7 * max(hist[0], 1e-30) / np.abs(bi).max(), (it, factor)
        hist.append(fu.cost(bi, bj, Nm, Th, d))
        bj = fu.als_right(bi, Nm, Th, d, D)
        h = 1e-6 * np.abs(bj).max()
        grad = np.zeros_like(bj)
        for idx in np.ndindex(bj.shape):
            e = np.zeros_like(bj)
            e[idx] = h
            grad[idx] = (fu.cost(bi, bj + e, Nm, Th, d) - fu.cost(bi, bj - e, Nm, Th, d)) / (2 * h)
        assert np.abs(grad).max() < 1e-7 * max(hist[0], 1e-30) / np.abs(bj).max(), it
        hist.append(fu.cost(bi, bj, Nm, Th, d))
    assert all(b <= a * (1 + 1e-12) + 1e-300 for a, b in zip(hist, hist[1:]))
    assert hist[-1] < hist[0]


def test_commuting_ising_gates_reach_onsager():
    tau, n = 0.05, 3
    Hz = -np.kron(wl.SZ, wl.SZ)
    A = wl.product_itps([np.array([1.0, 1.0]) / math.sqrt(2)] * N, 2)
    env = _converged(A, chi=16, sweeps=2)
    for _ in range(n):
        fu.full_update_step(env, [[Hz, Hz]] * N, tau, als_iters=3, env_sweeps=2)
    for _ in range(25):
        env.sweep()
    ref = cf.nn_correlator(2 * n * tau)
    for s in range(N):
        for direction in (0, 1):
            assert abs(ob.expect(ob.rho_bond(env, s, direction), -Hz) - ref) < 1e-9


def test_isolated_dimers_follow_the_exact_two_site_evolution():
    rng = np.random.default_rng(5)
    Hd = rng.standard_normal((4, 4))
    Hd = Hd + Hd.T
    phis = [rng.standard_normal(2) for _ in range(N)]
    tau, n = 0.03, 4
    H = [[Hd if s in (0, 2) else ZERO4, ZERO4] for s in range(N)]
    env = _converged(wl.product_itps(phis, 2), chi=8, sweeps=2)
    for _ in range(n):
        fu.full_update_step(env, H, tau, als_iters=2, env_sweeps=1)
    for _ in range(5):
        env.sweep()
    for s in (0, 2):
        psi = expm(-n * tau * Hd) @ np.kron(phis[s], phis[s + 1])
        psi = psi / np.linalg.norm(psi)
        rho = ob.rho_bond(env, s, 0)
        assert np.abs(rho / np.trace(rho) - np.outer(psi, psi)).max() < 1e-12
