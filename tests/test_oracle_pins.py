"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test checks the oracle against a closed form, a brute-force contraction,
an independent library implementation, a value the paper prints, or an exact
invariant, chosen so that a dropped term, a wrong sign / index or a transposed
operand in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import bruteforce as bf
from oracle import closed_forms as cf
from oracle import observables as ob
from oracle import philox
from oracle.ctmrg import Environment, enlarged_corner, projectors, rotate_site

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox: pinned to numpy's independent implementation of the same generator
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((3, 4, 5, 6), (5, 7)),
                                     ((2**64 - 2, 9, 2**63, 1), (2**64 - 1, 12345))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox emits the block of counter + 1 first
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    ref = [int(v) for v in g.random_raw(4)]
    c = list(ctr)
    c[0] = (c[0] + 1) % 2**64
    if c[0] == 0:
        c[1] += 1
    assert list(philox.philox4x64_10(c, key)) == ref


def test_omega_vectorised_equals_scalar_and_is_dyadic():
    sid = philox.stream_id(7, 1, 3)
    a = philox.omega_matrix(99, sid, 3, 5, 11)
    b = philox.omega_matrix_fast(99, sid, 3, 5, 11)
    assert np.array_equal(a, b)
    assert a.min() >= -1.0 and a.max() < 1.0
    assert np.all((a + 1.0) * 2.0**52 == np.round((a + 1.0) * 2.0**52))
    # rows keyed by the logical (c, b) index: a smaller chi prefix is a prefix
    c = philox.omega_matrix_fast(99, sid, 2, 5, 11)
    assert np.array_equal(c, b[:10])


# --------------------------------------------------------------------------
# Closed forms pinned by textbook special values and by each other
# --------------------------------------------------------------------------
def test_onsager_two_forms_and_critical_point():
    for beta in (0.3, 0.5, 0.7):
        assert abs(cf.onsager_lnz(beta) - cf.onsager_lnz_double(beta)) < 1e-11
    bc = 1.0 / cf.critical_temperature()
    assert abs(cf.onsager_lnz(bc) - (np.log(2.0) / 2 + 2 * cf.CATALAN / np.pi)) < 1e-12
    assert abs(np.sinh(2 * bc) - 1.0) < 1e-14


def test_internal_energy_is_beta_derivative():
    for beta in (0.35, 0.5, 0.65):
        h = 1e-4
        du = -(cf.onsager_lnz(beta + h) - cf.onsager_lnz(beta - h)) / (2 * h)
        assert abs(du - cf.internal_energy(beta)) < 1e-7


def test_yang_limits():
    assert cf.yang_magnetization(0.3) == 0.0           # above Tc
    assert abs(cf.yang_magnetization(5.0) - 1.0) < 1e-12
    assert 0.9 < cf.yang_magnetization(0.5) < 0.92


# --------------------------------------------------------------------------
# Values printed in the paper (worked example of Sec. 5.2)
# --------------------------------------------------------------------------
def _read_golden(name):
    sections, cur = {}, None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            sections[cur] = []
            continue
        sections[cur].append(line.split())
    return sections


def test_heisenberg_elements_match_paper_and_spin_algebra():
    g = _read_golden("heisenberg_2x2.txt")
    op = np.zeros((4, 4))
    for a, b, c, e, re, im in g["elements"]:
        op[int(c) * 2 + int(e), int(a) * 2 + int(b)] = float(re)
    assert np.array_equal(op, wl.heisenberg_bond())
    sz = 0.5 * wl.SZ
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T
    ref = np.kron(sz, sz) + 0.5 * (np.kron(sp, sm) + np.kron(sm, sp))
    assert np.allclose(op, ref, atol=0, rtol=0)


def test_bond_list_is_plus_x_and_plus_y_of_every_site():
    g = _read_golden("heisenberg_2x2.txt")
    bonds = sorted((int(s), int(dx), int(dy)) for s, dx, dy in g["bonds"])
    ours = sorted([(i, 1, 0) for i in range(4)] + [(i, 0, 1) for i in range(4)])
    assert bonds == ours


# --------------------------------------------------------------------------
# Contraction order: single-layer ket/bra equals the double-layer definition
# --------------------------------------------------------------------------
def test_single_layer_corner_equals_double_layer():
    rng = np.random.default_rng(0)
    D, d, chi = 2, 3, 5
    A = rng.standard_normal((D, D, D, D, d))
    C = rng.standard_normal((chi, chi))
    Tn = rng.standard_normal((chi, chi, D * D))
    Tp = rng.standard_normal((chi, chi, D * D))
    G2 = enlarged_corner(C, Tn, Tp, A, layers=2)
    a = bf.double_layer(A)
    G1 = enlarged_corner(C, Tn, Tp, a, layers=1)
    assert np.allclose(G1, G2, rtol=1e-13, atol=1e-12)
    # and the plain einsum of the definition
    ref = np.einsum("ab,acu,dbl,lurx->crdx", C, Tn, Tp, a).reshape(chi * D * D, chi * D * D)
    assert np.allclose(G2, ref, rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------------
# Untruncated CTMRG equals brute-force contraction of the absorbed patch
# --------------------------------------------------------------------------
def _extents_after(Lx, Ly, moves):
    """Number of columns / rows each site's environment has absorbed per side."""
    ext = {(x, y): [0, 0, 0, 0] for x in range(Lx) for y in range(Ly)}
    for m in moves:
        if m == "L":
            for x in range(Lx):
                for y in range(Ly):
                    ext[((x + 1) % Lx, y)][0] = ext[(x, y)][0] + 1
        elif m == "R":
            for k in range(Lx):
                x = (-k) % Lx
                for y in range(Ly):
                    ext[((x - 1) % Lx, y)][1] = ext[(x, y)][1] + 1
        elif m == "U":
            for k in range(Ly):
                y = (-k) % Ly
                for x in range(Lx):
                    ext[(x, (y - 1) % Ly)][2] = ext[(x, y)][2] + 1
        else:
            for y in range(Ly):
                for x in range(Lx):
                    ext[(x, (y + 1) % Ly)][3] = ext[(x, y)][3] + 1
    return ext


@pytest.mark.parametrize("Lx,Ly,sweeps", [(1, 1, 2), (2, 2, 1), (2, 1, 1), (1, 2, 1)])
@pytest.mark.parametrize("mode", ["rsvd", "dense"])
def test_untruncated_ctmrg_matches_bruteforce(Lx, Ly, sweeps, mode):
    A = wl.random_itps(Lx, Ly, 2, 2, seed=3)
    env = Environment(A, Lx, Ly, chi=256, layers=2, mode=mode, seed=1)
    for _ in range(sweeps):
        env.sweep()
    ext = _extents_after(Lx, Ly, "LRUD" * sweeps)
    bdy = np.eye(2).reshape(-1)
    for x in range(Lx):
        for y in range(Ly):
            i = x + Lx * y
            L, R, U, Dn = ext[(x, y)]
            rho = ob.rho_one_site(env, i)
            ref = bf.patch_value(A, Lx, Ly, 2, bdy, x - L, x + R, y - Dn, y + U, open_sites={(x, y)})
            assert np.allclose(rho / np.trace(rho), ref / np.trace(ref), atol=1e-13)
            # horizontal bond: the patch of site i with the right column of t included
            rho2 = ob.rho_bond(env, i, 0)
            ext_t = ext[((x + 1) % Lx, y)]
            ref2 = bf.patch_value(A, Lx, Ly, 2, bdy, x - L, x + 1 + ext_t[1], y - Dn, y + U,
                                  open_sites={(x, y), (x + 1, y)})
            ref2 = ref2.transpose(0, 2, 1, 3).reshape(4, 4)
            assert np.allclose(rho2 / np.trace(rho2), ref2 / np.trace(ref2), atol=1e-13)


def test_untruncated_classical_impurity_matches_bruteforce():
    a = wl.random_classical(1, 1, 2, seed=5)
    b = np.random.default_rng(1).standard_normal((2, 2, 2, 2))
    w = np.array([1.0, 0.5])
    env = Environment(a, 1, 1, chi=64, layers=1, boundary=w, mode="dense")
    env.sweep()
    env.sweep()
    z_b = bf.patch_value(a, 1, 1, 1, w, -2, 2, -2, 2, replace={(0, 0): b})
    z_a = bf.patch_value(a, 1, 1, 1, w, -2, 2, -2, 2)
    assert abs(ob.impurity_ratio(env, 0, b) - z_b / z_a) < 1e-12 * max(1.0, abs(z_b / z_a))


# --------------------------------------------------------------------------
# Projectors: Eckart-Young, P Pt = I, randomized equals dense
# --------------------------------------------------------------------------
def _random_corners(n, seed, decay=0.7):
    rng = np.random.default_rng(seed)
    Gs = []
    for _ in range(4):
        U, _ = np.linalg.qr(rng.standard_normal((n, n)))
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Gs.append(U @ np.diag(decay ** np.arange(n)) @ V.T)
    return Gs


def test_projectors_best_rank_k_and_biorthogonal():
    n, chi = 24, 7
    G_ur, G_ul, G_ll, G_lr = _random_corners(n, 2)
    P, Pt = projectors(G_ur, G_ul, G_ll, G_lr, chi, 1e-14, mode="dense")
    assert np.allclose(P @ Pt, np.eye(chi), atol=1e-10)
    H_u, H_dT = G_ur @ G_ul, G_ll @ G_lr
    M = H_u @ H_dT
    U, S, Vh = np.linalg.svd(M)
    best = (U[:, :chi] * S[:chi]) @ Vh[:chi]
    assert np.allclose(H_u @ Pt @ P @ H_dT, best, atol=1e-12 * S[0])


def test_randomized_projectors_equal_dense():
    n, chi = 30, 6
    G_ur, G_ul, G_ll, G_lr = _random_corners(n, 4, decay=0.5)
    Pd, Ptd = projectors(G_ur, G_ul, G_ll, G_lr, chi, 1e-14, mode="dense")
    Pr, Ptr = projectors(G_ur, G_ul, G_ll, G_lr, chi, 1e-14, mode="rsvd",
                         oversample=10, power_iters=2, seed=3, sid=1, nc_beta=n, Db=1)
    assert np.allclose(Ptd @ Pd, Ptr @ Pr, atol=1e-9)
    assert np.allclose(Pd, Pr, atol=1e-9)   # same sign convention


def test_identity_projectors_when_cut_fits():
    n = 5
    G = _random_corners(n, 1)
    P, Pt = projectors(*G, chi=n, cutoff=1e-12, mode="dense")
    assert np.array_equal(P, np.eye(n)) and np.array_equal(Pt, np.eye(n))


# --------------------------------------------------------------------------
# Classical Ising (single layer) against Onsager / Yang
# --------------------------------------------------------------------------
def test_classical_ising_onsager_yang():
    beta = 0.5
    a, b, w = wl.ising_classical(beta)
    env = Environment([a], 1, 1, chi=16, layers=1, boundary=w, mode="rsvd",
                      oversample=16, power_iters=2, seed=5)
    n, delta, conv = env.run(400, 1e-12)
    assert conv, delta
    f = -ob.log_kappa(env) / beta
    assert abs(f - (-cf.onsager_lnz(beta) / beta)) < 1e-8
    assert abs(ob.impurity_ratio(env, 0, b) - cf.yang_magnetization(beta)) < 1e-5


def test_classical_ising_error_shrinks_with_chi():
    beta = 0.45          # closer to Tc: the finite-chi error is visible
    a, b, w = wl.ising_classical(beta)
    errs = []
    for chi in (4, 8, 12):
        env = Environment([a], 1, 1, chi=chi, layers=1, boundary=w, mode="dense")
        env.run(300, 1e-11)
        errs.append(abs(ob.impurity_ratio(env, 0, b) - cf.yang_magnetization(beta)))
    assert errs[2] < errs[1] < errs[0]


# --------------------------------------------------------------------------
# Double layer with exact answers: the Ising PEPS, also gauge transformed
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cell", ["1x1", "2x2gauged"])
def test_ising_peps_closed_forms(cell):
    beta = 0.5
    A, wp = wl.ising_peps(beta)
    if cell == "1x1":
        tensors, Lx, Ly = [A], 1, 1
    else:
        tensors, Lx, Ly = wl.gauged_2x2(A, 2, seed=7), 2, 2
        wp = None   # gauges on the boundary break the polarised product; use delta
    env = Environment(tensors, Lx, Ly, chi=16, layers=2, boundary=wp, mode="rsvd",
                      oversample=16, power_iters=2, seed=2)
    n, delta, conv = env.run(400, 1e-11)
    zz = np.kron(wl.SZ, wl.SZ)
    for i in range(Lx * Ly):
        for dirn in (0, 1):
            assert abs(ob.expect(ob.rho_bond(env, i, dirn), zz) - cf.nn_correlator(beta)) < 1e-9
        m = abs(ob.expect(ob.rho_one_site(env, i), wl.SZ))
        if cell == "1x1":
            assert abs(m - cf.yang_magnetization(beta)) < 1e-9
    if cell == "1x1":
        assert abs(ob.log_kappa(env) - cf.onsager_lnz(beta)) < 1e-10


# --------------------------------------------------------------------------
# Product states (D = 1, and zero padded to D = 4: rank-1 cut, cutoff path)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("D", [1, 4])
def test_product_state_exact(D):
    rng = np.random.default_rng(8)
    phis = [rng.standard_normal(2) for _ in range(4)]
    A = wl.product_itps(phis, D=D)
    env = Environment(A, 2, 2, chi=8, layers=2, mode="rsvd", oversample=8, seed=1)
    env.run(3, 1e-14)
    ops = [wl.SX, wl.SZ, np.array([[0.3, -1.2], [0.7, 2.0]])]
    for i in range(4):
        rho = ob.rho_one_site(env, i)
        for op in ops:
            exact = phis[i] @ op @ phis[i] / (phis[i] @ phis[i])
            assert abs(ob.expect(rho, op) - exact) < 1e-14
    j = 1  # right neighbour of site 0
    O2 = np.kron(wl.SZ, wl.SX)
    ex = (phis[0] @ wl.SZ @ phis[0]) * (phis[j] @ wl.SX @ phis[j]) / (phis[0] @ phis[0]) / (phis[j] @ phis[j])
    assert abs(ob.expect(ob.rho_bond(env, 0, 0), O2) - ex) < 1e-14


def test_tfim_mean_field_energy():
    h = 2.9
    phi, e_mf = wl.tfim_mean_field(h)
    A = wl.product_itps([phi], D=2)
    env = Environment(A, 1, 1, chi=8, layers=2, mode="rsvd", oversample=8, seed=1)
    env.run(3, 1e-14)
    assert abs(ob.energy_per_site(env, wl.tfim_bond(h)) - e_mf) < 1e-12


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------
def test_scale_and_replication_invariance():
    A = wl.random_itps(1, 1, 2, 2, seed=11)
    H = wl.heisenberg_bond()
    e = []
    for tensors, L in (([A[0]], 1), ([3.7 * A[0]], 1), ([A[0]] * 4, 2)):
        env = Environment(tensors, L, L, chi=12, layers=2, mode="dense")
        env.run(300, 1e-11)
        e.append(ob.energy_per_site(env, H))
    # scaling changes nothing; the replicated cell updates columns in a different
    # order and reaches a fixed point that agrees within the finite-chi error
    assert abs(e[0] - e[1]) < 1e-12 and abs(e[0] - e[2]) < 1e-6


def test_rotation_invariance():
    A = wl.random_itps(2, 1, 2, 2, seed=12)
    H = wl.heisenberg_bond()
    env = Environment(A, 2, 1, chi=12, layers=2, mode="dense")
    env.run(300, 1e-11)
    e0 = ob.energy_per_site(env, H)
    # lattice rotated 90 degrees counter-clockwise: (x, y) -> (-y, x), cell 1 x 2
    B = [None, None]
    for x in range(2):
        xr, yr = 0, x % 2
        B[xr + 1 * yr] = rotate_site(A[x], 1)
    env_r = Environment(B, 1, 2, chi=12, layers=2, mode="dense")
    env_r.run(300, 1e-11)
    assert abs(ob.energy_per_site(env_r, H) - e0) < 1e-6   # finite-chi fixed points


def test_c4v_symmetric_tensor_equal_corner_spectra():
    a, _, w = wl.ising_classical(0.4)
    env = Environment([a], 1, 1, chi=8, layers=1, boundary=w, mode="dense")
    env.run(200, 1e-12)
    s = env.corner_spectra()
    assert np.allclose(s, s[0][None, :], atol=1e-10)


def test_rho_hermitian_positive():
    A = wl.random_itps(2, 2, 2, 2, seed=13)
    env = Environment(A, 2, 2, chi=10, layers=2, mode="rsvd", oversample=8, seed=4)
    env.run(20, 1e-10)
    for i in range(4):
        for rho in (ob.rho_one_site(env, i), ob.rho_bond(env, i, 0), ob.rho_bond(env, i, 1)):
            rho = rho / np.trace(rho)
            assert np.allclose(rho, rho.T, atol=1e-8)
            assert np.linalg.eigvalsh(0.5 * (rho + rho.T)).min() > -1e-6


# --------------------------------------------------------------------------
# Correlation functions and the transfer-matrix spectrum (Sec. 5.3, Eq. (8),
# Eq. (9))
# --------------------------------------------------------------------------
def _op_layer(A, op):
    """Double-layer tensor with a one-site operator between ket and bra:
    sum_{p,p'} A[.., p] conj(A[.., p']) op[p', p]."""
    a = bf.double_layer(A, open_phys=True)
    return np.tensordot(a, op, axes=([4, 5], [1, 0]))


@pytest.mark.parametrize("Lx,Ly,direction", [(1, 1, 0), (1, 1, 1), (2, 1, 0), (1, 2, 1)])
def test_transfer_spectrum_untruncated_matches_strip(Lx, Ly, direction):
    """An untruncated environment is an exact finite network, so its transfer
    matrix over one period is the column transfer matrix of a strip of
    U + 1 + Dn sites closed by the boundary vectors: the leading eigenvalues
    (ratios to the largest) agree to rounding."""
    A = wl.random_itps(Lx, Ly, 2, 2, seed=3)
    env = Environment(A, Lx, Ly, chi=256, layers=2, mode="dense", seed=1)
    env.sweep()
    ext = _extents_after(Lx, Ly, "LRUD")
    bdy = np.eye(2).reshape(-1)
    lam = ob.transfer_spectrum(env, 0, direction, 6)
    if direction == 0:
        L, R, U, Dn = ext[(0, 0)]
        M = np.eye(4 ** (U + 1 + Dn))
        for x in range(Lx):
            M = M @ bf.strip_transfer(A[x], 2, bdy, U + 1 + Dn)
    else:
        # the +y transfer is the +x transfer of the lattice rotated three
        # quarter turns: sites rotated, the column runs over x
        L, R, U, Dn = ext[(0, 0)]
        M = np.eye(4 ** (L + 1 + R))
        for y in range(Ly):
            M = M @ bf.strip_transfer(rotate_site(A[Lx * y], 3), 2, bdy, L + 1 + R)
    ref = np.linalg.eigvals(M)
    ref = ref[np.argsort(-np.abs(ref), kind="stable")][:6]
    assert np.allclose(np.sort_complex(lam / lam[0]), np.sort_complex(ref / ref[0]), atol=1e-10)


@pytest.mark.parametrize("direction", [0, 1])
def test_correlation_untruncated_matches_bruteforce(direction):
    """C(r) = <A(0) B(r e)> of an untruncated 1x1 environment against the
    brute-force contraction of the finite network with the operators
    inserted, r = 0..2 (r = 0: the one-site value of the product A B)."""
    A = wl.random_itps(1, 1, 2, 2, seed=4)[0]
    env = Environment([A], 1, 1, chi=256, layers=2, mode="dense", seed=1)
    env.sweep()
    L, R, U, Dn = _extents_after(1, 1, "LRUD")[(0, 0)]
    opA = np.array([[0.3, -1.2], [0.7, 2.0]])
    opB = np.array([[1.1, 0.4], [-0.6, -0.5]])
    bdy = np.eye(2).reshape(-1)
    C = ob.correlation(env, 0, opA, opB, 2, direction)
    for r in range(3):
        if r == 0:
            rep = {(0, 0): _op_layer(A, opA @ opB)}
        else:
            rep = {(0, 0): _op_layer(A, opA), ((r, 0) if direction == 0 else (0, r)): _op_layer(A, opB)}
        x1 = R + (r if direction == 0 else 0)
        y1 = U + (r if direction == 1 else 0)
        num = bf.patch_value([A], 1, 1, 2, bdy, -L, x1, -Dn, y1, replace=rep)
        den = bf.patch_value([A], 1, 1, 2, bdy, -L, x1, -Dn, y1)
        assert abs(C[r] - num / den) < 1e-12 * max(1.0, abs(num / den)), r


def test_correlation_product_state():
    """Product states: C(r) = <A><B> for r >= 1, <A B> at r = 0, and the
    transfer matrix has one non-zero eigenvalue (infinite e_1)."""
    rng = np.random.default_rng(2)
    phis = [rng.standard_normal(2) for _ in range(4)]
    env = Environment(wl.product_itps(phis, D=2), 2, 2, chi=8, layers=2, mode="rsvd", oversample=8, seed=1)
    env.run(3, 1e-14)
    opA, opB = wl.SX, np.array([[0.3, -1.2], [0.7, 2.0]])
    ev = lambda phi, op: phi @ op @ phi / (phi @ phi)
    for i in range(4):
        for direction in (0, 1):
            C = ob.correlation(env, i, opA, opB, 5, direction)
            x, y = i % 2, i // 2
            assert abs(C[0] - ev(phis[i], opA @ opB)) < 1e-13
            for r in range(1, 6):
                j = ((x + r) % 2 + 2 * y) if direction == 0 else (x + 2 * ((y + r) % 2))
                assert abs(C[r] - ev(phis[i], opA) * ev(phis[j], opB)) < 1e-13
    lam = ob.transfer_spectrum(env, 0, 0, 3)
    xi, e = ob.correlation_length(lam, 2)
    assert abs(lam[1]) < 1e-12 * abs(lam[0]) and xi < 0.1


def test_ising_peps_correlation_closed_forms():
    """The Ising PEPS (beta = 0.5): <sz(0) sz(r)> at r = 1 is Onsager's
    nearest-neighbour correlator, and at large r the square of Yang's
    magnetisation (the connected part decays with the transfer-matrix gap,
    xi ~ 2); both directions."""
    beta = 0.5
    A, wp = wl.ising_peps(beta)
    env = Environment([A], 1, 1, chi=16, layers=2, boundary=wp, mode="rsvd", oversample=16, power_iters=2, seed=2)
    env.run(400, 1e-11)
    lam = ob.transfer_spectrum(env, 0, 0, 3)
    xi, e = ob.correlation_length(lam, 1)
    assert 1.5 < xi < 2.5
    for direction in (0, 1):
        C = ob.correlation(env, 0, wl.SZ, wl.SZ, 60, direction)
        assert abs(C[0] - 1.0) < 1e-12                       # sz^2 = 1
        assert abs(C[1] - cf.nn_correlator(beta)) < 1e-9
        assert abs(C[60] - cf.yang_magnetization(beta) ** 2) < 1e-8


def test_xi_extrapolation_recovers_line():
    """Eq. (9): 1/xi(inf) = e1(chi) + k (e2(chi) - e1(chi)); data placed
    exactly on such a line give back its intercept and k."""
    inv_xi, k = 0.37, 0.8
    delta = np.array([0.5, 0.3, 0.2, 0.12])
    e1 = inv_xi - k * delta
    e2 = e1 + delta
    got_inv, got_k = ob.xi_extrapolate(e1, e2)
    assert abs(got_inv - inv_xi) < 1e-14 and abs(got_k - k) < 1e-13
