"""Correlation functions and the transfer-matrix spectrum on the GPU (Sec. 5.3,
Eq. (8), (9)), through the C ABI, against the FP64 oracle.

The oracle's environment is loaded into the GPU context (or the environment
is an exact finite network on both sides), so both sides contract the same
tensors: values agree to rounding (1e-10 relative), eigenvalues of the
transfer matrix to the Arnoldi / ARPACK tolerance (1e-9 relative to the
largest).  Closed forms: the Ising PEPS (Onsager's nearest-neighbour
correlator, Yang's magnetisation squared at large distance) and product
states.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import bruteforce as bf
from oracle import closed_forms as cf
from oracle import observables as ob
from oracle.ctmrg import Environment, rotate_site
from tests._util import load_state

pytestmark = pytest.mark.gpu

OPA = np.array([[0.3, -1.2], [0.7, 2.0]])
OPB = np.array([[1.1, 0.4], [-0.6, -0.5]])


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


def _same_spectrum(got, ref, tol):
    """Every eigenvalue of `got` has one of `ref` within tol * |ref[0]| (as
    multisets; conjugate pairs of equal modulus may come in either order)."""
    ref = list(ref)
    scale = abs(ref[0])
    for g in got:
        k = int(np.argmin([abs(g - r) for r in ref]))
        assert abs(g - ref[k]) <= tol * scale, (got, ref)
        ref.pop(k)


def _tfim_state(L, D, chi, h, sweeps):
    A = wl.tfim_request_tensors(h, D, L, L, 0.1, seed=17 + D + L)
    ora = Environment(A, L, L, chi=chi, layers=2, mode="rsvd", oversample=16, power_iters=1, seed=9)
    for _ in range(sweeps):
        ora.sweep()
    return A, ora


@pytest.mark.parametrize("L,D,chi,h", [(2, 2, 12, 3.1), (2, 3, 30, 3.3)])
def test_correlation_and_spectrum_on_oracle_environment(lib, L, D, chi, h):
    """A transverse-field Ising state swept by the oracle, its environment
    loaded into the GPU context: C(r) for r = 0..12 from every site in both
    directions, 1e-10 relative to max(1, |C|); the four leading eigenvalues of
    the transfer matrix of every row and column, 1e-9 of the largest (the
    D = 3, chi = 30 matrix has dimension 8100: ARPACK on the oracle side)."""
    A, ora = _tfim_state(L, D, chi, h, 8)
    ctx = lib.Ctm(A, L, L, D, chi, rsvd_oversample=16, rsvd_power_iters=1, seed=9)
    load_state(ctx, ora)
    worst = 0.0
    for i in range(L * L):
        for direction in (0, 1):
            got = ctx.ctm_correlation(i, direction, OPA, OPB, 12)
            ref = ob.correlation(ora, i, OPA, OPB, 12, direction)
            err = np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))
            worst = max(worst, err)
            assert err < 1e-10, (i, direction, err)
    for direction in (0, 1):
        for line in range(L):
            lam, e, xi = ctx.ctm_transfer_spectrum(direction, line, 4)
            ref = ob.transfer_spectrum(ora, line, direction, 4)
            _same_spectrum(lam, ref, 1e-9)
            xi_ref, e_ref = ob.correlation_length(ref, L)
            assert abs(xi - xi_ref) <= 1e-8 * xi_ref and np.allclose(e, e_ref[:3], rtol=1e-8)
    print(f"L={L} D={D} chi={chi}: max relative C(r) difference {worst:.1e}")


@pytest.mark.parametrize("direction", [0, 1])
def test_untruncated_against_bruteforce(lib, direction):
    """One sweep of a 1x1 cell at chi = 256 (nothing truncated: the
    environment is an exact finite network): C(r), r = 0..2, against the
    brute-force contraction of the network with the operators inserted, and
    the transfer spectrum against the strip's column transfer matrix."""
    A = wl.random_itps(1, 1, 2, 2, seed=4)[0]
    ctx = lib.Ctm([A], 1, 1, 2, 256, rsvd_oversample=16, rsvd_power_iters=1, seed=1)
    ctx.ctm_sweep(1, 0.0)
    L = R = U = Dn = 1   # extents after one sweep of a 1x1 cell
    bdy = np.eye(2).reshape(-1)

    def op_layer(op):
        a = bf.double_layer(A, open_phys=True)
        return np.tensordot(a, op, axes=([4, 5], [1, 0]))

    C = ctx.ctm_correlation(0, direction, OPA, OPB, 2)
    for r in range(3):
        rep = ({(0, 0): op_layer(OPA @ OPB)} if r == 0 else
               {(0, 0): op_layer(OPA), ((r, 0) if direction == 0 else (0, r)): op_layer(OPB)})
        x1, y1 = R + (r if direction == 0 else 0), U + (r if direction == 1 else 0)
        num = bf.patch_value([A], 1, 1, 2, bdy, -L, x1, -Dn, y1, replace=rep)
        den = bf.patch_value([A], 1, 1, 2, bdy, -L, x1, -Dn, y1)
        assert abs(C[r] - num / den) < 1e-11 * max(1.0, abs(num / den)), r
    lam, _, _ = ctx.ctm_transfer_spectrum(direction, 0, 6)
    site = A if direction == 0 else rotate_site(A, 3)
    M = bf.strip_transfer(site, 2, bdy, 3)
    ref = np.linalg.eigvals(M)
    ref = ref[np.argsort(-np.abs(ref))]
    # the environment tensors are normalised: compare the ratios to the largest
    _same_spectrum(lam / lam[0], ref[:12] / ref[0], 1e-10)


def test_ising_peps_correlations_closed_forms(lib):
    """The Ising PEPS (beta = 0.5, polarised boundary) run to delta < 1e-11:
    <sz(0) sz(r)> is Onsager's nearest-neighbour correlator at r = 1 and
    Yang's magnetisation squared at r = 60 (1e-9 / 1e-8: finite chi); the
    correlation length against the oracle's converged run, 1e-8 relative."""
    beta = 0.5
    A, wp = wl.ising_peps(beta)
    ctx = lib.Ctm([A], 1, 1, 2, 16, boundary=wp, rsvd_oversample=16, rsvd_power_iters=2, seed=2)
    ctx.ctm_sweep(400, 1e-11)
    ora = Environment([A], 1, 1, chi=16, layers=2, boundary=wp, mode="rsvd", oversample=16, power_iters=2, seed=2)
    ora.run(400, 1e-11)
    for direction in (0, 1):
        C = ctx.ctm_correlation(0, direction, wl.SZ, wl.SZ, 60)
        assert abs(C[0] - 1.0) < 1e-12
        assert abs(C[1] - cf.nn_correlator(beta)) < 1e-9
        assert abs(C[60] - cf.yang_magnetization(beta) ** 2) < 1e-8
        ref = ob.correlation(ora, 0, wl.SZ, wl.SZ, 60, direction)
        assert np.max(np.abs(C - ref)) < 1e-10
        lam, e, xi = ctx.ctm_transfer_spectrum(direction, 0, 3)
        xi_ref, _ = ob.correlation_length(ob.transfer_spectrum(ora, 0, direction, 3), 1)
        assert abs(xi - xi_ref) < 1e-8 * xi_ref
    print(f"Ising PEPS: xi = {xi:.10f}")


def test_product_state(lib):
    """Product states: C(r) = <A><B> (r >= 1), <A B> (r = 0); the transfer
    matrix has a single non-zero eigenvalue."""
    rng = np.random.default_rng(2)
    phis = [rng.standard_normal(2) for _ in range(4)]
    ctx = lib.Ctm(wl.product_itps(phis, D=2), 2, 2, 2, 8, rsvd_oversample=8, seed=1)
    ctx.ctm_sweep(3, 1e-14)
    ev = lambda phi, op: phi @ op @ phi / (phi @ phi)
    for i in range(4):
        x, y = i % 2, i // 2
        for direction in (0, 1):
            C = ctx.ctm_correlation(i, direction, OPA, OPB, 5)
            assert abs(C[0] - ev(phis[i], OPA @ OPB)) < 1e-13
            for r in range(1, 6):
                j = ((x + r) % 2 + 2 * y) if direction == 0 else (x + 2 * ((y + r) % 2))
                assert abs(C[r] - ev(phis[i], OPA) * ev(phis[j], OPB)) < 1e-13
    lam, e, xi = ctx.ctm_transfer_spectrum(0, 0, 3)
    assert abs(lam[1]) < 1e-12 * abs(lam[0]) and xi < 0.1


def test_xi_extrapolation(lib):
    """Eq. (9) through the C ABI against the oracle's least squares."""
    rng = np.random.default_rng(5)
    e1 = rng.uniform(0.2, 0.6, 5)
    e2 = e1 + rng.uniform(0.05, 0.5, 5)
    from paper_2112_13184_amd._binding import ctm_xi_extrapolate
    got = ctm_xi_extrapolate(e1, e2)
    ref = ob.xi_extrapolate(e1, e2)
    assert abs(got[0] - ref[0]) < 1e-12 and abs(got[1] - ref[1]) < 1e-12
