"""Simple-update imaginary-time evolution and the mean-field environment, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU library never
imports this module.

What this follows
-----------------
* Sec. 2.3, Eqs. (1)-(3): the ground state is approached by imaginary-time
  evolution; the evolution operator is split by a first-order Suzuki-Trotter
  decomposition into a product of two-site gates exp(-tau H_ij), applied
  N_tau times.
* Sec. 2.3, Eq. (4) and the paragraph after it: after each gate the bond
  dimension is truncated back to D so that the new state is as close as
  possible to the gated one, with the rest of the network replaced by the
  mean-field environment (simple update, Jiang, Weng and Xiang, PRL 101,
  090603).
* Sec. 2.2, MFE paragraph: the mean-field environment of a tensor (or of a
  1 x 2 cluster) is a diagonal matrix of bond weights on every open virtual
  bond, taken from the singular values of the simple update; contracting the
  ket, the bra and those matrices gives local expectation values at O(D^4)
  (one site) or O(D^5) (a bond) cost, without the variational property of
  CTMRG.

State (Vidal form on the square lattice, the paper leaves its storage open)
--------------------------------------------------------------------------
* Site tensors G[s][l, u, r, d, p] (D^4 d values), site s = x + Lx * y,
  +y up, as in the CTMRG oracle.
* Bond weights lam_h[s] (D,) on the bond between s and its right neighbour
  ((x + 1) mod Lx, y), lam_v[s] (D,) on the bond between s and its upper
  neighbour (x, (y + 1) mod Ly).  Leg l of s carries lam_h of its left
  neighbour, u carries lam_v[s], r carries lam_h[s], d carries lam_v of its
  lower neighbour.  Lx >= 2 and Ly >= 2, so that every bond joins two
  different tensors.
* The iTPS the state stands for has A_s = G_s times sqrt(weight) on each leg.

Readings (the paper does not fix these)
---------------------------------------
* One Trotter step applies the gates of the horizontal bonds of sites
  0 .. N-1, then those of the vertical bonds of sites 0 .. N-1; each bond has
  its own two-site Hamiltonian H[s][dir][(out_i, out_j), (in_i, in_j)], i = s
  and j its right (dir 0) or upper (dir 1) neighbour; the gate is
  expm(-tau H).
* Bond update (i, j, shared weight lam): A_i = G_i with its three other legs
  multiplied by their weights, likewise A_j;
  Psi[(a, p), (b, q)] = sum_k A_i[a, k, p] lam[k] A_j[b, k, q] (a, b the
  three other legs in leg order, C order); Psi' = gate applied to (p, q);
  Psi' = U S V^T; the D largest triplets are kept;
  lam' = S[:D] / ||S[:D]||_2; G_i' = U[(a, p), k] divided by the weights of
  a, G_j' likewise from V.  A weight w <= 1e-13 is divided out as 0 (its index
  carries no state).
* Sign (phase) of a kept singular pair: the first entry (in (a, p) order) of
  U[:, k] whose modulus is at least (1 - 1e-8) of the column's largest is made
  real and positive, the pair's V column taking the same phase so that
  U S V^H is unchanged.  The tolerance makes the choice insensitive to
  rounding when symmetric entries tie.
* Complex tensors and Hamiltonians (Sec. 5.2 allows complex tensors): the
  bra is the complex conjugate of the ket; the two-site matrix is
  Psi = U S V^H, the new right tensor is the transpose of V^H (no conjugate:
  the ket tensors meet directly on the bond); the weights stay real.
* The initial weights are supplied by the caller (all ones in the tests).

Parity status
-------------
Pinned in tests/test_oracle_pins.py by: a field-only evolution of a product
state (closed form tanh(2 N tau h)); commuting Ising gates from |+x>, whose
exact result has bond dimension 2, against Onsager's nearest-neighbour
correlator (through the CTMRG oracle) and, with vertical gates off, the 1D
value tanh(2 N tau); an isolated two-site dimer evolved by a general gate
against expm(-N tau H) psi_0 (with the MFE, exact for a dimer); D = 1
evolutions against the mean-field TFIM energy and the Neel energy of the
Heisenberg antiferromagnet.
"""
import numpy as np
from scipy.linalg import expm

INV_CUT = 1e-13
SIGN_TOL = 1e-8


def right(Lx, Ly, s):
    x, y = s % Lx, s // Lx
    return (x + 1) % Lx + Lx * y


def left(Lx, Ly, s):
    x, y = s % Lx, s // Lx
    return (x - 1) % Lx + Lx * y


def up(Lx, Ly, s):
    x, y = s % Lx, s // Lx
    return x + Lx * ((y + 1) % Ly)


def down(Lx, Ly, s):
    x, y = s % Lx, s // Lx
    return x + Lx * ((y - 1) % Ly)


def leg_weights(lam_h, lam_v, Lx, Ly, s):
    """Weights on legs (l, u, r, d) of site s."""
    return [lam_h[left(Lx, Ly, s)], lam_v[s], lam_h[s], lam_v[down(Lx, Ly, s)]]


def bond(Lx, Ly, s, direction):
    """(i, leg of i, j, leg of j) of the horizontal (0) or vertical (1) bond of site s."""
    if direction == 0:
        return s, 2, right(Lx, Ly, s), 0
    return s, 1, up(Lx, Ly, s), 3


def gate(H, tau):
    """Trotter gate exp(-tau H) of a two-site Hamiltonian (Eq. (3))."""
    H = np.asarray(H)
    return expm(-tau * (H if np.iscomplexobj(H) else H.astype(np.float64)))


def _scale_legs(G, ws, skip, inverse=False):
    A = G
    for k in range(4):
        if k == skip:
            continue
        w = np.asarray(ws[k], dtype=np.float64)
        if inverse:
            w = np.where(w > INV_CUT, 1.0 / np.where(w > INV_CUT, w, 1.0), 0.0)
        shape = [1] * 5
        shape[k] = -1
        A = A * w.reshape(shape)
    return A


def _leg_last(A, leg):
    """[l, u, r, d, p] -> [three other legs in order, leg, p]."""
    outer = [k for k in range(4) if k != leg]
    return A.transpose(outer + [leg, 4])


def _leg_back(B, leg):
    """Inverse of _leg_last."""
    outer = [k for k in range(4) if k != leg]
    order = outer + [leg, 4]
    inv = [order.index(k) for k in range(5)]
    return B.transpose(inv)


def sign_fix(U, Vt):
    """Sign (phase) rule of the kept singular pairs (see the module docstring)."""
    U = U.copy()
    Vt = Vt.copy()
    for k in range(U.shape[1]):
        col = np.abs(U[:, k])
        m = col.max()
        if m == 0.0:
            continue
        first = int(np.argmax(col >= (1.0 - SIGN_TOL) * m))
        if np.iscomplexobj(U):
            ph = U[first, k] / abs(U[first, k])
            U[:, k] = U[:, k] * np.conj(ph)
            Vt[k, :] = Vt[k, :] * ph
        elif U[first, k] < 0.0:
            U[:, k] = -U[:, k]
            Vt[k, :] = -Vt[k, :]
    return U, Vt


def two_site(Gi, Gj, wi, wj, lam, leg_i, leg_j):
    """Psi[a, p, b, q] of the bond (weights on every other leg, lam on the bond)."""
    Ai = _leg_last(_scale_legs(Gi, wi, leg_i), leg_i)      # [a1 a2 a3, k, p]
    Aj = _leg_last(_scale_legs(Gj, wj, leg_j), leg_j)      # [b1 b2 b3, k, q]
    return np.einsum("abckp,k,efgkq->abcpefgq", Ai, np.asarray(lam, dtype=np.float64), Aj)


def bond_update(Gi, Gj, wi, wj, lam, g, leg_i, leg_j, D):
    """One simple-update step on a bond; returns (Gi', Gj', lam', discarded S)."""
    d = Gi.shape[4]
    Psi = two_site(Gi, Gj, wi, wj, lam, leg_i, leg_j)
    Da = Psi.shape[:3]
    Db = Psi.shape[4:7]
    g4 = np.asarray(g).reshape(d, d, d, d)
    Psi = np.einsum("PQpq,abcpefgq->abcPefgQ", g4, Psi)
    M = Psi.reshape(int(np.prod(Da)) * d, int(np.prod(Db)) * d)
    U, S_all, Vt = np.linalg.svd(M, full_matrices=False)
    U, S, Vt = U[:, :D], S_all[:D].copy(), Vt[:D, :]
    discarded = S_all[D:]
    U, Vt = sign_fix(U, Vt)
    nrm = np.sqrt(np.sum(S * S))
    lam_new = S / nrm
    Bi = U.reshape(*Da, d, D).transpose(0, 1, 2, 4, 3)      # [a, k, p]
    Bj = Vt.T.reshape(*Db, d, D).transpose(0, 1, 2, 4, 3)
    Gi_new = _scale_legs(_leg_back(Bi, leg_i), wi, leg_i, inverse=True)
    Gj_new = _scale_legs(_leg_back(Bj, leg_j), wj, leg_j, inverse=True)
    return Gi_new, Gj_new, lam_new, discarded


def trotter_step(G, lam_h, lam_v, gates, Lx, Ly, D):
    """One first-order Trotter step in place; gates[s][dir] is a d^2 x d^2 gate."""
    N = Lx * Ly
    worst = 0.0
    for direction in (0, 1):
        for s in range(N):
            i, li, j, lj = bond(Lx, Ly, s, direction)
            lam_b = lam_h[s] if direction == 0 else lam_v[s]
            wi = leg_weights(lam_h, lam_v, Lx, Ly, i)
            wj = leg_weights(lam_h, lam_v, Lx, Ly, j)
            Gi, Gj, lam_new, disc = bond_update(G[i], G[j], wi, wj, lam_b, gates[s][direction], li, lj, D)
            G[i], G[j] = Gi, Gj
            if direction == 0:
                lam_h[s] = lam_new
            else:
                lam_v[s] = lam_new
            if disc.size:
                worst = max(worst, float(disc[0] / max(np.sqrt(np.sum(np.asarray(lam_new) ** 2)), 1e-300)))
    return worst


def simple_update(G, lam_h, lam_v, H, tau, Lx, Ly, nsteps):
    """nsteps Trotter steps of the bond Hamiltonians H[s][dir] at time step tau.

    Returns new (G, lam_h, lam_v) lists; the inputs are not modified."""
    assert Lx >= 2 and Ly >= 2
    cplx = any(np.iscomplexobj(g) for g in G) or any(np.iscomplexobj(np.asarray(h)) for row in H for h in row)
    G = [np.array(g, dtype=np.complex128 if cplx else np.float64) for g in G]
    lam_h = [np.array(v, dtype=np.float64) for v in lam_h]
    lam_v = [np.array(v, dtype=np.float64) for v in lam_v]
    D = G[0].shape[0]
    gates = [[gate(H[s][0], tau), gate(H[s][1], tau)] for s in range(Lx * Ly)]
    for _ in range(nsteps):
        trotter_step(G, lam_h, lam_v, gates, Lx, Ly, D)
    return G, lam_h, lam_v


def to_itps(G, lam_h, lam_v, Lx, Ly):
    """Site tensors of the iTPS: G_s with sqrt(weight) on each of its legs."""
    out = []
    for s in range(Lx * Ly):
        ws = [np.sqrt(np.asarray(w)) for w in leg_weights(lam_h, lam_v, Lx, Ly, s)]
        out.append(_scale_legs(G[s], ws, skip=-1))
    return out


def weighted(G, lam_h, lam_v, Lx, Ly):
    """G_s with the full weight on every leg (the gauge-independent form the
    GPU parity tests compare: indices of a zero weight carry nothing)."""
    return [_scale_legs(G[s], leg_weights(lam_h, lam_v, Lx, Ly, s), skip=-1) for s in range(Lx * Ly)]


# ---------------------------------------------------------------------------
# Mean-field environment (Sec. 2.2)
# ---------------------------------------------------------------------------
def mfe_rho_site(G, lam_h, lam_v, Lx, Ly, s):
    """rho[p, p'] (ket, bra) of site s: the weights squared on all four legs
    (each leg's weight once on the ket and once on the bra).  Not normalised."""
    A = _scale_legs(G[s], leg_weights(lam_h, lam_v, Lx, Ly, s), skip=-1)
    d = A.shape[4]
    A = A.reshape(-1, d)
    return A.T @ A.conj()


def mfe_rho_bond(G, lam_h, lam_v, Lx, Ly, s, direction):
    """rho[(p_i, p_j), (p_i', p_j')] of the bond (s, s + x) (direction 0) or
    (s, s + y) (1): the 1 x 2 cluster of Psi with weights on its six open legs,
    contracted with its copy.  Not normalised."""
    i, li, j, lj = bond(Lx, Ly, s, direction)
    lam_b = lam_h[s] if direction == 0 else lam_v[s]
    wi = leg_weights(lam_h, lam_v, Lx, Ly, i)
    wj = leg_weights(lam_h, lam_v, Lx, Ly, j)
    Psi = two_site(G[i], G[j], wi, wj, lam_b, li, lj)       # [a, p, b, q]
    d = G[i].shape[4]
    Da = int(np.prod(Psi.shape[:3]))
    X = Psi.reshape(Da, d, Da, d).transpose(1, 3, 0, 2).reshape(d * d, Da * Da)
    return X @ X.conj().T


def expect(rho, op):
    """<O> = sum rho[in, out] O[out, in] / tr rho (real part: Hermitian O)."""
    return float(np.real(np.sum(rho.T * op) / np.trace(rho)))


def mfe_energy(G, lam_h, lam_v, Lx, Ly, H, onsite=None):
    """(1/N) sum_s (<H[s][0]> + <H[s][1]> + <onsite>) in the mean-field environment."""
    N = Lx * Ly
    e = 0.0
    for s in range(N):
        for direction in (0, 1):
            e += expect(mfe_rho_bond(G, lam_h, lam_v, Lx, Ly, s, direction), H[s][direction])
        if onsite is not None:
            e += expect(mfe_rho_site(G, lam_h, lam_v, Lx, Ly, s), onsite)
    return e / N
