"""Full-update imaginary-time evolution, plain FP64.  TEST INFRASTRUCTURE ONLY.

What this follows
-----------------
* Sec. 2.3, Eqs. (1)-(4): after each Trotter gate exp(-tau H_ij) the bond is
  truncated back to D by minimising || Psi_new - exp(-tau H_ij) Psi || (Eq. (4));
  the full update evaluates that norm with the CTMRG environment of the
  bond (the simple update with the mean-field one).  The method is that of
  Jordan et al. (PRL 101, 250602) in the reduced-tensor form of Phien et al.
  (PRB 92, 035142).

Steps of one bond update (i, j), tensors A_s[l, u, r, d, p] of the iTPS
(no bond weights), the CTMRG environment of the current tensors:
1. reduced tensors: A_i as the matrix [(three other legs), (bond k, p)] =
   X_i a_i (QR; X_i D^3 x r with orthonormal columns, a_i r x D d), likewise j;
2. bond environment N[(rho_i, rho_j), (rho_i', rho_j')]: the two-site patch of
   the environment (3x4, or 4x3 for a vertical bond, as for a bond density
   matrix) with X_i and X_j in place of the sites, the bond between them cut,
   and their reduced legs open on ket (rho) and bra (rho'); divided by its
   trace;
3. N <- (N + N^T) / 2 with its negative eigenvalues set to zero;
4. Theta'[(rho_i, P), (rho_j, Q)] = sum_{p q} g[(P Q), (p q)] sum_k a_i[rho_i, (k p)] a_j[rho_j, (k q)];
5. start: Theta' = U S V^T, b_i = U[:, :D] sqrt(S), b_j = V[:, :D] sqrt(S);
6. alternating least squares: the cost
     d(b_i, b_j) = sum_{P Q} (psi - Theta')[rho_i P, rho_j Q] N[(rho_i rho_j), (rho_i' rho_j')] (psi - Theta')[rho_i' P, rho_j' Q],
     psi[(rho_i P), (rho_j Q)] = sum_k b_i[(rho_i P), k] b_j[(rho_j Q), k],
   is quadratic in each factor; b_i <- pinv(R_i) S_i with
     R_i[(rho_i k), (rho_i' k')] = sum_{rho_j rho_j' Q} N[(rho_i rho_j), (rho_i' rho_j')] b_j[(rho_j Q), k] b_j[(rho_j' Q), k'],
     S_i[(rho_i k), P]          = sum N[(rho_i rho_j), (rho_i' rho_j')] b_j[(rho_j Q), k] Theta'[(rho_i' P), (rho_j' Q)],
   then b_j likewise; als_iters rounds (i then j);
7. A_i' = X_i b_i reshaped to [l, u, r, d, p] with k on the bond leg,
   likewise A_j'; sign rule; each divided by its largest |entry|;
8. env_sweeps CTMRG sweeps from the current environment (warm start).

Readings (the paper leaves these open)
--------------------------------------
* The Trotter order is that of the simple update (horizontal bonds of sites
  0..N-1, then vertical ones), every bond its own Hamiltonian.
* A fixed number of ALS rounds (no stopping test), pseudo-inverse with
  eigenvalues <= 1e-12 of the largest dropped; no further gauge fixing of N
  beyond the symmetric positive projection of step 3.
* Sign rule of bond index k: the first entry of A_i'[.., k, ..] (remaining
  indices in C order) whose modulus is within 1e-8 of the largest is made
  positive; A_j'[.., k, ..] is flipped with it.
* The environment is updated by env_sweeps full CTMRG sweeps after every
  bond update.

Parity status
-------------
Pinned in tests/test_oracle_fu_pins.py: contracting N with the untruncated
pair a_i a_j reproduces the CTMRG bond density matrix of the separately
pinned observables module (both bond directions); the ALS result is
stationary for the directly evaluated cost (finite differences) and that
cost decreases monotonically and ends at or below the simple-update
truncation's; commuting Ising gates from |+x> (exact at D = 2) reach
Onsager's nearest-neighbour correlator; isolated dimers follow
expm(-N tau H) psi_0.
"""
import numpy as np

from .ctmrg import rotate_site, view_site
from .observables import _env_view, _close, column, left_boundary, right_boundary
from .simple_update import SIGN_TOL, bond, gate

PINV_CUT = 1e-12


def _leg_last(A, leg):
    outer = [k for k in range(4) if k != leg]
    return A.transpose(outer + [leg, 4])


def _leg_back(B, leg):
    outer = [k for k in range(4) if k != leg]
    order = outer + [leg, 4]
    return B.transpose([order.index(k) for k in range(5)])


def reduce_site(A, leg):
    """Step 1: X (D^3 x r, orthonormal columns) and a (r x D d), A = X a."""
    D, d = A.shape[0], A.shape[4]
    M = _leg_last(A, leg).reshape(D ** 3, D * d)
    X, a = np.linalg.qr(M)
    return X, a


def embed(X, leg, D):
    """[l, u, r, d, rho]: X on the other legs (in leg order), the bond leg pinned to 0."""
    r = X.shape[1]
    out = np.zeros((D, D, D, D, r))
    idx = [slice(None)] * 5
    idx[leg] = 0
    out[tuple(idx)] = X.reshape(D, D, D, r)
    return out


def bond_environment(env, s, direction, Ei, Ej):
    """Step 2: N[(rho_i, rho_j), (rho_i', rho_j')] for the bond (s, s + x) or
    (s, s + y) with the embedded reduced tensors Ei, Ej (physical frame)."""
    r = 0 if direction == 0 else 3
    Lx, Ly = env.Lx, env.Ly
    x, y = s % Lx, s // Lx
    for _ in range(r):
        x, y = -y, x
    si = view_site(Lx, Ly, r, x, y)
    ti = view_site(Lx, Ly, r, x + 1, y)
    assert si == s
    Cs, Ts, _ = _env_view(env, si, r)
    Ct, Tt, _ = _env_view(env, ti, r)
    LB = left_boundary(Cs[0], Ts[3], Cs[3])
    RB = right_boundary(Ct[1], Tt[1], Ct[2])
    X = column(LB, Ts[0], Ts[2], rotate_site(Ei, r), 2, open_phys=True)
    X = column(X, Tt[0], Tt[2], rotate_site(Ej, r), 2, open_phys=True)
    R = _close(X, RB)                                   # [ri, ri', rj, rj']
    n = R.shape[0]
    N = R.transpose(0, 2, 1, 3).reshape(n * n, n * n)
    return N / np.trace(N)


def positive_part(N):
    """Step 3."""
    Ns = 0.5 * (N + N.T)
    w, V = np.linalg.eigh(Ns)
    return (V * np.maximum(w, 0.0)) @ V.T


def gated_core(ai, aj, g, D, d):
    """Step 4: Theta'[(rho_i, P), (rho_j, Q)]."""
    ri, rj = ai.shape[0], aj.shape[0]
    A = ai.reshape(ri, D, d)
    B = aj.reshape(rj, D, d)
    T = np.einsum("xkp,ykq->xpyq", A, B)
    G = np.asarray(g).reshape(d, d, d, d)
    return np.einsum("PQpq,xpyq->xPyQ", G, T).reshape(ri * d, rj * d)


def cost(bi, bj, N, Th, d):
    """d(b_i, b_j) of step 6, evaluated directly."""
    ri, rj = bi.shape[0] // d, bj.shape[0] // d
    diff = (bi @ bj.T - Th).reshape(ri, d, rj, d).transpose(0, 2, 1, 3).reshape(ri * rj, d * d)
    return float(np.sum(diff * (N @ diff)))


def _pinv_solve(R, S):
    w, V = np.linalg.eigh(0.5 * (R + R.T))
    keep = w > PINV_CUT * max(w.max(), 0.0)
    inv = np.where(keep, 1.0 / np.where(keep, w, 1.0), 0.0)
    return (V * inv) @ (V.T @ S)


def als_left(bj, N, Th, d, D):
    """b_i minimising the cost with b_j fixed."""
    rj = bj.shape[0] // d
    ri = Th.shape[0] // d
    N4 = N.reshape(ri, rj, ri, rj)
    Bj = bj.reshape(rj, d, D)
    Rm = np.einsum("xyXY,yQk,YQK->xkXK", N4, Bj, Bj).reshape(ri * D, ri * D)
    Th4 = Th.reshape(ri, d, rj, d)
    Sm = np.einsum("xyXY,yQk,XPYQ->xkP", N4, Bj, Th4).reshape(ri * D, d)
    X = _pinv_solve(Rm, Sm).reshape(ri, D, d)
    return X.transpose(0, 2, 1).reshape(ri * d, D)


def als_right(bi, N, Th, d, D):
    """b_j minimising the cost with b_i fixed."""
    ri = bi.shape[0] // d
    rj = Th.shape[1] // d
    N4 = N.reshape(ri, rj, ri, rj)
    Bi = bi.reshape(ri, d, D)
    Rm = np.einsum("xyXY,xPk,XPK->ykYK", N4, Bi, Bi).reshape(rj * D, rj * D)
    Th4 = Th.reshape(ri, d, rj, d)
    Sm = np.einsum("xyXY,xPk,XPYQ->ykQ", N4, Bi, Th4).reshape(rj * D, d)
    X = _pinv_solve(Rm, Sm).reshape(rj, D, d)
    return X.transpose(0, 2, 1).reshape(rj * d, D)


def svd_start(Th, D):
    """Step 5."""
    U, S, Vt = np.linalg.svd(Th)
    sq = np.sqrt(S[:D])
    return U[:, :D] * sq, Vt[:D].T * sq


def sign_fix(Ai, Aj, li, lj):
    Ai, Aj = Ai.copy(), Aj.copy()
    for k in range(Ai.shape[li]):
        v = np.take(Ai, k, axis=li).reshape(-1)
        m = np.abs(v).max()
        if m == 0.0:
            continue
        first = int(np.argmax(np.abs(v) >= (1.0 - SIGN_TOL) * m))
        if v[first] < 0.0:
            idx_i = [slice(None)] * 5
            idx_i[li] = k
            Ai[tuple(idx_i)] *= -1.0
            idx_j = [slice(None)] * 5
            idx_j[lj] = k
            Aj[tuple(idx_j)] *= -1.0
    return Ai, Aj


def bond_update(env, s, direction, g, als_iters, history=None):
    """Steps 1-7 on the bond of site s; replaces env.A[i], env.A[j]."""
    i, li, j, lj = bond(env.Lx, env.Ly, s, direction)
    Ai, Aj = env.A[i], env.A[j]
    D, d = Ai.shape[0], Ai.shape[4]
    Xi, ai = reduce_site(Ai, li)
    Xj, aj = reduce_site(Aj, lj)
    N = positive_part(bond_environment(env, s, direction, embed(Xi, li, D), embed(Xj, lj, D)))
    Th = gated_core(ai, aj, g, D, d)
    bi, bj = svd_start(Th, D)
    if history is not None:
        history.append(cost(bi, bj, N, Th, d))
    for _ in range(als_iters):
        bi = als_left(bj, N, Th, d, D)
        bj = als_right(bi, N, Th, d, D)
        if history is not None:
            history.append(cost(bi, bj, N, Th, d))
    ri, rj = Xi.shape[1], Xj.shape[1]
    Bi = (Xi @ bi.reshape(ri, d * D)).reshape(D, D, D, d, D).transpose(0, 1, 2, 4, 3)   # [o1 o2 o3, k, P]
    Bj = (Xj @ bj.reshape(rj, d * D)).reshape(D, D, D, d, D).transpose(0, 1, 2, 4, 3)
    Ai_new, Aj_new = sign_fix(_leg_back(Bi, li), _leg_back(Bj, lj), li, lj)
    env.A[i] = Ai_new / np.abs(Ai_new).max()
    env.A[j] = Aj_new / np.abs(Aj_new).max()
    return N, Th, bi, bj


def full_update_step(env, H, tau, als_iters=5, env_sweeps=1):
    """One Trotter step of the full update on env (tensors and environment in place)."""
    N = env.Lx * env.Ly
    for direction in (0, 1):
        for s in range(N):
            bond_update(env, s, direction, gate(H[s][direction], tau), als_iters)
            for _ in range(env_sweeps):
                env.sweep()
