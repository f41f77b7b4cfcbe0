"""Expectation values from a converged environment.  TEST INFRASTRUCTURE ONLY.

Sec. 5.3 of the paper lists what is measured after the CTMRG: one-site
observables, nearest-neighbour two-site observables (with r = (1, 0) the right
neighbour and r = (0, 1) the upper one), correlation functions
C(r, r0) = <A(r0) B(r0 + r)> (Eq. (8)) and the correlation length.  Two-site
operators use the paper's element convention: op[(out_i, out_j), (in_i, in_j)].

Every quantity here is a ratio of two contractions of the same finite patch
(3x3 for one site, 3x4 / 4x3 for a bond), so the normalisation of C and T
drops out.  The patch is contracted column by column: a left boundary
LB[t1, l, t3] = C1 T4 C4, one column per site (T1 above, site, T3 below),
and a right boundary RB[t1, r, t3] = C2 T2 C3.

ln kappa (1x1 cell) is the per-site free energy density of the network,
ln Z(3x3) + ln Z(corners) - ln Z(2x3) - ln Z(3x2) (Orus and Vidal,
PRB 80, 094403).
"""
import numpy as np

from .ctmrg import rotate_site, view_site


def _env_view(env, i, r):
    """(C, T, A) of site i in the frame rotated r quarter turns."""
    C = [env.C[i][(m + r) % 4] for m in range(4)]
    T = [env.T[i][(m + r) % 4] for m in range(4)]
    return C, T, rotate_site(env.A[i], r)


def left_boundary(C1, T4, C4):
    # C1[t1, a], T4[b, a, l], C4[b, t3] -> LB[t1, l, t3]
    X = np.tensordot(C1, T4, axes=([1], [1]))          # [t1, b, l]
    return np.tensordot(X, C4, axes=([1], [0]))        # [t1, l, t3]


def right_boundary(C2, T2, C3):
    # C2[a, t1], T2[a, b, r], C3[t3, b] -> RB[t1, r, t3]
    X = np.tensordot(C2, T2, axes=([0], [0]))          # [t1, b, r]
    return np.tensordot(X, C3, axes=([1], [1]))        # [t1, r, t3]


def column(LB, T1, T3, A, layers, open_phys=False):
    """Push the boundary LB[t1, l, t3 (, extra...)] through one column.

    T1[t1, t1', u] sits above the site, T3[t3', t3, d] below.  With open_phys
    the ket and bra physical indices p, p' are left open and appended.
    Returns LB'[t1', r, t3' (, extra..., p, p')].
    """
    extra = LB.shape[3:]
    ne = len(extra)
    X = np.tensordot(LB, T1, axes=([0], [0]))          # [l, t3, e.., t1', u]
    if layers == 2:
        D = A.shape[0]
        d = A.shape[4]
        X = X.reshape((D, D) + X.shape[1:-1] + (D, D))  # [l, l', t3, e.., t1', u, u']
        # ket: sum l, u
        ax_u = 3 + ne + 1
        X = np.tensordot(X, A, axes=([0, ax_u], [0, 1]))  # [l', t3, e.., t1', u', r, d, p]
        # bra: sum l', u' (and p unless open)
        ax_up = 1 + 1 + ne + 1
        if open_phys:
            Y = np.tensordot(X, A.conj(), axes=([0, ax_up], [0, 1]))
            # Y axes: t3, e(ne), t1', r, d, p, r', d', p'
            order = [1 + ne, 2 + ne, 5 + ne, 0, 3 + ne, 6 + ne] + list(range(1, 1 + ne)) + [4 + ne, 7 + ne]
            Y = Y.transpose(order)                      # [t1', r, r', t3, d, d', e.., p, p']
            sh = Y.shape
            Y = Y.reshape((sh[0], D * D, sh[3], D * D) + sh[6:])   # [t1', R, t3, Dd, e.., p, p']
        else:
            Y = np.tensordot(X, A.conj(), axes=([0, ax_up, 4 + ne + 2], [0, 1, 4]))
            # Y axes: t3, e(ne), t1', r, d, r', d'
            order = [1 + ne, 2 + ne, 4 + ne, 0, 3 + ne, 5 + ne] + list(range(1, 1 + ne))
            Y = Y.transpose(order)
            sh = Y.shape
            Y = Y.reshape((sh[0], D * D, sh[3], D * D) + sh[6:])   # [t1', R, t3, Dd, e..]
        # close with T3[t3', t3, d]: sum t3 and Dd
        Z = np.tensordot(Y, T3, axes=([2, 3], [1, 2]))             # [t1', R, e.., (p, p'), t3']
        return np.moveaxis(Z, -1, 2)                               # [t1', R, t3', e.., (p, p')]
    # classical network: A = a[l, u, r, d]
    X = np.tensordot(X, A, axes=([0, 2 + ne + 1], [0, 1]))         # [t3, e.., t1', r, d]
    Z = np.tensordot(X, T3, axes=([0, 3 + ne], [1, 2]))            # [e.., t1', r, t3']
    return np.moveaxis(Z, [ne, ne + 1, ne + 2], [0, 1, 2])


def _close(LB, RB):
    """Contract LB[t1, x, t3, e..] with RB[t1, x, t3] -> e.."""
    return np.tensordot(LB, RB, axes=([0, 1, 2], [0, 1, 2]))


def rho_one_site(env, i):
    """rho[p, p'] of site i from the 3x3 patch (ket index first)."""
    C, T, A = _env_view(env, i, 0)
    LB = left_boundary(C[0], T[3], C[3])
    RB = right_boundary(C[1], T[1], C[2])
    X = column(LB, T[0], T[2], A, env.layers, open_phys=True)
    return _close(X, RB)


def rho_bond(env, i, direction):
    """rho[(p_s, p_t), (p_s', p_t')] for s = i and t = s + x (direction 0) or s + y (1).

    The vertical bond is measured as a horizontal one in the frame rotated
    three quarter turns counter-clockwise, where +y becomes +x.
    """
    r = 0 if direction == 0 else 3
    Lx, Ly = env.Lx, env.Ly
    x, y = i % Lx, i // Lx
    for _ in range(r):
        x, y = -y, x                                   # physical -> view coordinates
    s = view_site(Lx, Ly, r, x, y)
    t = view_site(Lx, Ly, r, x + 1, y)
    assert s == i
    Cs, Ts, As = _env_view(env, s, r)
    Ct, Tt, At = _env_view(env, t, r)
    LB = left_boundary(Cs[0], Ts[3], Cs[3])
    RB = right_boundary(Ct[1], Tt[1], Ct[2])
    X = column(LB, Ts[0], Ts[2], As, env.layers, open_phys=True)     # [.., ps, ps']
    X = column(X, Tt[0], Tt[2], At, env.layers, open_phys=True)      # [.., ps, ps', pt, pt']
    R = _close(X, RB)                                                # [ps, ps', pt, pt']
    d = R.shape[0]
    return R.transpose(0, 2, 1, 3).reshape(d * d, d * d)


def expect(rho, op):
    """<O> = sum rho[in, out] O[out, in] / tr rho."""
    return float(np.real(np.sum(rho.T * op) / np.trace(rho)))


def energy_per_site(env, bond_op, onsite_op=None):
    """(1/N) sum_s (<h_{s,s+x}> + <h_{s,s+y}> + <h_s>); each bond counted once."""
    N = env.Lx * env.Ly
    e = 0.0
    for i in range(N):
        e += expect(rho_bond(env, i, 0), bond_op)
        e += expect(rho_bond(env, i, 1), bond_op)
        if onsite_op is not None:
            e += expect(rho_one_site(env, i), onsite_op)
    return e / N


def _z3x3(env, i, site_tensor=None):
    C, T, A = _env_view(env, i, 0)
    if site_tensor is not None:
        A = site_tensor
    LB = left_boundary(C[0], T[3], C[3])
    RB = right_boundary(C[1], T[1], C[2])
    X = column(LB, T[0], T[2], A, env.layers)
    return float(_close(X, RB))


def impurity_ratio(env, i, b):
    """Z(b) / Z(a) on the 3x3 patch of site i: b replaces the site tensor."""
    return _z3x3(env, i, np.asarray(b, dtype=np.float64)) / _z3x3(env, i)


def log_kappa(env):
    """ln kappa per site for a 1x1 cell: ln Z3x3 + ln Zc - ln Z2x3 - ln Z3x2."""
    assert env.Lx == 1 and env.Ly == 1
    C, T, _ = _env_view(env, 0, 0)
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    z33 = _z3x3(env, 0)
    # corners only: C1[a, b] C2[c, a] C3[d, c] C4[b, d]
    zc = float(np.einsum("ab,ca,dc,bd->", C1, C2, C3, C4))
    # two rows, three columns: T1's pair leg joins T3's pair leg directly
    LB0 = np.tensordot(C1, C4, axes=([1], [0]))                       # [t1, t3]
    RB0 = np.tensordot(C2, C3, axes=([0], [1]))                       # [t1', t3']
    z23 = float(np.einsum("ab,acu,dbu,cd->", LB0, T1, T3, RB0))
    # three rows, two columns: T4's pair leg joins T2's pair leg directly
    z32 = float(np.einsum("ta,bal,bs,ct,cel,se->", C1, T4, C4, C2, T2, C3))
    vals = np.array([z33, zc, z23, z32])
    if np.any(vals <= 0):
        # signs cancel in the ratio; take magnitudes of the positive combination
        return float(np.log(abs(z33 * zc / (z23 * z32))))
    return float(np.log(z33) + np.log(zc) - np.log(z23) - np.log(z32))


def _line(env, i, direction):
    """Frame and view coordinates for a walk from site i along +x (direction
    0) or +y (1): the +y walk is a +x walk in the frame rotated three quarter
    turns counter-clockwise.  Returns (r, xv, yv)."""
    r = 0 if direction == 0 else 3
    x, y = i % env.Lx, i // env.Lx
    for _ in range(r):
        x, y = -y, x                                   # physical -> view coordinates
    return r, x, y


def correlation(env, i, opA, opB, rmax, direction=0):
    """C(r) = <A(r0) B(r0 + r e)> for r = 0..rmax (Sec. 5.3, Eq. (8)).

    r0 is site i, e = (1, 0) (direction 0) or (0, 1) (direction 1); A and B
    are one-site operators op[out, in].  r = 0 is the one-site expectation
    of the product A B.  For r >= 1 the patch is the left boundary of r0, the
    column of r0 with A inserted, r - 1 plain columns, the column of r0 + r e
    with B inserted and its right boundary, over the same patch without
    operators.  Both boundaries are rescaled by the same factor after every
    column (the ratio is unchanged).
    """
    Lx, Ly = env.Lx, env.Ly
    r_frame, xv, yv = _line(env, i, direction)
    vs = lambda a: view_site(Lx, Ly, r_frame, a, yv)
    assert vs(xv) == i
    out = [expect(rho_one_site(env, i), np.asarray(opA) @ np.asarray(opB))]
    C0, T0, A0 = _env_view(env, i, r_frame)
    LB = left_boundary(C0[0], T0[3], C0[3])
    Xop = column(LB, T0[0], T0[2], A0, env.layers, open_phys=True)
    Xop = np.tensordot(Xop, opA, axes=([3, 4], [1, 0]))       # sum_{p,p'} X[p,p'] A[p',p]
    Xid = column(LB, T0[0], T0[2], A0, env.layers)
    for dist in range(1, rmax + 1):
        j = vs(xv + dist)
        Cj, Tj, Aj = _env_view(env, j, r_frame)
        RB = right_boundary(Cj[1], Tj[1], Cj[2])
        num_col = column(Xop, Tj[0], Tj[2], Aj, env.layers, open_phys=True)
        den_col = column(Xid, Tj[0], Tj[2], Aj, env.layers)
        num = np.tensordot(_close(num_col, RB), opB, axes=([0, 1], [1, 0]))
        den = _close(den_col, RB)
        out.append(float(np.real(num / den)))
        Xop = column(Xop, Tj[0], Tj[2], Aj, env.layers)
        Xid = den_col
        sc = np.max(np.abs(Xid))
        Xop, Xid = Xop / sc, Xid / sc
    return np.array(out)


def transfer_apply(env, line, direction):
    """The transfer matrix of one period of the unit cell along +x (direction
    0, in row `line`) or +y (direction 1, in column `line`), as a function on
    flattened left boundaries LB[t1, l, t3]: the columns (T1 above, the
    double-layer site, T3 below) of the period's sites, in order.  Returns
    (apply, dim, period)."""
    Lx, Ly = env.Lx, env.Ly
    i = (0 + Lx * line) if direction == 0 else (line + 0)
    r_frame, xv, yv = _line(env, i, direction)
    period = Lx if direction == 0 else Ly
    cols = []
    for k in range(period):
        C, T, A = _env_view(env, view_site(Lx, Ly, r_frame, xv + k, yv), r_frame)
        cols.append((T[0], T[2], A))
    shape = (cols[0][0].shape[0], env.Db, cols[0][1].shape[1])

    def apply(v):
        X = np.asarray(v).reshape(shape)
        for T1, T3, A in cols:
            X = column(X, T1, T3, A, env.layers)
        return X.reshape(-1)

    return apply, int(np.prod(shape)), period


def transfer_spectrum(env, line, direction, nev=4):
    """The nev eigenvalues of largest modulus of the transfer matrix of one
    period (sorted by modulus, descending, complex).  Dense eigenvalues of
    the formed matrix up to dimension 3000, else ARPACK (implicitly
    restarted Arnoldi) through scipy."""
    apply, dim, _ = transfer_apply(env, line, direction)
    if dim <= 3000:
        M = np.empty((dim, dim))
        e = np.zeros(dim)
        for c in range(dim):
            e[c] = 1.0
            M[:, c] = apply(e)
            e[c] = 0.0
        lam = np.linalg.eigvals(M)
    else:
        from scipy.sparse.linalg import LinearOperator, eigs
        op = LinearOperator((dim, dim), matvec=apply, dtype=np.float64)
        lam = eigs(op, k=min(nev, dim - 2), which="LM", return_eigenvectors=False, tol=1e-13, ncv=40)
    lam = lam[np.argsort(-np.abs(lam), kind="stable")]
    return lam[:nev]


def correlation_length(lam, period):
    """(xi, e) from transfer-matrix eigenvalues (Sec. 5.3): e_k =
    -log|lam_k / lam_0| per lattice spacing (the matrix spans `period`
    sites), xi = 1 / e_1."""
    lam = np.asarray(lam)
    with np.errstate(divide="ignore"):
        e = -np.log(np.abs(lam[1:]) / np.abs(lam[0])) / period
    return (1.0 / e[0] if e[0] > 0 else np.inf), e


def xi_extrapolate(e1, e2):
    """Finite-chi extrapolation of Eq. (9) over runs at several chi: the
    least-squares line e1 = 1/xi(inf) - k (e2 - e1).  Returns (1/xi(inf), k)."""
    e1, e2 = np.asarray(e1, dtype=np.float64), np.asarray(e2, dtype=np.float64)
    delta = e2 - e1
    Amat = np.stack([np.ones_like(delta), -delta], axis=1)
    (inv_xi, k), *_ = np.linalg.lstsq(Amat, e1, rcond=None)
    return float(inv_xi), float(k)
