"""Expectation values from a converged environment.  TEST INFRASTRUCTURE ONLY.

Sec. 4.5 of the paper lists what is measured after the CTMRG: one-site
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


def correlation_x(env, i, opA, opB, rmax):
    """C(r) = <A(s) B(s + r x)> for r = 1..rmax along +x (Eq. (8))."""
    Lx = env.Lx
    y = i // Lx
    out = []
    C0, T0, A0 = _env_view(env, i, 0)
    LB = left_boundary(C0[0], T0[3], C0[3])
    Xop = column(LB, T0[0], T0[2], A0, env.layers, open_phys=True)
    Xop = np.tensordot(Xop, opA, axes=([3, 4], [1, 0]))       # apply A: sum_{p,p'} X[p,p'] A[p',p]
    Xid = column(LB, T0[0], T0[2], A0, env.layers)
    x = i % Lx
    for r in range(1, rmax + 1):
        j = ((x + r) % Lx) + Lx * y
        Cj, Tj, Aj = _env_view(env, j, 0)
        RB = right_boundary(Cj[1], Tj[1], Cj[2])
        num_col = column(Xop, Tj[0], Tj[2], Aj, env.layers, open_phys=True)
        den_col = column(Xid, Tj[0], Tj[2], Aj, env.layers)
        num = np.tensordot(_close(num_col, RB), opB, axes=([0, 1], [1, 0]))
        den = _close(den_col, RB)
        out.append(float(num / den))
        Xop = column(Xop, Tj[0], Tj[2], Aj, env.layers)
        Xid = den_col
        # keep the scale of both boundaries comparable
        sc = np.max(np.abs(Xid))
        Xop, Xid = Xop / sc, Xid / sc
    return np.array(out)
