"""CTMRG for an iTPS on an Lx x Ly unit cell, plain FP64.  TEST INFRASTRUCTURE ONLY.

What this follows
-----------------
* Sec. 2.2 and Fig. 2: the norm network is the double layer of ket and bra
  site tensors, read as one tensor of bond dimension D**2; the environment of
  every site is four corner matrices C (chi x chi) and four edge tensors T
  (chi x chi x D**2), fixed iteratively.
* Sec. 2.2: the directional-move CTMRG for arbitrary unit cells of Corboz et
  al. (PRL 113, 046402), modified so that no QR of the half systems is done,
  and with the SVD taken as a partial (randomized, Halko et al. 2011) SVD that
  only applies the matrix to vectors.
* Sec. 5.2 / 5.3: bra = complex conjugate of ket; +y points up.

Conventions (the paper leaves these open; each one is a reading)
-----------------------------------------------------------------
* Site tensor A[l, u, r, d, p]; a classical (single-layer) network has
  a[l, u, r, d].  Site index i = x + Lx * y.
* Pair index of a double-layer bond = ket * D + bra, dimension Db = D**2
  (Db = D for a classical network).
* The eight environment tensors of site s are stored clockwise,
  C1 T1 C2 T2 C3 T3 C4 T4 (C1 upper-left, T1 above, ...).  A corner is
  C_k[next, prev] and an edge T_k[prev, next, pair], where next/prev name the
  clockwise neighbour.  With this rule a 90-degree rotation of the lattice
  only relabels tensors: C_k -> C_{k-1}, T_k -> T_{k-1}, A -> A.transpose(1,2,3,0,4).
* The left move absorbs columns x = 0..Lx-1 in order; all projectors of one
  column come from the environment before that column is updated.  Up, right
  and down moves are left moves on the lattice rotated by 1, 2, 3 quarter
  turns counter-clockwise.  A sweep is left, right, up, down.
* Projectors of the cut between rows y and y-1 at column x, with the four
  enlarged corners G (each G[next, prev], n x n with n = chi*Db):
      M  = G_UR G_UL G_LL G_LR,      H_u = G_UR G_UL,   H_d' = G_LL G_LR,
      M  = U S V^T (top k),  P = S^-1/2 U^T H_u,  Pt = H_d' V S^-1/2.
  The side above the cut takes Pt, the side below takes P.  With QR factors
  H_u = Q_u R_u the same U, S, V describe R_u R_d^T, so skipping the QR
  changes nothing (the claim of Sec. 2.2).
* If the cut bond has n_alpha <= chi, P = Pt = identity (nothing is
  discarded, the environment stays exact).  Otherwise exactly chi singular
  triplets are kept; those with sigma_i <= cutoff * sigma_0 get zero
  projector rows / columns, so bond dimensions depend only on shapes.  Nor
  is any singular value past the smallest bond of the four-corner product
  kept (it can only be rounding noise).
* Sign of each singular pair: the entry of largest modulus of U[:, i] (first
  one on ties) is made positive.
* Every new C and T is divided by its largest absolute entry.
* Convergence: singular values of every corner, normalised to sum 1;
  delta = max over corners of sum |s_new - s_old| (zero padded).
"""
import numpy as np

from .philox import omega_matrix_fast, stream_id

SWEEP_ROTATIONS = (0, 2, 1, 3)  # left, right, up, down as rotations of a left move


def rotate_site(A, j):
    """Site tensor of the lattice rotated j quarter turns counter-clockwise."""
    perm = (1, 2, 3, 0, 4)[:A.ndim]
    for _ in range(j % 4):
        A = A.transpose(perm)
    return A


def view_dims(Lx, Ly, r):
    return (Lx, Ly) if r % 2 == 0 else (Ly, Lx)


def view_site(Lx, Ly, r, xv, yv):
    """Physical site index of view position (xv, yv) in the frame rotated r quarter turns."""
    x, y = xv, yv
    for _ in range(r % 4):
        x, y = y, -x  # inverse of (x, y) -> (-y, x)
    return (x % Lx) + Lx * (y % Ly)


class Environment:
    """Site tensors plus the eight CTM tensors of every site of the unit cell."""

    def __init__(self, tensors, Lx, Ly, chi, layers=2, boundary=None, cutoff=1e-12,
                 mode="rsvd", oversample=32, power_iters=1, seed=0):
        self.Lx, self.Ly, self.chi, self.layers = Lx, Ly, chi, layers
        self.A = [np.asarray(t, dtype=np.float64) for t in tensors]
        assert len(self.A) == Lx * Ly
        self.D = self.A[0].shape[0]
        self.Db = self.D * self.D if layers == 2 else self.D
        self.cutoff, self.mode = cutoff, mode
        self.oversample, self.power_iters, self.seed = oversample, power_iters, seed
        self.moves = 0
        if boundary is None:
            if layers == 2:
                boundary = np.eye(self.D).reshape(-1)  # pair (ket, bra) = delta
            else:
                boundary = np.ones(self.D)
        boundary = np.asarray(boundary, dtype=np.float64).reshape(self.Db)
        self.C = [[np.ones((1, 1)) for _ in range(4)] for _ in range(Lx * Ly)]
        self.T = [[boundary.reshape(1, 1, self.Db).copy() for _ in range(4)]
                  for _ in range(Lx * Ly)]

    # -- building blocks ---------------------------------------------------
    def site(self, i, j):
        return rotate_site(self.A[i], j)

    def corner(self, i, j):
        """Enlarged corner j (0:C1 .. 3:C4) of site i as an n_next x n_prev matrix."""
        return enlarged_corner(self.C[i][j], self.T[i][j], self.T[i][(j - 1) % 4],
                               self.site(i, j), self.layers)

    def left_move(self, r):
        """One left move in the frame rotated r quarter turns (Sec. 2.2)."""
        Lx, Ly = view_dims(self.Lx, self.Ly, r)
        vs = lambda xv, yv: view_site(self.Lx, self.Ly, r, xv, yv)
        for x in range(Lx):
            proj = {}
            for y in range(Ly):
                G_ul = self.corner(vs(x, y), (0 + r) % 4)
                G_ur = self.corner(vs(x + 1, y), (1 + r) % 4)
                G_lr = self.corner(vs(x + 1, y - 1), (2 + r) % 4)
                G_ll = self.corner(vs(x, y - 1), (3 + r) % 4)
                # rows of the sketch are the prev leg of G_lr: its chi bond is T_prev's far leg
                nc_beta = G_lr.shape[1] // self.Db
                sid = stream_id(self.moves, x, y % Ly)
                proj[y % Ly] = projectors(G_ur, G_ul, G_ll, G_lr, self.chi, self.cutoff,
                                          self.mode, self.oversample, self.power_iters,
                                          self.seed, sid, nc_beta, self.Db)
            new = {}
            for y in range(Ly):
                s, t = vs(x, y), vs(x + 1, y)
                P_dn, Pt_dn = proj[y % Ly]
                P_up, Pt_up = proj[(y + 1) % Ly]
                c1 = (0 + r) % 4
                c4 = (3 + r) % 4
                t1, t3, t4 = (0 + r) % 4, (2 + r) % 4, (3 + r) % 4
                C1n = renorm_corner_upper(self.C[s][c1], self.T[s][t1], Pt_up)
                T4n = renorm_edge(self.T[s][t4], self.site(s, r), P_up, Pt_dn, self.layers)
                C4n = renorm_corner_lower(self.C[s][c4], self.T[s][t3], P_dn)
                new[t] = (C1n, T4n, C4n)
            for t, (C1n, T4n, C4n) in new.items():
                self.C[t][(0 + r) % 4] = normalize(C1n)
                self.T[t][(3 + r) % 4] = normalize(T4n)
                self.C[t][(3 + r) % 4] = normalize(C4n)
        self.moves += 1

    def sweep(self):
        for r in SWEEP_ROTATIONS:
            self.left_move(r)

    def corner_spectra(self):
        """Normalised singular values of every corner, zero padded to chi."""
        out = []
        for i in range(self.Lx * self.Ly):
            for k in range(4):
                s = np.linalg.svd(self.C[i][k], compute_uv=False)
                s = s / s.sum()
                pad = np.zeros(self.chi)
                pad[:min(len(s), self.chi)] = s[:self.chi]
                out.append(pad)
        return np.array(out)

    def run(self, max_sweeps, tol):
        """Sweep until delta < tol or max_sweeps.  Returns (sweeps, delta, converged)."""
        prev = self.corner_spectra()
        delta = np.inf
        for n in range(1, max_sweeps + 1):
            self.sweep()
            cur = self.corner_spectra()
            delta = float(np.max(np.sum(np.abs(cur - prev), axis=1)))
            prev = cur
            if delta < tol:
                return n, delta, True
        return max_sweeps, delta, False


def normalize(X):
    m = np.max(np.abs(X))
    if not np.isfinite(m) or m == 0.0:
        raise FloatingPointError("environment tensor is zero or not finite")
    return X / m


def enlarged_corner(C, Tn, Tp, A, layers):
    """Canonical upper-left enlarged corner G[(cn, o_n), (cp, o_p)].

    C[tn, tp] is the corner, Tn[tn, cn, i_n] the edge on its next side,
    Tp[cp, tp, i_p] the edge on its prev side, A[i_p, i_n, o_n, o_p(, p)] the
    site as seen from this corner.  Ket and bra are contracted one after the
    other (single-layer contractions, the O(D^10) route of Sec. 2.2).
    """
    X1 = np.tensordot(C, Tn, axes=([0], [0]))               # [tp, cn, i_n]
    X2 = np.tensordot(Tp, X1, axes=([1], [0]))              # [cp, i_p, cn, i_n]
    cp, cn = X2.shape[0], X2.shape[2]
    if layers == 2:
        D = A.shape[0]
        X2 = X2.reshape(cp, D, D, cn, D, D)                 # [cp, l, l', cn, u, u']
        X3 = np.tensordot(X2, A, axes=([1, 4], [0, 1]))     # [cp, l', cn, u', r, d, p]
        X4 = np.tensordot(X3, A.conj(), axes=([1, 3, 6], [0, 1, 4]))  # [cp, cn, r, d, r', d']
        G = X4.transpose(1, 2, 4, 0, 3, 5)                  # [cn, r, r', cp, d, d']
        return G.reshape(cn * D * D, cp * D * D)
    X4 = np.tensordot(X2, A, axes=([1, 3], [0, 1]))         # [cp, cn, r, d]
    G = X4.transpose(1, 2, 0, 3)
    D = A.shape[0]
    return G.reshape(cn * D, cp * D)


def _fix_signs(U, V):
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        if U[j, i] < 0:
            U[:, i] *= -1.0
            V[:, i] *= -1.0
    return U, V


def _orth(Y):
    """Orthonormal basis of the range of Y (Householder QR, LAPACK)."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def projectors(G_ur, G_ul, G_ll, G_lr, chi, cutoff, mode="rsvd", oversample=32,
               power_iters=1, seed=0, sid=0, nc_beta=None, Db=None):
    """QR-free projectors of one cut (Sec. 2.2).  Returns (P, Pt).

    If the cut bond is no larger than chi (n_alpha <= chi) nothing has to be
    discarded and both projectors are the identity, so the environment stays
    an exact finite network.  Otherwise P has shape (chi, n_alpha) and Pt
    shape (n_alpha, chi); singular values at or below cutoff * sigma_0 (and
    missing ones when the cut has rank < chi) give zero rows / columns, which
    is the same as dropping them.  mode "dense" forms M and takes its full SVD;
    mode "rsvd" follows the randomized SVD with oversampling p and q power
    iterations (Halko et al. 2011, Alg. 4.4 + 5.1), applying M and M^T only
    as products with the four corners.
    """
    n_alpha = G_ul.shape[1]
    if n_alpha <= chi:
        I = np.eye(n_alpha)
        return I, I.copy()
    H_u = G_ur @ G_ul           # beta x alpha
    H_dT = G_ll @ G_lr          # alpha x beta
    if mode == "dense":
        M = H_u @ H_dT
        U, S, Vh = np.linalg.svd(M)
        V = Vh.T
    elif mode == "rsvd":
        n_beta = G_lr.shape[1]
        k = chi + oversample
        Om = omega_matrix_fast(seed, sid, nc_beta, Db, k)
        apply_M = lambda X: G_ur @ (G_ul @ (G_ll @ (G_lr @ X)))
        apply_Mt = lambda X: G_lr.T @ (G_ll.T @ (G_ul.T @ (G_ur.T @ X)))
        Q = _orth(apply_M(Om))
        for _ in range(power_iters):
            Q = _orth(apply_Mt(Q))
            Q = _orth(apply_M(Q))
        Bt = apply_Mt(Q)                     # B^T = M^T Q, shape n_beta x k'
        Vb, S, UbT = np.linalg.svd(Bt, full_matrices=False)   # B = Ub S Vb^T
        U = Q @ UbT.T
        V = Vb
        assert U.shape[0] == n_beta
    else:
        raise ValueError(mode)
    if not S.size or not S[0] > 0 or not np.all(np.isfinite(S)):
        raise FloatingPointError("the cut has no singular value above zero")
    # M = G_ur G_ul G_ll G_lr cannot have rank above its smallest bond: any
    # singular value past that bound is rounding noise and is not kept.
    r_struct = min(G_ur.shape + G_ul.shape + G_ll.shape + G_lr.shape)
    m = min(chi, S.size)
    U, V, S = U[:, :m].copy(), V[:, :m].copy(), S[:m].copy()
    keep = (S > cutoff * S[0]) & (np.arange(m) < r_struct)
    U, V = _fix_signs(U, V)
    isq = np.where(keep, 1.0 / np.sqrt(np.where(keep, S, 1.0)), 0.0)
    P = np.zeros((chi, n_alpha))
    Pt = np.zeros((n_alpha, chi))
    P[:m] = (U * isq).T @ H_u
    Pt[:, :m] = H_dT @ (V * isq)
    return P, Pt


def renorm_corner_upper(C1, T1, Pt):
    """C1'[c2, k] = sum C1[t1, t4] T1[t1, c2, u] Pt[(t4, u), k]."""
    X = np.tensordot(C1, T1, axes=([0], [0]))                      # [t4, c2, u]
    Pt3 = Pt.reshape(C1.shape[1], T1.shape[2], -1)                 # [t4, u, k]
    return np.tensordot(X, Pt3, axes=([0, 2], [0, 1]))             # [c2, k]


def renorm_corner_lower(C4, T3, P):
    """C4'[k, c3] = sum P[k, (t4, d)] C4[t4, t3] T3[c3, t3, d]."""
    X = np.tensordot(C4, T3, axes=([1], [1]))                      # [t4, c3, d]
    P3 = P.reshape(-1, C4.shape[0], T3.shape[2])                   # [k, t4, d]
    return np.tensordot(P3, X, axes=([1, 2], [0, 2]))              # [k, c3]


def renorm_edge(T4, A, P_up, Pt_dn, layers):
    """T4'[kd, ku, r] = sum Pt_dn[(c4, d), kd] T4[c4, c1, l] a[l, u, r, d] P_up[ku, (c1, u)]."""
    c4, c1, Db = T4.shape
    ku, kd = P_up.shape[0], Pt_dn.shape[1]
    if layers == 2:
        D = A.shape[0]
        T = T4.reshape(c4, c1, D, D)
        P3 = P_up.reshape(ku, c1, D, D)                            # [ku, c1, u, u']
        X = np.tensordot(T, P3, axes=([1], [1]))                   # [c4, l, l', ku, u, u']
        X = np.tensordot(X, A, axes=([1, 4], [0, 1]))              # [c4, l', ku, u', r, d, p]
        X = np.tensordot(X, A.conj(), axes=([1, 3, 6], [0, 1, 4]))  # [c4, ku, r, d, r', d']
        Pt3 = Pt_dn.reshape(c4, D, D, kd)                          # [c4, d, d', kd]
        Y = np.tensordot(X, Pt3, axes=([0, 3, 5], [0, 1, 2]))      # [ku, r, r', kd]
        return Y.transpose(3, 0, 1, 2).reshape(kd, ku, D * D)
    P3 = P_up.reshape(ku, c1, Db)
    X = np.tensordot(T4, P3, axes=([1], [1]))                      # [c4, l, ku, u]
    X = np.tensordot(X, A, axes=([1, 3], [0, 1]))                  # [c4, ku, r, d]
    Pt3 = Pt_dn.reshape(c4, Db, kd)
    Y = np.tensordot(X, Pt3, axes=([0, 3], [0, 1]))                # [ku, r, kd]
    return Y.transpose(2, 0, 1)
