"""Exact contraction of small finite networks.  TEST INFRASTRUCTURE ONLY.

An untruncated CTMRG environment is an exact finite network: every absorbed
column or row adds one strip of site tensors, and the initial boundary vector
closes the outer legs.  This module contracts such a rectangle directly,
with the double-layer tensor of Fig. 2(b) built from its definition
a[(l l'), (u u'), (r r'), (d d')] = sum_p A[l u r d p] conj(A[l' u' r' d' p]),
row by row from the bottom, so that CTMRG results at chi >= the bond
dimension of the patch can be checked against it.
"""
import numpy as np


def double_layer(A, open_phys=False):
    D = A.shape[0]
    if open_phys:
        a = np.einsum("lurdp,LURDq->lLuUrRdDpq", A, A.conj())
        d = A.shape[4]
        return a.reshape(D * D, D * D, D * D, D * D, d, d)
    a = np.einsum("lurdp,LURDp->lLuUrRdD", A, A.conj())
    return a.reshape(D * D, D * D, D * D, D * D)


def contract_grid(grid, boundary):
    """Contract grid[row][col] (row 0 at the bottom) of tensors t[l, u, r, d, extra...].

    Every outer leg is closed with ``boundary``.  Extra legs are returned in
    the order the tensors are visited (rows bottom to top, columns left to right).
    """
    H, W = len(grid), len(grid[0])
    w = np.asarray(boundary, dtype=np.float64)
    S = w
    for _ in range(W - 1):
        S = np.multiply.outer(S, w)
    S = S.reshape((w.size,) * W)
    nex = 0
    for row in grid:
        S = np.tensordot(w, S, axes=0)            # [h, d_0, ..., d_{W-1}, extras]
        for j, t in enumerate(row):
            # wires: u_0..u_{j-1} (j axes), h (axis j), d_j..d_{W-1}
            S = np.tensordot(S, t, axes=([j, j + 1], [0, 3]))
            # -> [u_0..u_{j-1}, d_{j+1}.., extras(nex), u_j, r, extra_t..]
            te = t.ndim - 4
            nw = W + 1 - 2                          # wires left before the new u, r
            src = [nw + nex, nw + nex + 1]
            S = np.moveaxis(S, src, [j, j + 1])
            nex += te
        S = np.tensordot(S, w, axes=([W], [0]))     # close the right end
        # now [u_0..u_{W-1}, extras]: these become the d legs of the next row
    for _ in range(W):
        S = np.tensordot(w, S, axes=([0], [0]))
    return S


def patch_value(tensors, Lx, Ly, layers, boundary, x0, x1, y0, y1, open_sites=(),
                replace=None):
    """Contract sites x0..x1, y0..y1 (inclusive) of the periodic unit cell.

    open_sites: positions (x, y) whose physical indices stay open (ket, bra).
    replace:    {(x, y): single-layer tensor} substituted at those positions.
    """
    grid = []
    for y in range(y0, y1 + 1):
        row = []
        for x in range(x0, x1 + 1):
            A = np.asarray(tensors[(x % Lx) + Lx * (y % Ly)], dtype=np.float64)
            if replace is not None and (x, y) in replace:
                row.append(np.asarray(replace[(x, y)], dtype=np.float64))
            elif layers == 2:
                row.append(double_layer(A, open_phys=(x, y) in open_sites))
            else:
                row.append(A)
        grid.append(row)
    return contract_grid(grid, boundary)


def strip_transfer(A, layers, boundary, H):
    """Column transfer matrix of a strip H sites high, closed at the top and
    the bottom by ``boundary``: M[(l_1..l_H), (r_1..r_H)] with site 1 at the
    top, each leg of the double-layer (or classical) tensor.  Used to check
    the transfer-matrix spectrum of an untruncated environment."""
    t = double_layer(A) if layers == 2 else np.asarray(A, dtype=np.float64)
    w = np.asarray(boundary, dtype=np.float64)
    # top site: close its up leg -> S[l1, r1, d1]
    S = np.tensordot(t, w, axes=([1], [0]))            # [l, r, d]
    for _ in range(H - 1):
        # next site below: contract the open down leg with its up leg
        S = np.tensordot(S, t, axes=([-1], [1]))       # [..., l_k, r_k, d_k]
    S = np.tensordot(S, w, axes=([-1], [0]))           # close the bottom
    # axes now (l_1, r_1, l_2, r_2, ..., l_H, r_H)
    b = t.shape[0]
    S = S.reshape((b, b) * H)
    S = S.transpose(list(range(0, 2 * H, 2)) + list(range(1, 2 * H, 2)))
    return S.reshape(b ** H, b ** H)
