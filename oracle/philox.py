"""Philox4x64-10 and the randomized-SVD test matrix.  TEST INFRASTRUCTURE ONLY.

The paper (Sec. 2.2) computes the projector SVD with a partial SVD such as
the randomized SVD of Halko, Martinsson and Tropp.  That method needs a random
test matrix Omega.  To let an independent implementation reproduce Omega bit
for bit, Omega is drawn from the counter-based generator Philox4x64-10
(Salmon, Moraes, Dror, Shaw, SC'11), written here from its published
definition: ten rounds of two 64x64->128-bit multiplies with the multipliers
below, a Weyl sequence on the key, and the fixed word permutation.

Pinned against ``numpy.random.Philox`` (an independent implementation of the
same generator) in tests/test_oracle_philox.py.

Omega entries are uniform on [-1, 1) with 53 random bits, so every entry is
an exactly representable double; see ``omega_entry``.
"""
import numpy as np

_MASK = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1


def _mulhilo(a, b):
    p = a * b
    return (p >> 64) & _MASK, p & _MASK


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: 4 counter words, 2 key words -> 4 words."""
    x0, x1, x2, x3 = (int(c) & _MASK for c in ctr)
    k0, k1 = (int(k) & _MASK for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & _MASK
            k1 = (k1 + PHILOX_W1) & _MASK
        hi0, lo0 = _mulhilo(PHILOX_M0, x0)
        hi1, lo1 = _mulhilo(PHILOX_M1, x2)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def stream_id(move, x, y):
    """Key of one cut's sketch: move counter since init, view column, cut row."""
    return ((int(move) & 0xFFFFFFFF) << 32) | ((int(x) & 0xFFFF) << 16) | (int(y) & 0xFFFF)


def omega_entry(seed, sid, c, b, j):
    """Omega[(c, b), j] for chi-bond index c, pair index b, sketch column j.

    Counter = (c, b, j // 4, sid), key = (seed, 0); word j % 4 of the block,
    mapped to (w >> 11) * 2**-52 - 1, uniform on [-1, 1).
    """
    w = philox4x64_10((c, b, j // 4, sid), (seed, 0))[j % 4]
    return float(w >> 11) * 2.0 ** -52 - 1.0


def omega_matrix(seed, sid, nc, nb, k):
    """Sketch matrix with rows ordered (c, b), c < nc, b < nb; shape (nc*nb, k)."""
    out = np.empty((nc * nb, k))
    for c in range(nc):
        for b in range(nb):
            for j in range(k):
                out[c * nb + b, j] = omega_entry(seed, sid, c, b, j)
    return out


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo_vec(a, b):
    """Elementwise 64x64->128 product of uint64 arrays via 32-bit limbs."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    lo = (p00 & _M32) | ((mid & _M32) << _S32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10_vec(x0, x1, x2, x3, k0, k1):
    """Vectorised Philox4x64-10 over uint64 arrays (same rounds as above)."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in (x0, x1, x2, x3))
    k0 = np.uint64(int(k0) & _MASK)
    k1 = np.uint64(int(k1) & _MASK)
    m0, m1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
    w0, w1 = np.uint64(PHILOX_W0), np.uint64(PHILOX_W1)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = k0 + w0
                k1 = k1 + w1
            hi0, lo0 = _mulhilo_vec(m0, x0)
            hi1, lo1 = _mulhilo_vec(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def omega_matrix_fast(seed, sid, nc, nb, k):
    """Same values as ``omega_matrix``, computed with whole-array Philox."""
    c, b, j = np.meshgrid(np.arange(nc, dtype=np.uint64), np.arange(nb, dtype=np.uint64),
                          np.arange(k, dtype=np.uint64), indexing="ij")
    words = philox4x64_10_vec(c, b, j >> np.uint64(2), np.full(c.shape, sid, dtype=np.uint64),
                              seed, 0)
    sel = (j & np.uint64(3)).astype(np.int64)
    w = np.choose(sel, words)
    return ((w >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0).reshape(nc * nb, k)
