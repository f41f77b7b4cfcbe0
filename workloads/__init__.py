"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no CTMRG arithmetic: it only builds site tensors, boundary
vectors, operators and request streams from a seed.  Both the oracle and the
GPU library receive the same arrays from here.

Workloads (sizes as in the benchmark configurations):
* ``ising_classical(beta)``: vertex form of the 2D Ising model, one spin per
  tensor, a[l, u, r, d] = sum_s W[s,l] W[s,u] W[s,r] W[s,d] with
  W W^T = exp(beta s s'); impurity b (spin-weighted) and the polarised
  boundary vector w+ = W[+, :].
* ``ising_peps(beta)``: D = d = 2 iTPS whose norm is the Ising partition
  function (Verstraete et al., PRL 96, 220601): A[l,u,r,d,p] = prod W'[p, leg]
  with W' W'^T = exp((beta/2) s s').
* ``random_itps(Lx, Ly, D, d, seed)``: N(0, 1) entries (PCG64, sites drawn in
  order, C order), each tensor divided by its max-abs entry.
* ``random_environment(Lx, Ly, chi, Db, seed)``: N(0, 1) corners and edges
  with every leg of full size (generic spectra at every cut).
* ``heisenberg_bond()``: S=1/2 Heisenberg bond operator of the paper's worked
  example (Sec. 5.2), op[(out_i, out_j), (in_i, in_j)].
* ``tfim_bond(h)`` / ``tfim_product_state(h)``: transverse-field Ising in
  Pauli units, H = -sum sz sz - h sum sx, with the field split over the four
  bonds of each site.
* ``serving_stream(...)``: the mixed request stream of the serving benchmark.
"""
import math

import numpy as np

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
SY_IM = np.array([[0.0, -1.0], [1.0, 0.0]])  # sigma_y / i (real)
ID2 = np.eye(2)


def ising_weights(beta):
    c, s = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
    return np.array([[c, s], [c, -s]])          # row: spin (+, -), column: bond index


def ising_classical(beta):
    """(a, b, w_plus) for the vertex-form Ising network at inverse temperature beta."""
    W = ising_weights(beta)
    spin = np.array([1.0, -1.0])
    a = np.einsum("sl,su,sr,sd->lurd", W, W, W, W)
    b = np.einsum("s,sl,su,sr,sd->lurd", spin, W, W, W, W)
    return a, b, W[0].copy()


def ising_peps(beta):
    """(A, w_plus_pair) for the D = d = 2 Ising PEPS; boundary on the (ket, bra) pair."""
    W = ising_weights(0.5 * beta)
    A = np.einsum("pl,pu,pr,pd->lurdp", W, W, W, W)
    wp = W[0]
    return A, np.outer(wp, wp).reshape(-1)


def random_gauges(D, seed):
    """Well-conditioned random invertible matrices for bond gauge tests."""
    rng = np.random.default_rng(seed)
    while True:
        G = np.eye(D) + 0.3 * rng.standard_normal((D, D))
        if np.linalg.cond(G) < 10:
            return G


def gauged_2x2(A, D, seed):
    """A 2x2 cell of copies of A with a random invertible G G^-1 inserted on
    every bond (the state, and every expectation value, is unchanged; the four
    site tensors differ)."""
    Gh = [random_gauges(D, seed + k) for k in range(4)]       # horizontal bonds
    Gv = [random_gauges(D, seed + 10 + k) for k in range(4)]  # vertical bonds
    out = []
    for y in range(2):
        for x in range(2):
            h_right = Gh[x + 2 * y]
            h_left = Gh[((x - 1) % 2) + 2 * y]
            v_up = Gv[x + 2 * y]
            v_down = Gv[x + 2 * ((y - 1) % 2)]
            B = np.einsum("lurdp,Rr->luRdp", A, h_right)
            B = np.einsum("lurdp,lL->Lurdp", B, np.linalg.inv(h_left))
            B = np.einsum("lurdp,Uu->lUrdp", B, v_up)
            B = np.einsum("lurdp,dD->lurDp", B, np.linalg.inv(v_down))
            out.append(B)
    return out


def random_itps(Lx, Ly, D, d, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(Lx * Ly):
        A = rng.standard_normal((D, D, D, D, d))
        out.append(A / np.max(np.abs(A)))
    return out


def random_environment(Lx, Ly, chi, Db, seed):
    """Random corners and edges, every chi leg of full size: one ([C1..C4],
    [T1..T4]) pair per site, N(0, 1) entries (PCG64, sites in order, C
    matrices then T tensors, C order), C_k of shape (chi, chi) and T_k of
    shape (chi, chi, Db)."""
    rng = np.random.default_rng(seed)
    env = []
    for _ in range(Lx * Ly):
        C = [rng.standard_normal((chi, chi)) for _ in range(4)]
        T = [rng.standard_normal((chi, chi, Db)) for _ in range(4)]
        env.append((C, T))
    return env


def random_classical(Lx, Ly, D, seed, positive=True):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(Lx * Ly):
        a = rng.random((D,) * 4) + (0.5 if positive else -0.5)
        out.append(a / np.max(np.abs(a)))
    return out


def heisenberg_bond():
    """S_i.S_j for S = 1/2 from the element list of the paper's example (Sec. 5.2).

    Each line there is (in_i, in_j, out_i, out_j, Re, Im); states up = 0, down = 1.
    """
    lines = [(0, 0, 0, 0, 0.25), (1, 0, 1, 0, -0.25), (0, 1, 1, 0, 0.5),
             (1, 0, 0, 1, 0.5), (0, 1, 0, 1, -0.25), (1, 1, 1, 1, 0.25)]
    op = np.zeros((4, 4))
    for a, b, c, e, v in lines:
        op[c * 2 + e, a * 2 + b] = v
    return op


def tfim_bond(h):
    """-sz sz - (h/4)(sx 1 + 1 sx): field split over the 4 bonds of a site."""
    return -np.kron(SZ, SZ) - 0.25 * h * (np.kron(SX, ID2) + np.kron(ID2, SX))


def tfim_mean_field(h):
    """Mean-field product state of the Pauli TFIM: sin(theta) = min(h/4, 1)."""
    s = min(h / 4.0, 1.0)
    th = math.asin(s)
    # spin along (sin th) x + (cos th) z
    phi = np.array([math.cos(th / 2.0), math.sin(th / 2.0)])
    energy = -2.0 * math.cos(th) ** 2 - h * math.sin(th)
    return phi, energy


def product_itps(phis, D=1):
    """Product state: A[0,0,0,0,:] = phi, all other entries zero (bond dim D)."""
    out = []
    for phi in phis:
        A = np.zeros((D, D, D, D, len(phi)))
        A[0, 0, 0, 0, :] = phi
        out.append(A)
    return out


def tfim_request_tensors(h, D, Lx, Ly, eps, seed):
    """Mean-field state in A[0,0,0,0,:] plus eps * N(0,1) elsewhere, / max-abs."""
    rng = np.random.default_rng(seed)
    phi, _ = tfim_mean_field(h)
    out = []
    for _ in range(Lx * Ly):
        A = eps * rng.standard_normal((D, D, D, D, 2))
        A[0, 0, 0, 0, :] = phi
        out.append(A / np.max(np.abs(A)))
    return out


def serving_stream(n=512, seed=4, rate_hz=None, eps=0.1):
    """The mixed TFIM request stream: h ~ U[2.5, 3.5], D ~ U{2..5}, chi ~ U{16..100},
    cell ~ U{1x1, 2x2}, Poisson arrivals at rate_hz (None: all at t = 0).  The
    arrival times come from a generator of their own, so the requests are the
    same at every rate."""
    rng = np.random.default_rng(seed)
    arrivals = np.random.default_rng(seed + 7919)
    reqs = []
    t = 0.0
    for i in range(n):
        h = float(rng.uniform(2.5, 3.5))
        D = int(rng.integers(2, 6))
        chi = int(rng.integers(16, 101))
        L = 1 if rng.random() < 0.5 else 2
        if rate_hz:
            t += float(arrivals.exponential(1.0 / rate_hz))
        reqs.append(dict(index=i, h=h, D=D, chi=chi, Lx=L, Ly=L, arrival=t,
                         tensor_seed=seed * 100003 + i))
    return reqs
