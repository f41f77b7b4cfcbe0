"""Closed forms of the square-lattice Ising model (J = 1, k_B = 1).  TEST INFRASTRUCTURE ONLY.

These pin the classical CTMRG (a 2D classical network is the single-layer
case of the contraction of Sec. 2.2, Fig. 2(b)) and the Ising-PEPS double
layer, whose norm equals the Ising partition function.

* Free energy per site (Onsager 1944), two independent forms:
    -beta f = ln(2 cosh 2b) + 1/(2 pi) int_0^pi ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt
    -beta f = ln 2 + 1/(2 pi^2) int int ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)]
  with k = 2 sinh 2b / cosh^2 2b.
* Spontaneous magnetisation (Yang 1952): m = (1 - sinh(2b)^-4)^(1/8), T < Tc.
* Internal energy per site: u = -coth 2b [1 + (2/pi)(2 tanh^2 2b - 1) K(k)],
  K the complete elliptic integral of the first kind; the nearest-neighbour
  correlator is <s s> = -u / 2.
* Tc = 2 / ln(1 + sqrt 2); at Tc, -beta f = ln(2)/2 + 2G/pi (G = Catalan).
"""
import numpy as np
from scipy import integrate, special

CATALAN = 0.915965594177219015054603514932384110774


def onsager_lnz(beta):
    b2 = 2.0 * beta
    k = 2.0 * np.sinh(b2) / np.cosh(b2) ** 2
    f = lambda t: np.log(0.5 * (1.0 + np.sqrt(max(0.0, 1.0 - k * k * np.sin(t) ** 2))))
    val, _ = integrate.quad(f, 0.0, np.pi, epsabs=1e-15, epsrel=1e-15, limit=400)
    return np.log(2.0 * np.cosh(b2)) + val / (2.0 * np.pi)


def onsager_lnz_double(beta):
    b2 = 2.0 * beta
    ch, sh = np.cosh(b2) ** 2, np.sinh(b2)
    f = lambda t2, t1: np.log(ch - sh * (np.cos(t1) + np.cos(t2)))
    val, _ = integrate.dblquad(f, 0.0, np.pi, 0.0, np.pi, epsabs=1e-13, epsrel=1e-13)
    # the integrand is even in both angles: int_0^{2pi} int_0^{2pi} = 4 int_0^pi int_0^pi
    return np.log(2.0) + 4.0 * val / (8.0 * np.pi ** 2)


def yang_magnetization(beta):
    s = np.sinh(2.0 * beta)
    x = 1.0 - s ** -4
    return x ** 0.125 if x > 0 else 0.0


def internal_energy(beta):
    b2 = 2.0 * beta
    k = 2.0 * np.sinh(b2) / np.cosh(b2) ** 2
    K = special.ellipk(k * k)          # scipy's ellipk takes m = k^2
    return -1.0 / np.tanh(b2) * (1.0 + (2.0 / np.pi) * (2.0 * np.tanh(b2) ** 2 - 1.0) * K)


def nn_correlator(beta):
    return -0.5 * internal_energy(beta)


def critical_temperature():
    return 2.0 / np.log(1.0 + np.sqrt(2.0))
