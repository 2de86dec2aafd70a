"""Special functions for the CPU FP64 oracle (test infrastructure only).

Everything here is a plain definition evaluated in double precision:

* spherical Bessel j_l, y_l and Hankel h_l^(1) = j_l + i y_l (SciPy);
* the normalised associated Legendre function used by the scalar spherical
  wavefunctions of App. I.A ("Vector spherical wavefunctions"):
  Pbar_l^m(x) = sqrt((2l+1)/2 * (l-m)!/(l+m)!) * (1-x^2)^(m/2) * d^m P_l/dx^m,
  0 <= m <= l, without the Condon-Shortley phase (reading: the paper only says
  "normalized"; this choice is orthonormal on [-1, 1]);
* the angular functions pi = m * Pbar_l^|m| / sin(theta) and
  tau = d Pbar_l^|m| / d theta that appear in the plane-wave expansion of
  App. II ("Implementing jinc source in the vector spherical harmonic basis"),
  evaluated from Legendre-polynomial derivatives so that theta = 0 and pi are
  regular points;
* Wigner 3j symbols (exact rationals from SymPy), used by the translation
  coefficients of App. I.C.
"""
from functools import lru_cache
from math import factorial, sqrt

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy import special as sps


def sph_jn(l, x):
    return sps.spherical_jn(l, x)


def sph_yn(l, x):
    return sps.spherical_yn(l, x)


def sph_h1(l, x):
    """Spherical Hankel function of the first kind, h_l^(1) = j_l + i y_l."""
    return sps.spherical_jn(l, x) + 1j * sps.spherical_yn(l, x)


def _legendre_derivative(l, order, x):
    """order-th derivative of the Legendre polynomial P_l at x."""
    if order > l:
        return np.zeros_like(np.asarray(x, dtype=float))
    c = np.zeros(l + 1)
    c[l] = 1.0
    if order > 0:
        c = npleg.legder(c, order)
    return npleg.legval(x, c)


def _norm(l, m):
    return sqrt((2 * l + 1) / 2.0 * factorial(l - m) / factorial(l + m))


def pbar(l, m, x):
    """Normalised associated Legendre function Pbar_l^|m|(x) (no CS phase)."""
    m = abs(m)
    x = np.asarray(x, dtype=float)
    if m > l:
        return np.zeros_like(x)
    s2 = np.clip(1.0 - x * x, 0.0, None)
    return _norm(l, m) * s2 ** (0.5 * m) * _legendre_derivative(l, m, x)


def pi_fn(l, m, theta):
    """m * Pbar_l^|m|(cos theta) / sin(theta), with signed m (0 for m = 0)."""
    theta = np.asarray(theta, dtype=float)
    if m == 0:
        return np.zeros_like(theta)
    am = abs(m)
    if am > l:
        return np.zeros_like(theta)
    x = np.cos(theta)
    s2 = np.clip(1.0 - x * x, 0.0, None)
    return m * _norm(l, am) * s2 ** (0.5 * (am - 1)) * _legendre_derivative(l, am, x)


def tau_fn(l, m, theta):
    """d/dtheta of Pbar_l^|m|(cos theta)."""
    theta = np.asarray(theta, dtype=float)
    am = abs(m)
    if am > l:
        return np.zeros_like(theta)
    x = np.cos(theta)
    s2 = np.clip(1.0 - x * x, 0.0, None)
    if am == 0:
        return -_norm(l, 0) * np.sqrt(s2) * _legendre_derivative(l, 1, x)
    t1 = am * x * s2 ** (0.5 * (am - 1)) * _legendre_derivative(l, am, x)
    t2 = s2 ** (0.5 * (am + 1)) * _legendre_derivative(l, am + 1, x)
    return _norm(l, am) * (t1 - t2)


@lru_cache(maxsize=None)
def wigner3j(j1, j2, j3, m1, m2, m3):
    """Wigner 3j symbol as a float (exact rational evaluation by SymPy)."""
    from sympy.physics.wigner import wigner_3j

    return float(wigner_3j(j1, j2, j3, m1, m2, m3))
