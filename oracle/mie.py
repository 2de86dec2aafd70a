"""Mie T-matrix of a homogeneous sphere and its radius derivative (oracle, FP64).

Test infrastructure only.

The paper's T-matrix (App. I.B, eq. "def_tmatrix") maps regular incident
coefficients to outgoing scattered ones, s = T a.  For a sphere it is diagonal
and independent of m; with the e^{-i w t} convention (outgoing h^(1)) the
M-type (p = 0) entry is -b_l and the N-type (p = 1) entry is -a_l, where a_l,
b_l are the Lorenz-Mie coefficients written with Riccati-Bessel functions
psi_l(z) = z j_l(z), xi_l(z) = z h_l^(1)(z) (Bohren & Huffman, sec. 4.4):
  a_l = [m psi(mx) psi'(x) - psi(x) psi'(mx)] / [m psi(mx) xi'(x) - xi(x) psi'(mx)]
  b_l = [psi(mx) psi'(x) - m psi(x) psi'(mx)] / [psi(mx) xi'(x) - m xi(x) psi'(mx)]
with x = k r and m the relative refractive index.  dt/dr follows from the
chain rule with psi'' = (l(l+1)/z^2 - 1) psi (the Riccati-Bessel equation).
The scatterer model is the sphere special case of App. I.B (the paper's own
scatterers are cylinders whose T-matrix it obtains by the null-field method).
"""
import numpy as np
from scipy import special as sps

from .vswf import index_list


def _rb(l, z):
    """psi, psi', xi, xi' at complex or real z."""
    j = sps.spherical_jn(l, z)
    jd = sps.spherical_jn(l, z, derivative=True)
    y = sps.spherical_yn(l, z)
    yd = sps.spherical_yn(l, z, derivative=True)
    h = j + 1j * y
    hd = jd + 1j * yd
    return z * j, j + z * jd, z * h, h + z * hd


def mie_ab(l, x, m):
    """(a_l, b_l, da_l/dx, db_l/dx) at size parameter x, relative index m.

    Derivatives are with respect to x at fixed m (d/dr = k d/dx).
    """
    y = m * x
    px, pdx, xx, xdx = _rb(l, x)
    py, pdy, _, _ = _rb(l, y)
    ll = l * (l + 1)
    pddx = (ll / x**2 - 1.0) * px
    xddx = (ll / x**2 - 1.0) * xx
    pddy = (ll / y**2 - 1.0) * py
    na = m * py * pdx - px * pdy
    da = m * py * xdx - xx * pdy
    nb = py * pdx - m * px * pdy
    db = py * xdx - m * xx * pdy
    # derivatives w.r.t. x (dy/dx = m)
    na_x = m * m * pdy * pdx + m * py * pddx - pdx * pdy - m * px * pddy
    da_x = m * m * pdy * xdx + m * py * xddx - xdx * pdy - m * xx * pddy
    nb_x = m * pdy * pdx + py * pddx - m * pdx * pdy - m * m * px * pddy
    db_x = m * pdy * xdx + py * xddx - m * xdx * pdy - m * m * xx * pddy
    a = na / da
    b = nb / db
    dadx = (na_x * da - na * da_x) / da**2
    dbdx = (nb_x * db - nb * db_x) / db**2
    return a, b, dadx, dbdx


def mie_tmatrix_diag(lmax, k, radius, m):
    """Diagonal of T (length 2 lmax(lmax+2)) and its radius derivative."""
    x = k * radius
    t = np.zeros(2 * lmax * (lmax + 2), dtype=complex)
    dt = np.zeros_like(t)
    ab = {l: mie_ab(l, x, m) for l in range(1, lmax + 1)}
    for n, (p, l, _m) in enumerate(index_list(lmax)):
        a, b, dadx, dbdx = ab[l]
        if p == 0:
            t[n], dt[n] = -b, -k * dbdx
        else:
            t[n], dt[n] = -a, -k * dadx
    return t, dt


def mie_tmatrix_diag_many(lmax, k, radii, m):
    ts, dts = zip(*(mie_tmatrix_diag(lmax, k, r, m) for r in np.asarray(radii, dtype=float)))
    return np.array(ts), np.array(dts)
