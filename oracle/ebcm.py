"""Null-field (EBCM) T-matrix of an axisymmetric scatterer (oracle, FP64).

Test infrastructure only.

App. I.B ("Transition matrix") computes T from the matrices
  P_{lmp; l'm'p'} = int [ R Phi_{l'm'p'}(k_s x) x Phi_{l,-m,1-p}(k_b x)
                          - (k_s/k_b) R Phi_{l'm',1-p'}(k_s x) x Phi_{l,-m,p}(k_b x) ] . n dS
and Q the same with the regular R Phi_{l,-m,.}(k_b x) in place of the
outgoing Phi_{l,-m,.}(k_b x).  Readings (fixed by the sphere pin: EBCM on a
sphere must give the Lorenz-Mie T of oracle.mie):
  * the two cross products add: with this basis's curl relations
    Phi_lm1 = (1/k) curl Phi_lm0, Phi_lm0 = (1/k) curl Phi_lm1, the surface
    term of the vector Green identity is n.[E x curl G + (curl E) x G], so the
    integrand is R Phi_{l'm'p'}(k_s) x Phi_{l,-m,1-p}(k_b)
    + (k_s/k_b) R Phi_{l'm',1-p'}(k_s) x Phi_{l,-m,p}(k_b) (the print's minus
    belongs to another sign convention of the basis);
  * T = -Q P^{-1} in the print's names, i.e. minus the regular-test matrix
    times the inverse of the outgoing-test matrix (the null-field method's
    T = -RgQ Q^{-1}; the print's T = -P Q^{-1} swaps the two);
  * the surface is the scatterer's own surface (the null-field method's
    boundary; the display names the enclosing sphere's symbol);
  * k_s = n_rel k_b (a complex n_rel is allowed, Im > 0 lossy);
  * for a body of revolution about z the azimuthal integral is
    2 pi delta_{m m'} (the test wave carries e^{-imphi}, the internal one
    e^{im'phi}, and the normal has no phi component), so T is block-diagonal
    in m and each block is formed and inverted on its own.
The basis is that of oracle.vswf (App. I.A), written out here for complex
wavenumbers.  Pinned in the tests by the sphere (EBCM on a sphere = Mie), and,
for cylinders, by reciprocity of the far-field amplitude and the optical
theorem of a lossless body, through the oracle's own solve and readout.
"""
import numpy as np
from scipy import special as sps

from .special import pbar, pi_fn, tau_fn
from .vswf import index_list, n_coeffs


def _zl(l, x, regular):
    """j_l (regular) or h_l^(1) at complex x, and (x z_l)'/x."""
    x = np.asarray(x, dtype=complex)
    if regular:
        z = sps.spherical_jn(l, x)
        zm = sps.spherical_jn(l - 1, x)
    else:
        z = sps.spherical_jn(l, x) + 1j * sps.spherical_yn(l, x)
        zm = sps.spherical_jn(l - 1, x) + 1j * sps.spherical_yn(l - 1, x)
    return z, zm - l * z / x


def vswf_components(l, m, p, k, r, theta, regular):
    """(r, theta, phi) components of Phi_lmp(k x) at (r, theta) without the
    e^{i m phi} factor, for a complex wavenumber k -> [..., 3]."""
    x = k * np.asarray(r, dtype=float)
    z, dz = _zl(l, x, regular)
    P = pbar(l, m, np.cos(theta))
    pi = pi_fn(l, m, theta)
    tau = tau_fn(l, m, theta)
    nrm = 1.0 / np.sqrt(2.0 * l * (l + 1))
    if p == 0:
        return nrm * np.stack([np.zeros_like(z), 1j * pi * z, -tau * z], -1)
    return nrm * np.stack([l * (l + 1) * z / x * P, tau * dz, 1j * pi * dz], -1)


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)


def cylinder_surface(radius, height, n_quad):
    """Gauss-Legendre nodes on the generating curve of a cylinder centred at
    the origin (axis z): bottom cap, side, top cap.  Returns r, theta, the
    normal in (r, theta) components [.., 2] and the weight rho dl."""
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    u = 0.5 * (xg + 1.0)
    segs = []
    # bottom cap z = -h/2, rho from 0 to a, normal -z
    rho, z = radius * u, np.full(n_quad, -0.5 * height)
    segs.append((rho, z, np.array([0.0, -1.0]), 0.5 * radius * wg))
    # side rho = a, z from -h/2 to h/2, normal rho_hat
    rho, z = np.full(n_quad, radius), height * (u - 0.5)
    segs.append((rho, z, np.array([1.0, 0.0]), 0.5 * height * wg))
    # top cap z = h/2, normal +z
    rho, z = radius * u, np.full(n_quad, 0.5 * height)
    segs.append((rho, z, np.array([0.0, 1.0]), 0.5 * radius * wg))
    R, TH, N, W = [], [], [], []
    for rho, z, nc, w in segs:
        r = np.hypot(rho, z)
        th = np.arctan2(rho, z)
        # (rho_hat, z_hat) -> (r_hat, theta_hat): rho_hat = (sin, cos), z_hat = (cos, -sin)
        nr = nc[0] * np.sin(th) + nc[1] * np.cos(th)
        nt = nc[0] * np.cos(th) - nc[1] * np.sin(th)
        R.append(r)
        TH.append(th)
        N.append(np.stack([nr, nt], -1))
        W.append(w * rho)
    return np.concatenate(R), np.concatenate(TH), np.concatenate(N), np.concatenate(W)


def spheroid_surface(a, c, n_quad):
    """A spheroid with semi-axes (a, a, c) about z: Gauss-Legendre nodes in
    the parameter t of (rho, z) = (a sin t, c cos t); outward normal along
    (rho/a^2, z/c^2); weight rho |d(rho, z)/dt|."""
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    t = np.arccos(xg)  # nodes in t over (0, pi) with weight sin t dt folded below
    rho, z = a * np.sin(t), c * np.cos(t)
    dl = np.hypot(a * np.cos(t), c * np.sin(t))  # |d(rho, z)/dt|
    nx, nz = rho / a ** 2, z / c ** 2
    nn = np.hypot(nx, nz)
    nx, nz = nx / nn, nz / nn
    r = np.hypot(rho, z)
    th = np.arctan2(rho, z)
    nr = nx * np.sin(th) + nz * np.cos(th)
    nt = nx * np.cos(th) - nz * np.sin(th)
    # dt = dx / sin t for x = cos t
    return r, th, np.stack([nr, nt], -1), wg / np.sin(t) * dl * rho


def sphere_surface(radius, n_quad):
    """Gauss-Legendre nodes in theta on a sphere (normal r_hat, weight a^2 sin)."""
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    th = np.arccos(xg)
    return (np.full(n_quad, radius), th, np.stack([np.ones(n_quad), np.zeros(n_quad)], -1),
            radius * radius * wg)


def ebcm_tmatrix(lmax, k, n_rel, surface):
    """T [L, L] in the coefficient order of oracle.vswf for a body of
    revolution given by surface = (r, theta, normal (r, theta), weight)."""
    r, th, nrm, w = surface
    ks = complex(n_rel) * k
    idx = index_list(lmax)
    L = n_coeffs(lmax)
    T = np.zeros((L, L), dtype=complex)
    ncomp = np.stack([nrm[:, 0], nrm[:, 1], np.zeros(len(r))], -1)
    for m in range(-lmax, lmax + 1):
        rows = [n for n, (p, l, mm) in enumerate(idx) if mm == m]
        Pm = np.zeros((len(rows), len(rows)), dtype=complex)
        Qm = np.zeros_like(Pm)
        for a, n in enumerate(rows):
            p, l, _ = idx[n]
            out1 = vswf_components(l, -m, 1 - p, k, r, th, regular=False)
            out0 = vswf_components(l, -m, p, k, r, th, regular=False)
            reg1 = vswf_components(l, -m, 1 - p, k, r, th, regular=True)
            reg0 = vswf_components(l, -m, p, k, r, th, regular=True)
            for b, n2 in enumerate(rows):
                pp, lp, _ = idx[n2]
                in_p = vswf_components(lp, m, pp, ks, r, th, regular=True)
                in_q = vswf_components(lp, m, 1 - pp, ks, r, th, regular=True)
                fP = _cross(in_p, out1) + (ks / k) * _cross(in_q, out0)
                fQ = _cross(in_p, reg1) + (ks / k) * _cross(in_q, reg0)
                Pm[a, b] = 2.0 * np.pi * np.sum(w * np.sum(fP * ncomp, -1))
                Qm[a, b] = 2.0 * np.pi * np.sum(w * np.sum(fQ * ncomp, -1))
        Tm = -Qm @ np.linalg.inv(Pm)
        T[np.ix_(rows, rows)] = Tm
    return T
