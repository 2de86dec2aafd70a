"""Jinc sources and their spherical-wave expansion (oracle, FP64).

Test infrastructure only.

App. II ("Computation of Jinc Sources") represents an incident field that
propagates along +z and is band-limited to the light cone by its samples on a
lambda/2 grid in a transverse plane; each sample becomes an independent
"jinc source".  A jinc source centred at (x0, y0) in the plane z = z0 with
transverse polarisation A^T is defined here through its k-space form (the
second display of the section), a uniform disk of propagating plane waves:
  E(x) = (1/2pi) int_0^{pi/2} int_0^{2pi} A(beta, alpha)
            exp[i k(beta, alpha).(x - x0)] sin(beta) cos(beta) dalpha dbeta,
  k(beta, alpha) = k0 (sin b cos a, sin b sin a, cos b),
  A(beta, alpha) = A^T - z_hat tan(beta) (A_x cos a + A_y sin a),
so that A . k = 0 for every component.  Readings (checked numerically in the
tests):
  * the measure sin(beta) cos(beta) dalpha dbeta is d^2 k^T / k0^2, so at
    z = z0 the transverse field is A^T J_1(k0 rho)/(k0 rho) with the
    cylindrical Bessel function J_1 (the k-space form's inverse transform of
    a disk), not the spherical j_1 printed in the spatial form;
  * the Nyquist interpolation of a disk-band-limited field from samples on the
    lambda/2 grid weights each jinc by (pi/2) times its sample (the cell area
    (lambda/2)^2 times k0^2 / (2 pi));
  * the plane wave about a scatterer centre x' carries exp[i k.(x' - x0)],
    the field phase at x' (the same sign reading as for plane waves);
  * the Bessel identity used for Gamma_m reads
    J_m(rho) = (1/2pi) int exp[i(rho sin t - m t)] dt (the print omits an i).
The coefficients about x' are a_lmp = (1/2pi) int int a_lmp(beta, alpha)
exp[i k.(x' - x0)] sin b cos b da db, with a_lmp(beta, alpha) the plane-wave
coefficients of App. II (oracle.vswf.plane_wave_angular).  The alpha integral
is done in closed form with
  Gamma_m(xi, eta, rho) = (1/2pi) int exp(-i m a) exp[i rho cos(a - xi)] cos(a - eta) da
                        = (i^{m-1} e^{-i m xi}/2) [e^{i(xi-eta)} J_{m-1}(rho)
                                                  - e^{-i(xi-eta)} J_{m+1}(rho)],
and the beta integral by Gauss-Legendre quadrature.
"""
import numpy as np
from scipy import special as sps

from .special import pi_fn, tau_fn
from .vswf import index_list, n_coeffs, plane_wave_angular


def jinc(x):
    """J_1(x)/x with its limit 1/2 at x = 0."""
    x = np.asarray(x, dtype=float)
    out = np.full(x.shape, 0.5)
    nz = np.abs(x) > 1e-8
    out[nz] = sps.j1(x[nz]) / x[nz]
    return out


def transverse_field_at_source_plane(src, k, pts):
    """A^T J_1(k rho)/(k rho) at points of the plane z = z0 -> [P, 3]."""
    x0, y0, z0, ax, ay = src
    pts = np.asarray(pts, dtype=float)
    rho = np.hypot(pts[:, 0] - x0, pts[:, 1] - y0)
    j = jinc(k * rho)
    return np.stack([ax * j, ay * j, np.zeros_like(j, dtype=complex)], -1)


def _beta_nodes(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.25 * np.pi * (x + 1.0), 0.25 * np.pi * w


def jinc_field(src, k, pts, n_beta=256, n_alpha=256):
    """E(x) of one jinc source by direct quadrature of its k-space form
    (Gauss-Legendre in beta, trapezoid in alpha) -> [P, 3]."""
    x0, y0, z0, ax, ay = src
    pts = np.asarray(pts, dtype=float)
    d = pts - np.array([x0, y0, z0])
    b, wb = _beta_nodes(n_beta)
    a = np.arange(n_alpha) * 2.0 * np.pi / n_alpha
    B, Al = np.meshgrid(b, a, indexing='ij')
    W = (wb[:, None] * np.full(n_alpha, 2.0 * np.pi / n_alpha)[None, :]) * np.sin(B) * np.cos(B) / (2 * np.pi)
    kv = k * np.stack([np.sin(B) * np.cos(Al), np.sin(B) * np.sin(Al), np.cos(B)], -1)
    tr = ax * np.cos(Al) + ay * np.sin(Al)
    A = np.stack([np.full(B.shape, ax, dtype=complex), np.full(B.shape, ay, dtype=complex),
                  -np.tan(B) * tr], -1)
    ph = np.exp(1j * np.einsum('bac,pc->pba', kv, d))
    return np.einsum('ba,pba,bac->pc', W, ph, A)


def gamma_closed(m, xi, eta, rho):
    """Gamma_m(xi, eta, rho) in closed form (Bessel J_{m-1}, J_{m+1})."""
    return (1j ** (m - 1)) * np.exp(-1j * m * xi) / 2.0 * (
        np.exp(1j * (xi - eta)) * sps.jv(m - 1, rho) - np.exp(-1j * (xi - eta)) * sps.jv(m + 1, rho))


def gamma_quadrature(m, xi, eta, rho, n=512):
    """Gamma_m by the trapezoid rule on its defining integral (periodic, so
    spectrally accurate)."""
    a = np.arange(n) * 2.0 * np.pi / n
    return np.mean(np.exp(-1j * m * a) * np.exp(1j * rho * np.cos(a - xi)) * np.cos(a - eta))


def jinc_coeffs_quadrature(lmax, k, src, positions, n_beta=128, n_alpha=128):
    """a[i, n] about every x_i by direct 2-D quadrature of the plane-wave
    coefficients over the disk (alpha by the trapezoid rule)."""
    x0, y0, z0, ax, ay = src
    pos = np.asarray(positions, dtype=float)
    d = pos - np.array([x0, y0, z0])
    b, wb = _beta_nodes(n_beta)
    a = np.arange(n_alpha) * 2.0 * np.pi / n_alpha
    out = np.zeros((len(pos), n_coeffs(lmax)), dtype=complex)
    for ib in range(n_beta):
        sb, cb = np.sin(b[ib]), np.cos(b[ib])
        for al in a:
            khat = np.array([sb * np.cos(al), sb * np.sin(al), cb])
            A = np.array([ax, ay, -np.tan(b[ib]) * (ax * np.cos(al) + ay * np.sin(al))])
            c = plane_wave_angular(lmax, khat, A)
            w = wb[ib] * (2.0 * np.pi / n_alpha) * sb * cb / (2.0 * np.pi)
            out += w * np.exp(1j * k * d @ khat)[:, None] * c[None, :]
    return out


def jinc_coeffs(lmax, k, src, positions, n_beta=128):
    """a[i, n] about every x_i with the alpha integral in closed form (Gamma_m)
    and Gauss-Legendre in beta: the paper's route."""
    x0, y0, z0, ax, ay = src
    pos = np.asarray(positions, dtype=float)
    d = pos - np.array([x0, y0, z0])
    rho_t = np.hypot(d[:, 0], d[:, 1])  # r0 sin(theta0)
    phi0 = np.arctan2(d[:, 1], d[:, 0])
    zc = d[:, 2]  # r0 cos(theta0)
    b, wb = _beta_nodes(n_beta)
    out = np.zeros((len(pos), n_coeffs(lmax)), dtype=complex)
    for n, (p, l, m) in enumerate(index_list(lmax)):
        acc = np.zeros(len(pos), dtype=complex)
        for ib in range(n_beta):
            sb, cb = np.sin(b[ib]), np.cos(b[ib])
            pi = float(pi_fn(l, m, b[ib]))   # m Pbar / sin(beta)
            tau = float(tau_fn(l, m, b[ib]))
            rho = k * rho_t * sb
            g0 = gamma_closed(m, phi0, 0.0, rho)
            g1 = gamma_closed(m, phi0, 0.5 * np.pi, rho)
            pref = -4.0 * np.exp(1j * k * zc * cb) * sb / np.sqrt(2.0 * l * (l + 1))
            if p == 0:
                c0 = 1j * pi * ax + tau * cb * ay
                c1 = 1j * pi * ay - tau * cb * ax
                acc += wb[ib] * pref * (1j ** l) * (c0 * g0 + c1 * g1)
            else:
                c0 = tau * ax - 1j * pi * ay * cb
                c1 = tau * ay + 1j * pi * ax * cb
                acc += wb[ib] * pref * (1j ** (l + 1)) * (c0 * g0 + c1 * g1)
        out[:, n] = acc
    return out


def nyquist_weights_reconstruct(samples, grid, k, pts):
    """sum_ij (pi/2) f(x_ij) J_1(k |x - x_ij|)/(k |x - x_ij|) at points pts [P, 2]."""
    pts = np.asarray(pts, dtype=float)
    d = pts[:, None, :] - np.asarray(grid)[None, :, :]
    return 0.5 * np.pi * (jinc(k * np.hypot(d[..., 0], d[..., 1])) @ np.asarray(samples))
