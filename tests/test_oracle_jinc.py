"""Pins of the oracle's jinc sources (App. II), independent of the HIP path:
Gamma_m's closed form against its defining integral, the k-space jinc field
at its source plane against A^T J_1(k rho)/(k rho), the Gamma route to the
expansion coefficients against direct 2-D quadrature, the expansion against
the field pointwise, and the Nyquist reconstruction of a band-limited field
from lambda/2 samples with (pi/2)-weighted jincs."""
import numpy as np
import pytest
from scipy import special as sps

import workloads as wl
from oracle.jinc import (gamma_closed, gamma_quadrature, jinc, jinc_coeffs, jinc_coeffs_quadrature,
                         jinc_field, nyquist_weights_reconstruct, transverse_field_at_source_plane)
from oracle.vswf import vswf

K = wl.K


@pytest.mark.parametrize("m", [-4, -1, 0, 1, 3, 7])
def test_gamma_closed_form(m):
    for xi, eta, rho in [(0.3, 0.0, 2.5), (2.1, 0.5 * np.pi, 17.0), (-1.2, 0.4, 0.01), (0.0, 0.0, 60.0)]:
        a = gamma_closed(m, xi, eta, rho)
        b = gamma_quadrature(m, xi, eta, rho, n=1024)
        assert abs(a - b) < 1e-13, (m, xi, eta, rho, a, b)


def test_jinc_field_in_its_source_plane_is_the_cylindrical_jinc():
    src = (0.3, -0.2, 1.0, 0.7 + 0.2j, -0.4 + 0.1j)
    pts = np.array([[0.3, -0.2, 1.0], [0.5, 0.1, 1.0], [1.7, -1.1, 1.0], [-2.0, 3.0, 1.0]])
    E = jinc_field(src, K, pts, n_beta=400, n_alpha=400)
    ref = transverse_field_at_source_plane(src, K, pts)
    assert np.abs(E[:, :2] - ref[:, :2]).max() < 1e-10
    # the spherical j_1 of the spatial display is a different function
    rho = np.hypot(pts[:, 0] - 0.3, pts[:, 1] + 0.2)
    sph = np.where(rho > 0, sps.spherical_jn(1, K * np.maximum(rho, 1e-12)) / (K * np.maximum(rho, 1e-12)), 1 / 3)
    assert np.abs(sph - jinc(K * rho)).max() > 0.1


def test_gamma_route_matches_direct_quadrature():
    lmax = 3
    src = (0.1, 0.2, -1.5, 1.0, 0.5j)
    pos = np.array([[0.0, 0.0, 0.0], [0.6, 0.0, 0.0], [1.2, -1.8, 0.0], [2.4, 0.6, 0.0]])
    a = jinc_coeffs(lmax, K, src, pos, n_beta=96)
    b = jinc_coeffs_quadrature(lmax, K, src, pos, n_beta=96, n_alpha=96)
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_expansion_reproduces_the_field_pointwise():
    """sum_n a_n R Phi_n(k(x - x_i)) equals the jinc field near x_i."""
    lmax = 16
    src = (0.2, -0.1, -1.0, 1.0, 0.3)
    xi = np.array([0.6, 0.3, 0.0])
    a = jinc_coeffs(lmax, K, src, xi[None], n_beta=200)[0]
    pts = xi + np.array([[0.05, -0.03, 0.04], [-0.08, 0.02, -0.05], [0.0, 0.07, 0.02]])
    E = np.einsum('n,pnc->pc', a, vswf(lmax, K, pts - xi, regular=True))
    ref = jinc_field(src, K, pts, n_beta=200, n_alpha=256)
    assert np.abs(E - ref).max() < 1e-10 * np.abs(ref).max()


def test_nyquist_reconstruction_of_a_band_limited_field():
    """f(rho) = J_4(k' rho)/(k' rho)^4, band-limited to k' = 0.8 k, from its
    samples on the lambda/2 grid: the (pi/2)-weighted jincs reproduce it."""
    kp = 0.8 * K
    c = np.array([0.13, -0.07])

    def f(x):
        r = np.hypot(x[..., 0] - c[0], x[..., 1] - c[1])
        u = np.maximum(kp * r, 1e-12)
        return np.where(kp * r > 1e-6, sps.jv(4, u) / u ** 4, 1.0 / 384.0)

    h = 0.5  # lambda / 2
    M = 40
    ii = np.arange(-M, M + 1) * h
    grid = np.stack(np.meshgrid(ii, ii, indexing='ij'), -1).reshape(-1, 2)
    pts = np.array([[0.0, 0.0], [0.21, 0.34], [-0.4, 0.17], [1.1, -0.9]])
    rec = nyquist_weights_reconstruct(f(grid), grid, K, pts)
    assert np.abs(rec - f(pts)).max() < 1e-6 * np.abs(f(pts)).max()
