"""Pins of the CPU oracle against facts outside the oracle itself.

Each test checks one oracle function against a closed form, an invariant, a
textbook special case or an independent numerical route, chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails.
"""
import numpy as np
import pytest

from oracle import special as sp
from oracle.mie import mie_ab, mie_tmatrix_diag
from oracle.translation import Translation
from oracle.vswf import (index_list, n_coeffs, plane_wave_angular, plane_wave_coeffs,
                         vswf, vswf_farfield)

K = 2.0 * np.pi


# ----------------------------------------------------------------- Bessel / Legendre
def test_hankel_closed_forms():
    x = np.linspace(0.3, 40.0, 97)
    e = np.exp(1j * x)
    h0 = -1j * e / x
    h1 = -e * (x + 1j) / x**2
    h2 = 1j * e * (x**2 + 3j * x - 3) / x**3
    for l, ref in ((0, h0), (1, h1), (2, h2)):
        assert np.allclose(sp.sph_h1(l, x), ref, rtol=1e-13, atol=0)
    # Wronskian j_l y_{l-1} - j_{l-1} y_l = 1/x^2
    for l in range(1, 7):
        w = sp.sph_jn(l, x) * sp.sph_yn(l - 1, x) - sp.sph_jn(l - 1, x) * sp.sph_yn(l, x)
        assert np.allclose(w * x**2, 1.0, rtol=1e-11)


def test_pbar_orthonormal_and_scipy():
    from scipy.special import lpmv

    xg, wg = np.polynomial.legendre.leggauss(40)
    for m in range(0, 5):
        for l in range(m, 8):
            for l2 in range(m, 8):
                v = np.sum(wg * sp.pbar(l, m, xg) * sp.pbar(l2, m, xg))
                assert abs(v - (1.0 if l == l2 else 0.0)) < 1e-12
            # scipy includes the Condon-Shortley phase (-1)^m
            from math import factorial
            nrm = np.sqrt((2 * l + 1) / 2 * factorial(l - m) / factorial(l + m))
            ref = (-1) ** m * nrm * lpmv(m, l, xg)
            assert np.allclose(sp.pbar(l, m, xg), ref, atol=1e-12)


def test_pi_tau_definitions():
    th = np.linspace(0.05, np.pi - 0.05, 31)
    h = 1e-6
    for l in range(1, 6):
        for m in range(-l, l + 1):
            P = sp.pbar(l, m, np.cos(th))
            assert np.allclose(sp.pi_fn(l, m, th), m * P / np.sin(th), atol=1e-12)
            fd = (sp.pbar(l, m, np.cos(th + h)) - sp.pbar(l, m, np.cos(th - h))) / (2 * h)
            assert np.allclose(sp.tau_fn(l, m, th), fd, atol=1e-7)
    # poles: pi_l^{+-1}(0) = +-sqrt((2l+1)/2 * l(l+1)) / 2 ; tau_l^1(0) the same value
    for l in range(1, 6):
        v = np.sqrt((2 * l + 1) / 2 / (l * (l + 1))) * l * (l + 1) / 2
        assert abs(sp.pi_fn(l, 1, 0.0) - v) < 1e-12
        assert abs(sp.tau_fn(l, 1, 0.0) - v) < 1e-12
        assert abs(sp.pi_fn(l, 2, 0.0)) < 1e-14


# ----------------------------------------------------------------- VSWFs
def _curl(f, x, h=1e-5):
    J = [(f(x + e) - f(x - e)) / (2 * h) for e in np.eye(3) * h]
    return np.stack([J[1][..., 2] - J[2][..., 1], J[2][..., 0] - J[0][..., 2],
                     J[0][..., 1] - J[1][..., 0]], -1)


@pytest.mark.parametrize("regular", [False, True])
def test_vswf_curl_relations(regular):
    lmax = 3
    L = n_coeffs(lmax)
    f = lambda x: vswf(lmax, K, x, regular)  # noqa: E731
    for x0 in (np.array([0.31, -0.22, 0.17]), np.array([-0.4, 0.1, -0.35])):
        V = f(x0)
        c = _curl(f, x0) / K
        scale = np.abs(V).max()
        # Phi_lm1 = (1/k) curl Phi_lm0 and, by the vector Helmholtz equation, back
        assert np.abs(c[:L // 2] - V[L // 2:]).max() / scale < 1e-8
        assert np.abs(c[L // 2:] - V[:L // 2]).max() / scale < 1e-8
        # divergence-free
        h = 1e-5
        div = sum((f(x0 + e)[:, a] - f(x0 - e)[:, a]) / (2 * h) for a, e in enumerate(np.eye(3) * h))
        assert np.abs(div).max() / scale < 1e-7


def test_vswf_m_type_from_scalar():
    """Phi_lm0 = (1/sqrt(2l(l+1))) grad(phi_lm) x x, by finite differences."""
    lmax = 3
    x0 = np.array([0.21, 0.33, -0.12])
    h = 1e-6

    def phi(x, l, m):
        r = np.linalg.norm(x)
        th = np.arccos(x[2] / r)
        f = np.arctan2(x[1], x[0])
        return sp.sph_h1(l, K * r) * sp.pbar(l, m, np.cos(th)) * np.exp(1j * m * f)

    V = vswf(lmax, K, x0)
    for n, (p, l, m) in enumerate(index_list(lmax)):
        if p:
            continue
        g = np.array([(phi(x0 + e, l, m) - phi(x0 - e, l, m)) / (2 * h) for e in np.eye(3) * h])
        ref = np.cross(g, x0) / np.sqrt(2 * l * (l + 1))
        assert np.allclose(V[n], ref, atol=1e-7 * np.abs(V).max())


def test_farfield_asymptotics():
    lmax = 3
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    F = vswf_farfield(lmax, d)
    errs = []
    for r in (1e3, 2e3, 4e3):
        V = vswf(lmax, K, r * d) * (K * r) * np.exp(-1j * K * r)
        errs.append(np.abs(V - F).max())
    # remainder is O(1/(kr)), halving with r
    assert errs[2] < 2e-4 and errs[1] / errs[2] > 1.8


# ----------------------------------------------------------------- plane wave
def test_plane_wave_expansion_pointwise(rng):
    for trial in range(3):
        khat = rng.normal(size=3)
        khat /= np.linalg.norm(khat)
        e1 = np.cross(khat, rng.normal(size=3))
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(khat, e1)
        pol = e1 + (0.3 - 0.7j) * e2
        pts = rng.uniform(-0.2, 0.2, size=(5, 3))
        a = plane_wave_angular(18, khat, pol)
        E = np.einsum('n,pnc->pc', a, vswf(18, K, pts, regular=True))
        ref = pol[None, :] * np.exp(1j * K * pts @ khat)[:, None]
        assert np.abs(E - ref).max() < 1e-12
    # normal incidence (pole of the angular functions)
    a = plane_wave_angular(18, [0, 0, 1.0], [1.0, 0, 0])
    pts = rng.uniform(-0.2, 0.2, size=(5, 3))
    E = np.einsum('n,pnc->pc', a, vswf(18, K, pts, regular=True))
    assert np.abs(E - np.array([1.0, 0, 0])[None] * np.exp(1j * K * pts[:, 2])[:, None]).max() < 1e-12


def test_plane_wave_about_shifted_centre(rng):
    x0 = np.array([1.3, -0.4, 0.2])
    khat = np.array([np.sin(0.4), 0.0, np.cos(0.4)])
    pol = np.array([np.cos(0.4), 0.0, -np.sin(0.4)])
    a0 = plane_wave_coeffs(18, K, khat, pol, x0[None])[0]
    pts = x0 + rng.uniform(-0.15, 0.15, size=(4, 3))
    E = np.einsum('n,pnc->pc', a0, vswf(18, K, pts - x0, regular=True))
    assert np.abs(E - pol[None] * np.exp(1j * K * pts @ khat)[:, None]).max() < 1e-12


# ----------------------------------------------------------------- translation
def test_translation_addition_theorem_pointwise():
    """Phi_u(k(x-x_s)) = sum_v xi_uv(k(x_t-x_s)) R Phi_v(k(x-x_t)) near x_t."""
    xs = np.array([0.0, 0.0, 0.0])
    for xt in (np.array([0.43, -0.31, 0.22]), np.array([0.6, 0.0, 0.0]), np.array([-0.9, 1.2, 0.0])):
        pts = xt + np.array([[0.03, 0.02, -0.04], [-0.05, 0.01, 0.02], [0.0, -0.04, 0.03]])
        lhs = vswf(2, K, pts - xs)
        tr = Translation(K, 2, 14)
        X = tr.block(xt - xs)
        rhs = np.einsum('uv,pvc->puc', X, vswf(14, K, pts - xt, regular=True))
        assert np.abs(rhs - lhs).max() / np.abs(lhs).max() < 1e-12


@pytest.mark.parametrize("lmax,xt", [(3, (0.6, -0.6, 0.0)), (6, (0.6, 0.0, 0.0)), (5, (0.4, 0.3, 0.5))])
def test_translation_by_projection(lmax, xt):
    """Each xi_uv equals the projection of Phi_u(k(x-x_s)) onto R Phi_v on a
    sphere about x_t (Gauss-Legendre x trapezoid quadrature), an independent
    route to the same coefficients (up to lmax 6, the nearest-neighbour
    distance of the lattice included)."""
    xs = np.array([0.0, 0.0, 0.0])
    xt = np.array(xt)
    rho0 = 0.2
    xg, wg = np.polynomial.legendre.leggauss(36)
    nphi = 72
    phis = np.arange(nphi) * 2 * np.pi / nphi
    TH, PH = np.meshgrid(np.arccos(xg), phis, indexing='ij')
    W = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :])
    rh = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    th = np.stack([np.cos(TH) * np.cos(PH), np.cos(TH) * np.sin(PH), -np.sin(TH)], -1)
    ph = np.stack([-np.sin(PH), np.cos(PH), np.zeros_like(PH)], -1)
    E = vswf(lmax, K, xt + rho0 * rh - xs)  # [T, P, L, 3]
    X = Translation(K, lmax).block(xt - xs)
    kr = K * rho0
    for v, (p, l, m) in enumerate(index_list(lmax)):
        e = np.exp(1j * m * PH)
        pi = sp.pi_fn(l, m, TH)
        tau = sp.tau_fn(l, m, TH)
        C = (1j * pi * e)[..., None] * th - (tau * e)[..., None] * ph
        Bv = (tau * e)[..., None] * th + (1j * pi * e)[..., None] * ph
        ang = (C if p == 0 else Bv)
        proj = np.einsum('tp,tpuc,tpc->u', W, E, np.conj(ang))
        nrm = 2 * np.pi * l * (l + 1) / np.sqrt(2 * l * (l + 1))
        if p == 0:
            radial = sp.sph_jn(l, kr)
        else:
            radial = (kr * sp.sph_jn(l - 1, kr) - l * sp.sph_jn(l, kr)) / kr
        coef = proj / (nrm * radial)
        assert np.allclose(coef, X[:, v], atol=1e-11 * np.abs(X).max())


@pytest.mark.parametrize("lmax", [3, 4, 5, 6])
def test_translation_inplane_parity_pattern(lmax):
    """For d in the z = 0 plane, xi couples only indices with equal
    (l + m + p) mod 2 (z-mirror symmetry); each class holds lmax(lmax+2)."""
    X = Translation(K, lmax).blocks(np.array([[0.6, 0.0, 0.0], [1.2, -1.8, 0.0], [-0.6, 2.4, 0.0]]))
    cls = np.array([(l + m + p) % 2 for p, l, m in index_list(lmax)])
    mask = cls[:, None] != cls[None, :]
    assert np.abs(X[:, mask]).max() < 1e-15 * np.abs(X).max() + 1e-300
    assert np.count_nonzero(cls == 0) == np.count_nonzero(cls == 1) == lmax * (lmax + 2)
    # and the sign rule for d -> -d: xi(-d) = sigma xi(d) sigma, sigma = (-1)^(l+p)
    sig = np.array([(-1) ** (l + p) for p, l, m in index_list(lmax)])
    d = np.array([1.2, -1.8, 0.0])
    tr = Translation(K, lmax)
    assert np.allclose(tr.block(-d), sig[:, None] * tr.block(d) * sig[None, :], atol=1e-14)


def test_translation_dipole_green_function():
    """Electric-dipole (l = 1, N-type) to electric-dipole coupling is the free
    dyadic Green's function (I + grad grad / k^2) e^{ikd}/d, up to the basis
    normalisation: the radiated field of N-type l = 1 waves about x_s,
    re-expanded at x_t, must reproduce the field of the same dipole evaluated
    directly there.  Checked via the field at x_t itself (only l' = 1 regular
    N-type waves are nonzero at their own centre)."""
    xs = np.zeros(3)
    xt = np.array([0.7, 0.3, -0.2])
    lmax = 1
    X = Translation(K, lmax).block(xt - xs)
    # R Phi_{1m1}(0): the only nonzero regular waves at the origin
    eps = np.array([[1e-9, 0, 0]])
    R0 = vswf(1, K, eps, regular=True)[0]  # [L, 3]
    field_t = X @ R0  # sum_v xi_uv R Phi_v(0): [u, 3]
    direct = vswf(1, K, (xt - xs)[None])[0]
    assert np.allclose(field_t, direct, atol=1e-8 * np.abs(direct).max())
    # N-type l = 1 outgoing waves are electric-dipole fields: Phi_{1m1}(k d) =
    # G(d) . p_m with one fixed moment p_m for every d, G(d) the free dyadic
    # Green's function (I + grad grad / k^2) e^{ikd}/d (textbook closed form).
    def G(d):
        r = np.linalg.norm(d)
        rh = d / r
        kr = K * r
        g = np.exp(1j * kr) / r
        return g * ((1 + 1j / kr - 1 / kr**2) * np.eye(3) - (1 + 3j / kr - 3 / kr**2) * np.outer(rh, rh))

    ds = [np.array([0.7, 0.3, -0.2]), np.array([-0.2, 1.1, 0.5]), np.array([0.05, -0.3, 0.9])]
    for u in range(3, 6):
        pm = np.linalg.solve(G(ds[0]), vswf(1, K, ds[0][None])[0][u])
        for d in ds[1:]:
            ref = G(d) @ pm
            assert np.allclose(vswf(1, K, d[None])[0][u], ref, atol=1e-12 * np.abs(ref).max())


# ----------------------------------------------------------------- Mie
def test_mie_unitarity_and_rayleigh():
    for x in (0.3, 0.94, 1.57):
        for l in range(1, 5):
            a, b, _, _ = mie_ab(l, x, 2.0)
            for t in (-a, -b):
                assert abs(t.real + abs(t) ** 2) < 1e-14  # lossless: Re t = -|t|^2
    x = 1e-3
    m = 2.0
    a1, _, _, _ = mie_ab(1, x, m)
    ref = -2j / 3 * x**3 * (m * m - 1) / (m * m + 2)
    assert abs(a1 - ref) / abs(ref) < 1e-5


def test_mie_log_derivative_route():
    """a_l, b_l agree with the logarithmic-derivative form (B&H eq. 4.88) with
    D_l(mx) from downward recurrence: an independent algebraic route."""
    for x in (0.5, 1.2, 2.3):
        m = 2.0 + 0.1j
        mx = m * x
        nmax = 60
        D = np.zeros(nmax + 1, dtype=complex)
        for n in range(nmax, 0, -1):
            D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
        for l in range(1, 5):
            psi = lambda n: x * sp.sph_jn(n, x)  # noqa: E731
            xi = lambda n: x * sp.sph_h1(n, x)  # noqa: E731
            fa = D[l] / m + l / x
            fb = m * D[l] + l / x
            a_ref = (fa * psi(l) - psi(l - 1)) / (fa * xi(l) - xi(l - 1))
            b_ref = (fb * psi(l) - psi(l - 1)) / (fb * xi(l) - xi(l - 1))
            a, b, _, _ = mie_ab(l, x, m)
            assert abs(a - a_ref) < 1e-12 and abs(b - b_ref) < 1e-12


def test_mie_radius_derivative_fd():
    for r in (0.12, 0.2, 0.28):
        t, dt = mie_tmatrix_diag(3, K, r, 2.0)
        h = 1e-6
        tp, _ = mie_tmatrix_diag(3, K, r + h, 2.0)
        tm, _ = mie_tmatrix_diag(3, K, r - h, 2.0)
        fd = (tp - tm) / (2 * h)
        assert np.allclose(dt, fd, atol=1e-7 * np.abs(dt).max())


def test_mie_order_mapping():
    """p = 0 (M-type) carries -b_l, p = 1 (N-type) carries -a_l."""
    t, _ = mie_tmatrix_diag(2, K, 0.2, 2.0)
    for n, (p, l, m) in enumerate(index_list(2)):
        a, b, _, _ = mie_ab(l, K * 0.2, 2.0)
        assert t[n] == (-b if p == 0 else -a)
