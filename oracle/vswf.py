"""Vector spherical wavefunctions and plane-wave coefficients (oracle, FP64).

Test infrastructure only: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Basis (App. I.A, eq. "vector_spherical_wf"):
  phi_lm(kx)   = h_l(kr) Pbar_l^|m|(cos t) e^{i m f}      (outgoing)
  Rphi_lm(kx)  = j_l(kr) Pbar_l^|m|(cos t) e^{i m f}      (regular)
  Phi_lm0      = (1/sqrt(2l(l+1))) grad(phi_lm) x x        ("M-type")
  Phi_lm1      = (1/k) curl Phi_lm0                        ("N-type")
Written out in spherical components (rho = kr, z_l = h_l or j_l):
  Phi_lm0 = z_l [ i pi theta_hat - tau phi_hat ] e^{imf} / sqrt(2l(l+1))
  Phi_lm1 = [ l(l+1) z_l/rho Pbar r_hat + (rho z_l)'/rho (tau theta_hat
              + i pi phi_hat) ] e^{imf} / sqrt(2l(l+1))
with pi = m Pbar/sin t and tau = dPbar/dt.  Both forms are pinned against the
defining curl relations by finite differences in the tests.

Coefficient order (truncation of App. I.B): n = p*lmax(lmax+2) + l(l+1)-1+m,
l = 1..lmax, m = -l..l, p in {0, 1}; 2*lmax*(lmax+2) coefficients.
"""
import numpy as np

from .special import pbar, pi_fn, sph_h1, sph_jn, tau_fn


def n_coeffs(lmax):
    return 2 * lmax * (lmax + 2)


def index_list(lmax):
    """[(p, l, m)] in coefficient order."""
    out = []
    for p in (0, 1):
        for l in range(1, lmax + 1):
            for m in range(-l, l + 1):
                out.append((p, l, m))
    return out


def _spherical(pts):
    pts = np.asarray(pts, dtype=float)
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    theta = np.arccos(np.clip(z / r, -1.0, 1.0))
    phi = np.arctan2(y, x)
    return r, theta, phi


def _unit_vectors(theta, phi):
    st, ct, sf, cf = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    rh = np.stack([st * cf, st * sf, ct], -1)
    th = np.stack([ct * cf, ct * sf, -st], -1)
    ph = np.stack([-sf, cf, np.zeros_like(sf)], -1)
    return rh, th, ph


def vswf(lmax, k, pts, regular=False):
    """Phi_n(k x) (or R Phi_n when regular) at Cartesian points.

    pts: [..., 3] real, nonzero.  Returns complex array [..., L, 3]
    (Cartesian components), coefficient order as in index_list.
    """
    r, theta, phi = _spherical(pts)
    rho = k * r
    rh, th, ph = _unit_vectors(theta, phi)
    zf = sph_jn if regular else sph_h1
    z = [zf(l, rho) for l in range(lmax + 1)]
    out = []
    for p, l, m in index_list(lmax):
        norm = 1.0 / np.sqrt(2.0 * l * (l + 1))
        e = np.exp(1j * m * phi)
        P = pbar(l, m, np.cos(theta))
        pi = pi_fn(l, m, theta)
        tau = tau_fn(l, m, theta)
        if p == 0:
            v = (z[l] * (1j * pi * e))[..., None] * th - (z[l] * tau * e)[..., None] * ph
        else:
            dz = (rho * z[l - 1] - l * z[l]) / rho  # (rho z_l)'/rho
            v = ((l * (l + 1) * z[l] / rho * P * e)[..., None] * rh
                 + (dz * tau * e)[..., None] * th
                 + (dz * 1j * pi * e)[..., None] * ph)
        out.append(norm * v)
    return np.stack(out, axis=-2)


def vswf_farfield(lmax, dirs):
    """Angular far-field pattern of Phi_n: Phi_n(k r d) ~ e^{ikr}/(kr) * F_n(d).

    Uses the exact large-argument form h_l(x) ~ (-i)^{l+1} e^{ix}/x (reading of
    eq. "asymptotic", whose printed form drops this phase).  dirs: [..., 3]
    unit vectors.  Returns [..., L, 3].
    """
    _, theta, phi = _spherical(dirs)
    _, th, ph = _unit_vectors(theta, phi)
    out = []
    for p, l, m in index_list(lmax):
        norm = 1.0 / np.sqrt(2.0 * l * (l + 1))
        e = np.exp(1j * m * phi)
        pi = pi_fn(l, m, theta)
        tau = tau_fn(l, m, theta)
        if p == 0:
            c = (-1j) ** (l + 1)
            v = (c * 1j * pi * e)[..., None] * th - (c * tau * e)[..., None] * ph
        else:
            c = (-1j) ** l
            v = (c * tau * e)[..., None] * th + (c * 1j * pi * e)[..., None] * ph
        out.append(norm * v)
    return np.stack(out, axis=-2)


def plane_wave_angular(lmax, khat, pol):
    """a_{lmp}(beta, alpha) of App. II, eqs. "integrand_p_0"/"integrand_p_1".

    The plane wave A e^{i k khat.x} about the origin equals
    sum_n a_n R Phi_n(k x), with (beta, alpha) the polar/azimuthal angles of
    khat and
      a_lm0 = -4 i^l e^{-i m alpha}/sqrt(2l(l+1)) [i pi (beta_hat.A) + tau (alpha_hat.A)]
      a_lm1 = -4 i^{l+1} e^{-i m alpha}/sqrt(2l(l+1)) [tau (beta_hat.A) - i pi (alpha_hat.A)]
    (pi = m Pbar/sin beta, the m of the printed "i m pi" folded in).  The
    second printed form is used; the first ("4 i^m") is taken as a typo.
    """
    khat = np.asarray(khat, dtype=float)
    pol = np.asarray(pol, dtype=complex)
    beta = np.arccos(np.clip(khat[2], -1.0, 1.0))
    alpha = np.arctan2(khat[1], khat[0])
    _, bh, ah = _unit_vectors(np.array(beta), np.array(alpha))
    bA = np.dot(bh, pol)
    aA = np.dot(ah, pol)
    out = np.zeros(n_coeffs(lmax), dtype=complex)
    for n, (p, l, m) in enumerate(index_list(lmax)):
        pre = -4.0 * np.exp(-1j * m * alpha) / np.sqrt(2.0 * l * (l + 1))
        pi = float(pi_fn(l, m, beta))
        tau = float(tau_fn(l, m, beta))
        if p == 0:
            out[n] = pre * (1j ** l) * (1j * pi * bA + tau * aA)
        else:
            out[n] = pre * (1j ** (l + 1)) * (tau * bA - 1j * pi * aA)
    return out


def plane_wave_coeffs(lmax, k, khat, pol, positions):
    """Incident coefficients a0[i, n] of A e^{i k khat.x} about each x_i.

    App. I.C: the incident field is expanded in R Phi about every scatterer
    centre; for a plane wave the expansion about x_i is the one about the origin
    times the field phase at x_i, e^{i k khat.x_i} (reading of the phase sign).
    """
    ang = plane_wave_angular(lmax, khat, pol)
    ph = np.exp(1j * k * (np.asarray(positions, dtype=float) @ np.asarray(khat, dtype=float)))
    return ph[:, None] * ang[None, :]
