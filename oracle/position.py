"""Position sensitivities of a point-detector objective (oracle, FP64).

Test infrastructure only.

App. IV differentiates the objective through the Maxwell operator with
respect to every geometric parameter; for scatterer positions q_i (eq.
"grad_pos_overlap") three things move with x_i:
  * the translation blocks that touch scatterer i, A_jl = xi(k(x_j - x_l))^T
    with j = i (i as the target) or l = i (i as the source);
  * the incident coefficients about x_i (a plane wave carries e^{ik.x_i});
  * the detector vector v_c,i = Phi(k(x_d - x_i))_c (the field of scatterer i
    seen at the detector).
With B = I - T A, B s = T a0, O = f(z), z_c = sum_i v_c,i^T s_i, w =
sum_c f'_c v_c and B^T mu = w (the adjoint system of App. IV in
preconditioned form), lambda = T^T mu is the paper's adjoint unknown and
  dO/dq = 2 Re[ lambda^T (dA/dq s + da0/dq) + sum_c f'_c (dv_c/dq)^T s ].
The derivative of a translation block is taken analytically from eq.
"tran_coeff": with xi_uv(k d) = e^{i mu phi} sum_q C_uvq h_q(k r) Pbar_q^|mu|(cos theta),
mu = m_u - m_v,
  grad_d xi_uv = e^{i mu phi} sum_q C_uvq [ k h_q'(kr) Pbar r_hat
                 + h_q(kr) dPbar/dtheta theta_hat / r
                 + h_q(kr) i mu (Pbar / sin theta) phi_hat / r ].
The detector term uses the addition theorem about x_d itself:
Phi_u(k(x_d - x_i)) = sum_v xi_uv(k(x_d - x_i)) R Phi_v(0), where only the
l' = 1 regular waves are nonzero at their own centre, so
d/dx_i Phi_u(k(x_d - x_i)) = - sum_v grad xi_uv(k(x_d - x_i)) R Phi_v(0).
"""
import numpy as np

from .special import pbar, pi_fn, sph_h1, tau_fn
from .translation import Translation
from .vswf import n_coeffs, vswf


def _sph_h1_prime(q, x):
    from scipy import special as sps

    return sps.spherical_jn(q, x, derivative=True) + 1j * sps.spherical_yn(q, x, derivative=True)


def translation_gradient(tr, d):
    """G[a, u, v] = d xi_uv(k d) / d d_a (a = x, y, z) for one displacement
    d [3] (physical units; the translation object's k and truncations)."""
    d = np.asarray(d, dtype=float)
    r = np.linalg.norm(d)
    theta = np.arccos(np.clip(d[2] / r, -1.0, 1.0))
    phi = np.arctan2(d[1], d[0])
    st, ct, sf, cf = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    rh = np.array([st * cf, st * sf, ct])
    th = np.array([ct * cf, ct * sf, -st])
    ph = np.array([-sf, cf, 0.0])
    kr = tr.k * r
    Q = tr.qmax
    h = np.array([sph_h1(q, kr) for q in range(Q + 1)])
    hp = np.array([_sph_h1_prime(q, kr) for q in range(Q + 1)])
    # Legendre data per (q, |mu|): Pbar, dPbar/dtheta, Pbar/sin(theta)
    P = np.zeros((Q + 1, Q + 1))
    dP = np.zeros((Q + 1, Q + 1))
    Ps = np.zeros((Q + 1, Q + 1))
    for q in range(Q + 1):
        for am in range(q + 1):
            P[q, am] = pbar(q, am, ct)
            dP[q, am] = tau_fn(q, am, theta)
            Ps[q, am] = pi_fn(q, am, theta) / am if am else 0.0
    adm = np.abs(tr.dm)  # [u, v]
    mu = tr.dm
    # radial, polar and azimuthal parts: sum_q C_uvq (...)_q
    s_r = np.einsum('uvq,quv->uv', tr.coef, (tr.k * hp)[:, None, None] * P[:, adm])
    s_t = np.einsum('uvq,quv->uv', tr.coef, (h / r)[:, None, None] * dP[:, adm])
    s_p = np.einsum('uvq,quv->uv', tr.coef, (h / r)[:, None, None] * Ps[:, adm]) * (1j * mu)
    e = np.exp(1j * mu * phi)
    return e[None] * (s_r[None] * rh[:, None, None] + s_t[None] * th[:, None, None] +
                      s_p[None] * ph[:, None, None])


def regular_at_origin(k):
    """R Phi_v(0) [6, 3] for the lmax = 1 regular waves, the limit at their
    own centre: means of the values at +-delta along z cancel the odd part of
    the expansion about the centre, and Richardson extrapolation over delta
    and 2 delta (delta = 1e-4 wavelengths) the delta^2 part, leaving
    O((k delta)^4) ~ 2e-13 (only the N-type waves are nonzero there)."""
    d = 1e-4
    v = vswf(1, k, np.array([[0.0, 0.0, d], [0.0, 0.0, -d], [0.0, 0.0, 2 * d], [0.0, 0.0, -2 * d]]),
             regular=True)
    m1, m2 = 0.5 * (v[0] + v[1]), 0.5 * (v[2] + v[3])
    return (4.0 * m1 - m2) / 3.0


def detector_vector_gradient(positions, k, lmax, xd):
    """dv[c, i, n, a] = d/dx_i,a Phi_n(k(xd - x_i))_c (a = x, y, z)."""
    pos = np.asarray(positions, dtype=float)
    N, L = len(pos), n_coeffs(lmax)
    tr = Translation(k, lmax, 1)
    R0 = regular_at_origin(k)  # [6, 3]
    out = np.zeros((3, N, L, 3), dtype=complex)
    for i in range(N):
        G = translation_gradient(tr, np.asarray(xd, dtype=float) - pos[i])  # [a, u, v]
        out[:, i, :, :] = -np.einsum('auv,vc->cua', G, R0)
    return out


def objective_and_position_gradient_dense(positions, k, lmax, radii, mrel, khat, pol, xd,
                                          parts=False):
    """O = sum_c |E_inc,c(xd) + E_sca,c(xd)|^2 and dO/dx_i [N, 3] for
    homogeneous spheres under one plane wave (dense LU throughout).  With
    parts=True a fifth value holds the coupling, incident and detector terms
    (each [N, 3], their sum is the gradient)."""
    from .mie import mie_tmatrix_diag_many
    from .solver import detector_vectors, system_dense
    from .vswf import plane_wave_coeffs

    pos = np.asarray(positions, dtype=float)
    khat = np.asarray(khat, dtype=float)
    N, L = len(pos), n_coeffs(lmax)
    t, _ = mie_tmatrix_diag_many(lmax, k, radii, mrel)
    a0 = plane_wave_coeffs(lmax, k, khat, pol, pos)
    B, A, T = system_dense(pos, k, lmax, t)
    s = np.linalg.solve(B, (t * a0).ravel()).reshape(N, L)
    v = detector_vectors(pos, k, lmax, xd)  # [3, N, L]
    Einc = np.asarray(pol, dtype=complex) * np.exp(1j * k * np.dot(khat, xd))
    Etot = Einc + np.einsum('cil,il->c', v, s)
    O = float(np.sum(np.abs(Etot) ** 2))
    fp = np.conj(Etot)  # f'(z_c) for f = |E_c|^2
    w = np.einsum('c,cil->il', fp, v)
    mu = np.linalg.solve(B.T, w.ravel()).reshape(N, L)
    lam = t * mu
    tr = Translation(k, lmax)
    g = np.zeros((N, 3), dtype=complex)
    for j in range(N):
        for l in range(N):
            if j == l:
                continue
            G = translation_gradient(tr, pos[j] - pos[l])  # d xi(k(x_j - x_l)) / d(x_j - x_l)
            term = np.einsum('v,auv,u->a', lam[j], G, s[l])
            g[j] += term  # x_j moves the target end
            g[l] -= term  # x_l moves the source end
    g_inc = np.einsum('il,il->i', lam, a0)[:, None] * (1j * k * khat)[None, :]
    dv = detector_vector_gradient(pos, k, lmax, xd)  # [c, i, n, a]
    g_det = np.einsum('c,cina,in->ia', fp, dv, s)
    out = (O, 2.0 * np.real(g + g_inc + g_det), s, mu)
    if parts:
        out = out + ({"coupling": 2.0 * np.real(g), "incident": 2.0 * np.real(g_inc),
                      "detector": 2.0 * np.real(g_det)},)
    return out


def objective_dense(positions, k, lmax, radii, mrel, khat, pol, xd):
    """O alone (for finite differences in the positions)."""
    from .mie import mie_tmatrix_diag_many
    from .solver import detector_vectors, system_dense
    from .vswf import plane_wave_coeffs

    pos = np.asarray(positions, dtype=float)
    N, L = len(pos), n_coeffs(lmax)
    t, _ = mie_tmatrix_diag_many(lmax, k, radii, mrel)
    a0 = plane_wave_coeffs(lmax, k, khat, pol, pos)
    B, _, _ = system_dense(pos, k, lmax, t)
    s = np.linalg.solve(B, (t * a0).ravel()).reshape(N, L)
    v = detector_vectors(pos, k, lmax, xd)
    Etot = np.asarray(pol, dtype=complex) * np.exp(1j * k * np.dot(khat, xd)) + \
        np.einsum('cil,il->c', v, s)
    return float(np.sum(np.abs(Etot) ** 2))
