"""Physics-level pins of the oracle's solve, readout and adjoint.

The paper prints no worked values, so these tests pin the assembled system
against laws and closed forms: Mie's single-sphere cross sections, the
Rayleigh dipole, energy conservation (optical theorem), reciprocity,
translation invariance, independent solvers on the same system, and central
finite differences for the adjoint gradient.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.mie import mie_ab, mie_tmatrix_diag_many
from oracle.solver import (LatticeCoupling, coupling_dense, detector_vectors, extinction,
                           far_field, gmres,
                           near_field, objective_and_gradient_dense, rows_A, scattering,
                           solve_dense, system_dense)
from oracle.vswf import n_coeffs, plane_wave_coeffs

K = wl.K


def _random_cluster(rng, n, rmax=0.25, box=2.0, planar=False):
    pos = []
    while len(pos) < n:
        p = rng.uniform(-box, box, 3)
        if planar:
            p[2] = 0.0
        if all(np.linalg.norm(p - q) > 2.05 * rmax for q in pos):
            pos.append(p)
    return np.array(pos)


def _solve(pos, radii, lmax, khat, pol):
    t, _ = mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    a0 = plane_wave_coeffs(lmax, K, khat, pol, pos)
    return solve_dense(pos, K, lmax, t, a0)


def test_single_sphere_cross_sections():
    """One sphere: C_ext and C_sca through plane-wave coefficients, T, solve and
    far-field readout equal the truncated Mie series (2 pi/k^2) sum (2l+1) ..."""
    lmax = 3
    for r in (0.15, 0.28):
        kh, po = wl.incidence("p10")
        s = _solve(np.zeros((1, 3)), [r], lmax, kh, po)
        cext = extinction(s, np.zeros((1, 3)), K, lmax, kh, po)
        csca = scattering(s, np.zeros((1, 3)), K, lmax, 48, 96)
        x = K * r
        qe = qs = 0.0
        for l in range(1, lmax + 1):
            a, b, _, _ = mie_ab(l, x, wl.N_REL)
            qe += (2 * l + 1) * np.real(a + b)
            qs += (2 * l + 1) * (abs(a) ** 2 + abs(b) ** 2)
        ref_e = 2 * np.pi / K**2 * qe
        ref_s = 2 * np.pi / K**2 * qs
        assert abs(cext - ref_e) / ref_e < 1e-12
        assert abs(csca - ref_s) / ref_s < 1e-12


def test_rayleigh_dipole_far_field():
    """A tiny sphere radiates as an electric dipole p = r^3 (m^2-1)/(m^2+2) E0:
    F(d) = k^2 (d x p) x d."""
    r = 2e-3
    s = _solve(np.zeros((1, 3)), [r], 2, *wl.incidence("x"))
    dirs = np.array([[0.3, 0.4, np.sqrt(0.75)], [0.0, 1.0, 0.0], [-0.6, 0.0, -0.8]])
    F = far_field(s, np.zeros((1, 3)), K, 2, dirs)
    m2 = wl.N_REL**2
    p = np.array([1.0, 0, 0]) * r**3 * (m2 - 1) / (m2 + 2)
    ref = K**2 * np.cross(np.cross(dirs, p), dirs)
    assert np.abs(F - ref).max() / np.abs(ref).max() < 1e-3


@pytest.mark.parametrize("rhs", ["x", "p10"])
def test_optical_theorem_lattice(rhs):
    """Lossless spheres: extinction (forward amplitude) equals the scattered
    power integrated over all directions, for the 8 x 8 lattice at lmax 2."""
    pos, radii, _, _, cfg = wl.config_inputs("c1")
    kh, po = wl.incidence(rhs)
    s = _solve(pos, radii, cfg["lmax"], kh, po)
    cext = extinction(s, pos, K, cfg["lmax"], kh, po)
    csca = scattering(s, pos, K, cfg["lmax"], 96, 192)
    assert abs(cext - csca) / csca < 1e-10


def test_reciprocity(rng):
    """pol_s . F(k_s; k_i, pol_i) = pol_i . F(-k_i; -k_s, pol_s) on a random 3D
    cluster (checks the transpose structure of A and the plane-wave basis)."""
    pos = _random_cluster(rng, 7)
    radii = rng.uniform(0.12, 0.25, len(pos))
    lmax = 3

    def frame(k):
        e1 = np.cross(k, [0.3, -0.2, 0.9])
        e1 /= np.linalg.norm(e1)
        return e1, np.cross(k, e1)

    ki = rng.normal(size=3)
    ki /= np.linalg.norm(ki)
    ks = rng.normal(size=3)
    ks /= np.linalg.norm(ks)
    for pi_ in frame(ki):
        for ps_ in frame(ks):
            s1 = _solve(pos, radii, lmax, ki, pi_)
            f1 = np.dot(ps_, far_field(s1, pos, K, lmax, ks[None])[0])
            s2 = _solve(pos, radii, lmax, -ks, ps_)
            f2 = np.dot(pi_, far_field(s2, pos, K, lmax, -ki[None])[0])
            assert abs(f1 - f2) < 1e-11 * max(abs(f1), 1e-3)


def test_translation_invariance(rng):
    pos = _random_cluster(rng, 5, planar=True)
    radii = rng.uniform(0.12, 0.25, len(pos))
    kh, po = wl.incidence("p10")
    s = _solve(pos, radii, 2, kh, po)
    delta = np.array([0.37, -1.1, 0.0])
    s2 = _solve(pos + delta, radii, 2, kh, po)
    assert np.allclose(s2, s * np.exp(1j * K * kh @ delta), atol=1e-13 * np.abs(s).max())


def test_lattice_coupling_and_rows_match_dense(rng):
    nx, ny, lmax = 5, 4, 2
    pos = wl.lattice_positions(nx, ny)
    A = coupling_dense(pos, K, lmax)
    lc = LatticeCoupling(nx, ny, wl.PITCH, K, lmax)
    L = n_coeffs(lmax)
    x = rng.normal(size=(nx * ny, L)) + 1j * rng.normal(size=(nx * ny, L))
    assert np.allclose(lc.apply(x), (A @ x.ravel()).reshape(-1, L), atol=1e-13)
    assert np.allclose(lc.apply(x, transpose=True), (A.T @ x.ravel()).reshape(-1, L), atol=1e-13)
    rows = [0, 7, 19]
    assert np.allclose(rows_A(pos, K, lmax, x, rows), (A @ x.ravel()).reshape(-1, L)[rows], atol=1e-13)
    assert np.allclose(rows_A(pos, K, lmax, x, rows, transpose=True),
                       (A.T @ x.ravel()).reshape(-1, L)[rows], atol=1e-13)


def test_gmres_matches_lu():
    pos = wl.lattice_positions(6, 5)
    radii = wl.uniform_radii(30, 0.15, 0.25, 7)
    lmax = 3
    t, _ = mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    a0 = plane_wave_coeffs(lmax, K, *wl.incidence("x"), pos)
    B, A, T = system_dense(pos, K, lmax, t)
    b = (t * a0).ravel()
    s_lu = np.linalg.solve(B, b)
    assert np.linalg.norm(B @ s_lu - b) / np.linalg.norm(b) < 1e-14
    lc = LatticeCoupling(6, 5, wl.PITCH, K, lmax)
    mv = lambda x: x - (t * lc.apply(x.reshape(30, -1))).ravel()  # noqa: E731
    s_gm, it, rr = gmres(mv, b, tol=1e-13, restart=10)
    assert rr <= 1e-13 and it > 10  # exercised at least one restart
    assert np.linalg.norm(s_gm - s_lu) / np.linalg.norm(s_lu) < 1e-11


def test_near_field_tends_to_far_field():
    pos = wl.lattice_positions(3, 2)
    radii = wl.uniform_radii(6, 0.15, 0.25, 9)
    s = _solve(pos, radii, 2, *wl.incidence("x"))
    d = np.array([0.2, -0.3, 0.933])
    d /= np.linalg.norm(d)
    F = far_field(s, pos, K, 2, d[None])[0]
    errs = []
    for r in (2e3, 4e3):
        E = near_field(s, pos, K, 2, (r * d)[None])[0]
        errs.append(np.abs(E * r * np.exp(-1j * K * r) - F).max())
    assert errs[1] < 2e-3 * np.abs(F).max() and errs[0] / errs[1] > 1.8


def test_adjoint_gradient_fd():
    """dO/dr from one forward and one adjoint solve equals central differences
    (O = |E_inc + E_sca|^2 at a detector point above a 3 x 3 lattice)."""
    pos = wl.lattice_positions(3, 3)
    radii = wl.uniform_radii(9, 0.12, 0.28, 11)
    kh, po = wl.incidence("x")
    xd = np.array([0.6, 0.6, 3.0])
    lmax = 2
    O, g, _, _ = objective_and_gradient_dense(pos, K, lmax, radii, wl.N_REL, kh, po, xd)
    h = 1e-6
    for i in (0, 4, 8):
        rp = radii.copy()
        rp[i] += h
        rm = radii.copy()
        rm[i] -= h
        Op = objective_and_gradient_dense(pos, K, lmax, rp, wl.N_REL, kh, po, xd)[0]
        Om = objective_and_gradient_dense(pos, K, lmax, rm, wl.N_REL, kh, po, xd)[0]
        fd = (Op - Om) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * np.abs(g).max()


def test_detector_vectors_are_the_near_field(rng):
    """The point-detector functional of App. IV (eq. "performance_metric" with
    sigma a point mass at xd) is the scattered field at xd, eq.
    "sca_fld_concise": v[c] . s = E_sca,c(xd) for random s, on a 3-D cluster
    and on a lattice, with detectors above and below the lattice plane (a
    mirrored or reversed displacement in the detector vectors fails here)."""
    lmax = 3
    L = n_coeffs(lmax)
    cluster = _random_cluster(rng, 6)
    for pos, pts in ((cluster, ([0.7, -0.4, 3.5], [0.3, 1.1, -3.6], [4.0, 4.5, 0.2])),
                     (wl.lattice_positions(4, 3), ([0.7, 0.4, 2.5], [0.3, 1.1, -1.7], [5.0, 4.0, 0.9]))):
        s = rng.normal(size=(len(pos), L)) + 1j * rng.normal(size=(len(pos), L))
        for xd in pts:
            v = detector_vectors(pos, K, lmax, xd)
            z = np.einsum('cil,il->c', v, s)
            E = near_field(s, pos, K, lmax, np.array([xd]))[0]
            assert np.abs(z - E).max() <= 1e-12 * np.abs(E).max()
            # the mirror image of the detector sees a different field
            xm = np.array(xd) * np.array([1.0, 1.0, -1.0])
            zm = np.einsum('cil,il->c', detector_vectors(pos, K, lmax, xm), s)
            assert np.abs(zm - E).max() > 1e-3 * np.abs(E).max()


@pytest.mark.parametrize("xd", [[0.6, 0.6, 3.0], [0.9, 0.3, -2.2]])
def test_objective_is_total_intensity_at_the_detector(xd):
    """O returned with the gradient is |E_inc + E_sca|^2 at xd (reading of the
    adjoint workload's objective), with E_inc the plane wave's closed form and
    E_sca the direct-sum readout of the LU solution."""
    pos = wl.lattice_positions(3, 3)
    radii = wl.uniform_radii(9, 0.12, 0.28, 11)
    kh, po = wl.incidence("p10")
    lmax = 2
    xd = np.array(xd)
    O, g, s, mu = objective_and_gradient_dense(pos, K, lmax, radii, wl.N_REL, kh, po, xd)
    s_ref = _solve(pos, radii, lmax, kh, po)
    assert np.linalg.norm(s - s_ref) <= 1e-13 * np.linalg.norm(s_ref)
    E = po * np.exp(1j * K * np.dot(kh, xd)) + near_field(s_ref, pos, K, lmax, xd[None])[0]
    assert abs(O - np.sum(np.abs(E) ** 2)) <= 1e-12 * O
