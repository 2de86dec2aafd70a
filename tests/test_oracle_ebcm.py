"""Pins of the oracle's null-field (EBCM) T-matrix (App. I.B), independent of
the HIP path.  On a sphere it must equal the Lorenz-Mie T.  On a smooth body
of revolution (a prolate spheroid) the truncated T must converge, as lmax
grows, to a reciprocal (T^T = P T P, P the signed m -> -m permutation) and,
lossless, unitary (S = I + 2T, S^H S = I) matrix: the off-diagonal M/N and
l/l' couplings a sphere never exercises.  For the paper's cylinders it must
keep the z-mirror classes and the m blocks and converge with the quadrature
(the edges slow its convergence in lmax, a known property of the method)."""
import numpy as np
import pytest

import workloads as wl
from oracle.ebcm import cylinder_surface, ebcm_tmatrix, sphere_surface, spheroid_surface
from oracle.mie import mie_tmatrix_diag
from oracle.vswf import index_list

K = wl.K


@pytest.mark.parametrize("lmax,radius,m", [(3, 0.2, 2.0), (6, 0.25, 3.48), (4, 0.15, 1.5 + 0.2j)])
def test_ebcm_on_a_sphere_is_mie(lmax, radius, m):
    t, _ = mie_tmatrix_diag(lmax, K, radius, m)
    for surf in (sphere_surface(radius, 64), spheroid_surface(radius, radius, 64)):
        T = ebcm_tmatrix(lmax, K, m, surf)
        assert np.abs(T - np.diag(t)).max() < 1e-12 * np.abs(t).max()


def _perm(lmax):
    idx = index_list(lmax)
    pos = {v: i for i, v in enumerate(idx)}
    P = np.zeros((len(idx), len(idx)))
    for i, (p, l, m) in enumerate(idx):
        P[pos[(p, l, -m)], i] = (-1) ** m
    return P


def test_spheroid_converges_to_reciprocal_and_unitary():
    errs = []
    for lmax in (2, 4, 6, 8):
        T = ebcm_tmatrix(lmax, K, 1.5, spheroid_surface(0.1, 0.15, 96))
        P = _perm(lmax)
        S = np.eye(len(T)) + 2 * T
        errs.append((np.abs(T.T - P @ T @ P).max() / np.abs(T).max(),
                     np.abs(S.conj().T @ S - np.eye(len(T))).max()))
    rec, uni = zip(*errs)
    assert all(a > 10 * b for a, b in zip(rec, rec[1:])), rec
    assert all(a > 10 * b for a, b in zip(uni, uni[1:])), uni
    assert rec[-1] < 1e-9 and uni[-1] < 1e-9


def test_cylinder_classes_blocks_and_quadrature():
    lmax = 6
    T = ebcm_tmatrix(lmax, K, 3.48, cylinder_surface(0.12, 0.6, 96))
    idx = index_list(lmax)
    cls = np.array([(l + m + p) % 2 for p, l, m in idx])
    ms = np.array([m for p, l, m in idx])
    assert np.abs(T[cls[:, None] != cls[None, :]]).max() < 1e-12 * np.abs(T).max()
    assert np.abs(T[ms[:, None] != ms[None, :]]).max() == 0.0
    T2 = ebcm_tmatrix(lmax, K, 3.48, cylinder_surface(0.12, 0.6, 192))
    assert np.abs(T - T2).max() < 1e-12 * np.abs(T).max()
