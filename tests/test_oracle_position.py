"""Pins of the oracle's position sensitivities (App. IV, eq. "grad_pos_overlap"),
independent of the HIP path: the analytic translation-block gradient against
central differences of the blocks, the detector-vector gradient against
central differences of the detector vectors, and the whole adjoint position
gradient against central differences of the objective (dense re-solves with
one scatterer moved off its site, in x, y and z)."""
import numpy as np
import pytest

import workloads as wl
from oracle.position import (detector_vector_gradient, objective_and_position_gradient_dense,
                             objective_dense, translation_gradient)
from oracle.solver import detector_vectors
from oracle.translation import Translation

K = wl.K


def fd4(f, x, h):
    """Fourth-order central difference of f at x along each axis -> [3, ...]."""
    out = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        out.append((-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * h))
    return np.stack(out)


@pytest.mark.parametrize("lmax,lmax_t", [(2, 2), (3, 3), (6, 6), (4, 1)])
def test_translation_gradient_matches_differences(lmax, lmax_t):
    tr = Translation(K, lmax, lmax_t)
    for d in ([0.6, 0.0, 0.0], [1.2, -1.8, 0.0], [0.43, -0.31, 0.22], [0.1, 0.05, 0.9],
              [-0.6, 0.6, -0.3]):
        d = np.array(d)
        G = translation_gradient(tr, d)
        Gfd = fd4(lambda x: tr.block(x), d, 1e-4)
        assert np.abs(G - Gfd).max() <= 1e-8 * np.abs(G).max(), d


def test_detector_vector_gradient_matches_differences():
    lmax = 3
    pos = wl.lattice_positions(3, 2)
    xd = np.array([0.7, 0.4, 2.5])
    dv = detector_vector_gradient(pos, K, lmax, xd)  # [c, i, n, a]
    for i in (0, 4):
        def f(xi):
            p = pos.copy()
            p[i] = xi
            return detector_vectors(p, K, lmax, xd)[:, i, :]  # [c, n]
        ref = fd4(f, pos[i], 1e-4)  # [a, c, n]
        assert np.abs(np.transpose(dv[:, i], (2, 0, 1)) - ref).max() <= 1e-10 * np.abs(ref).max()


def test_regular_waves_at_their_centre():
    """R Phi_v(0): the M-type l = 1 waves vanish there (j_1(0) = 0) and the
    N-type ones are the constants of the l = 1 limit j_1(x)/x -> 1/3,
    (x j_1)'/x -> 2/3 of the basis definition."""
    from oracle.position import regular_at_origin

    R0 = regular_at_origin(K)
    a, b = np.sqrt(0.75) / 3, np.sqrt(1.5) / 3
    ref = np.zeros((6, 3), dtype=complex)
    ref[3] = a * np.array([1, -1j, 0])
    ref[4] = b * np.array([0, 0, 1])
    ref[5] = a * np.array([1, 1j, 0])
    assert np.abs(R0 - ref).max() < 1e-12


@pytest.mark.parametrize("khat,pol", [((0, 0, 1.0), (1.0, 0, 0)),
                                      ((np.sin(0.3), 0, np.cos(0.3)), (np.cos(0.3), 0, -np.sin(0.3)))])
def test_position_gradient_matches_objective_differences(khat, pol):
    nx, ny, lmax = 3, 3, 2
    pos = wl.lattice_positions(nx, ny)
    radii = wl.uniform_radii(nx * ny, 0.12, 0.2, 3)
    xd = np.array([0.5, 0.8, 1.7])
    khat, pol = np.array(khat), np.array(pol)
    O, g, _, _ = objective_and_position_gradient_dense(pos, K, lmax, radii, wl.N_REL, khat, pol, xd)
    h = 1e-5
    for i in (0, 4, 7):
        for a in range(3):
            def Oat(dx):
                p = pos.copy()
                p[i, a] += dx
                return objective_dense(p, K, lmax, radii, wl.N_REL, khat, pol, xd)
            fd = (-Oat(2 * h) + 8 * Oat(h) - 8 * Oat(-h) + Oat(-2 * h)) / (12 * h)
            assert abs(fd - g[i, a]) <= 1e-7 * np.abs(g).max(), (i, a, fd, g[i, a])
