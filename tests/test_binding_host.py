"""Argument checks of the Python binding that run before any pointer reaches
the library (no GPU needed): mis-shaped device arrays and host arrays raise
ValueError, wrong types raise TypeError."""
import numpy as np
import pytest
import torch

from paper_2107_09879_amd import tmhip

C128, F64 = torch.complex128, torch.float64


@pytest.fixture
def ctx():
    # a context object without a library handle: every call below must fail
    # in the binding's checks, before it would reach the C entry point
    c = tmhip.Context.__new__(tmhip.Context)
    c.n, c.L, c.lmax, c.k, c.h, c.lib = 12, 16, 2, 2 * np.pi, None, None
    c.device = torch.device("cuda", 0)
    return c


def z(*shape, dtype=C128):
    return torch.zeros(*shape, dtype=dtype)


@pytest.mark.parametrize("call", [
    lambda c: c.solve(z(11, 16)),
    lambda c: c.solve(z(2, 12, 15)),
    lambda c: c.solve(z(1, 2, 12, 16)),
    lambda c: c.adjoint_solve(z(12, 17)),
    lambda c: c.apply_operator(z(3, 13, 16)),
    lambda c: c.set_spheres(z(13, dtype=F64), 2.0),
    lambda c: c.set_tmatrix_diag(z(12, 15)),
    lambda c: c.set_tmatrix_dense(z(12, 16, 15)),
    lambda c: c.near_field(z(12, 16), z(5, 2, dtype=F64)),
    lambda c: c.near_field(z(11, 16), z(5, 3, dtype=F64)),
    lambda c: c.far_field(z(12, 16), z(4, dtype=F64)),
    lambda c: c.near_field_adjoint(z(5, 3, dtype=F64), z(2, 6, 3)),
    lambda c: c.grad_radius(z(12, 16), z(12, 16), z(12, 14)),
    lambda c: c.detector_vector([0.0, 0.0], [1, 0, 0]),
    lambda c: c.detector_vector([0.0, 0.0, 1.0], [1, 0]),
    lambda c: c.plane_wave_rhs([[0, 0, 1.0], [1.0, 0, 0]], [[1.0, 0, 0]]),
    lambda c: c.plane_wave_rhs([0, 0, 1.0, 0], [1.0, 0, 0]),
    lambda c: c.set_geometry(np.zeros((4, 2)), 1.0, 2),
])
def test_misshaped_arguments_raise_value_error(ctx, call):
    with pytest.raises(ValueError):
        call(ctx)


def test_x0_must_match_the_right_hand_side(ctx):
    with pytest.raises(ValueError):
        ctx.solve(z(2, 12, 16), x0=z(1, 12, 16))


def test_wrong_dtype_or_host_tensor_raise_type_error(ctx):
    with pytest.raises(TypeError):
        ctx.solve(z(12, 16, dtype=torch.complex64))
    with pytest.raises(TypeError):
        ctx.solve(z(12, 16))  # right shape, but host memory
    with pytest.raises(TypeError):
        ctx.near_field(np.zeros((12, 16), complex), z(5, 3, dtype=F64))
