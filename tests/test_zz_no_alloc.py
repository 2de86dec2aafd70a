"""The allocation-free operator entry point (tm_apply_operator_noalloc)
against tm_apply_operator, through the C ABI, on consecutive calls that
shrink the input (the shared scratch array keeps the earlier call's data)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import workloads as wl  # noqa: E402
from paper_2107_09879_amd import tmhip  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
# FP64: same arithmetic, different summation order; complex64: FP32
# accumulation in a different work split (each side within 2e-5 of FP64)
TOL = {"fp64": 1e-12, "mixed": 4e-5}


def rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def make_ctx(nx, ny, lmax, seed):
    ctx = tmhip.Context(0)
    ctx.set_geometry(wl.lattice_positions(nx, ny), wl.K, lmax)
    r = wl.uniform_radii(nx * ny, 0.15, 0.25, seed)
    ctx.set_spheres(torch.tensor(r, dtype=torch.float64, device=DEV), wl.N_REL)
    return ctx


def rand(R, N, L, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(R, N, L, 2, generator=g, dtype=torch.float64)
    return torch.view_as_complex(x).contiguous().to(DEV)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_operator_matches_apply_operator(precision):
    big = make_ctx(37, 21, 3, 11)   # 2 row bands of regular tiles + 5 wide-tile rows
    small = make_ctx(9, 5, 2, 12)
    try:
        # the transposed tables come from one ordinary call
        big.apply_operator(rand(1, big.n, big.L, 0), "coupling_t", precision)
        small.apply_operator(rand(1, small.n, small.L, 0), "adjoint", precision)
        cases = [(big, 3), (big, 1), (small, 2), (small, 1)]
        for op in ("forward", "coupling", "adjoint", "coupling_t"):
            for i, (ctx, R) in enumerate(cases):
                x = rand(R, ctx.n, ctx.L, 100 + i)
                ref = ctx.apply_operator(x, op, precision)
                out = torch.full_like(x, complex(np.nan, np.nan))
                got = ctx.apply_operator_noalloc(x, out, op, precision)
                torch.cuda.synchronize()
                assert got.data_ptr() == out.data_ptr()
                assert torch.isfinite(torch.view_as_real(got)).all(), (op, i)
                e = rel(got, ref)
                print(f"noalloc {precision} {op} case {i} (n={ctx.n}, R={R}): rel {e:.2e}", flush=True)
                assert e < TOL[precision], (op, i, e)
    finally:
        big.close()
        small.close()


def test_noalloc_operator_rejects_what_does_not_fit():
    ctx = make_ctx(40, 40, 3, 13)
    try:
        # 2 packed c128 vectors of 100 x 1600 x 32 slots = 164 MB > 128 MiB
        x = torch.zeros(100, ctx.n, ctx.L, dtype=torch.complex128, device=DEV)
        with pytest.raises(tmhip.TmError) as ei:
            ctx.apply_operator_noalloc(x, torch.empty_like(x), "forward", "fp64")
        assert ei.value.code == -1
        # transposed ops before the transposed tables exist: a state error
        x1 = rand(1, ctx.n, ctx.L, 5)
        with pytest.raises(tmhip.TmError) as ei:
            ctx.apply_operator_noalloc(x1, torch.empty_like(x1), "coupling_t", "fp64")
        assert ei.value.code == -7
        # a fitting call on the same context still works afterwards
        ref = ctx.apply_operator(x1, "forward", "fp64")
        got = ctx.apply_operator_noalloc(x1, torch.empty_like(x1), "forward", "fp64")
        torch.cuda.synchronize()
        assert rel(got, ref) < TOL["fp64"]
    finally:
        ctx.close()
