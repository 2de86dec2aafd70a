"""Jinc-source incident coefficients on the GPU (tm_jinc_rhs,
tm_jinc_rhs_batched) against the CPU oracle's Gamma-route expansion (pinned
on the CPU against direct 2-D quadrature, the source-plane closed form and
the pointwise field), and the batched solve driven by jinc groups
(tm_solve_batched_a0) against one-subregion solves.  FP64 throughout: the
coefficients agree to rounding (1e-11 relative) at equal polar nodes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import workloads as wl  # noqa: E402
from oracle.jinc import jinc_coeffs  # noqa: E402
from paper_2107_09879_amd import tmhip  # noqa: E402

pytestmark = pytest.mark.gpu
K = wl.K
DEV = torch.device("cuda", 0)

SOURCES = [(1.5, 1.2, -1.0, 1.0, 0.3j), (-2.0, 5.0, -3.0, 0.2 - 0.1j, 0.8), (2.7, 0.9, -0.4, 0.0, 1.0)]


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def ctx_for(nx, ny, lmax, seed=0):
    ctx = tmhip.Context(0)
    ctx.set_geometry(wl.lattice_positions(nx, ny), K, lmax)
    r = wl.uniform_radii(nx * ny, 0.15, 0.25, seed)
    ctx.set_spheres(torch.tensor(r, dtype=torch.float64, device=DEV), wl.N_REL)
    return ctx, r


@pytest.mark.parametrize("lmax", [3, 5])
def test_jinc_rhs_matches_oracle(lmax):
    print(f"[case] jinc rhs lmax={lmax}", flush=True)
    nx, ny = 7, 6
    ctx, _ = ctx_for(nx, ny, lmax)
    pos = wl.lattice_positions(nx, ny)
    a = host(ctx.jinc_rhs(SOURCES, n_beta=96))
    for r, src in enumerate(SOURCES):
        ref = jinc_coeffs(lmax, K, src, pos, n_beta=96)
        assert rel(a[r], ref) < 1e-11, r
    # automatic polar nodes against a converged oracle
    auto = host(ctx.jinc_rhs(SOURCES[:1]))[0]
    ref = jinc_coeffs(lmax, K, SOURCES[0], pos, n_beta=300)
    assert rel(auto, ref) < 1e-10
    ctx.close()


def test_jinc_groups_drive_the_batched_solve():
    print("[case] jinc batched", flush=True)
    nx, ny, lmax = 12, 10, 3
    ctx, radii = ctx_for(nx, ny, lmax, seed=3)
    pos = wl.lattice_positions(nx, ny)
    subs = [(0, 0, 7, 6), (3, 2, 9, 8)]
    groups = [[[SOURCES[0], SOURCES[2]]], [[SOURCES[1]]]]
    a0p = ctx.jinc_rhs_batched(subs, groups, n_beta=96)
    # packed coefficients equal the oracle's group sums on each subregion
    off = 0
    for (ox, oy, sx, sy), grp in zip(subs, groups):
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * nx + ix).ravel()
        ref = sum(jinc_coeffs(lmax, K, s, pos[idx], n_beta=96) for s in grp[0])
        n = sx * sy * ctx.L
        assert rel(host(a0p[off:off + n]).reshape(sx * sy, ctx.L), ref) < 1e-11
        off += n
    sb, info = ctx.solve_batched_a0(subs, a0p, 1, use_graph=True, tol=1e-11, precision="mixed")
    assert all(i["status"] == 0 for row in info for i in row), info
    for k, ((ox, oy, sx, sy), grp) in enumerate(zip(subs, groups)):
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * nx + ix).ravel()
        one = tmhip.Context(0)
        one.set_geometry(pos[idx], K, lmax)
        one.set_spheres(torch.tensor(radii[idx], dtype=torch.float64, device=DEV), wl.N_REL)
        a0 = one.jinc_rhs(grp[0], n_beta=96).sum(0, keepdim=True).contiguous()
        s1, i1 = one.solve(a0, tol=1e-12)
        assert i1[0]["status"] == 0
        assert rel(host(sb[k]), host(s1)) < 1e-9
        one.close()
    ctx.close()


def test_jinc_argument_checks():
    ctx, _ = ctx_for(3, 3, 2)
    with pytest.raises(tmhip.TmError) as e:
        ctx.jinc_rhs([(0.0, 0.0, np.nan, 1.0, 0.0)])
    assert e.value.code == -6
    with pytest.raises(tmhip.TmError) as e:
        ctx.jinc_rhs_batched([(0, 0, 5, 2)], [[[SOURCES[0]]]])  # box outside the 3x3 lattice
    assert e.value.code == -1
    ctx.close()
