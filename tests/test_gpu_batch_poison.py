"""A batch with a poisoned system: one subregion's right-hand side carries a
NaN, another cannot converge within max_iter.  The other systems must finish
with the same coefficients as when solved alone, the poisoned one must report
TM_ERR_NAN and the slow one TM_NOT_CONVERGED, and the call returns normally
(TM_NOT_CONVERGED) with every system's record."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import workloads as wl  # noqa: E402
from paper_2107_09879_amd import tmhip  # noqa: E402

pytestmark = pytest.mark.gpu
K = wl.K
DEV = torch.device("cuda", 0)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def packed_plane_wave(ctx, subs, nx, kh, po):
    """Incident coefficients of the full lattice gathered per subregion, in
    the packed [R][N_k][L] order of tm_solve_batched_a0."""
    full = host(ctx.plane_wave_rhs(kh, po))  # [R, N, L]
    parts = []
    for ox, oy, sx, sy in subs:
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        parts.append(full[:, (iy * nx + ix).ravel(), :].ravel())
    return np.concatenate(parts)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_poisoned_and_slow_systems_leave_the_batch(precision):
    print(f"[case] poisoned batch {precision}", flush=True)
    nx, ny, lmax = 40, 30, 3
    pos = wl.lattice_positions(nx, ny)
    radii = wl.lens_radii(nx, ny)
    kh, po = wl.incidences(["x"])
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device=DEV), wl.N_REL)
    # easy, poisoned (NaN in its block), easy, slow (needs thousands of steps)
    subs = [(0, 0, 12, 9), (3, 2, 8, 7), (30, 20, 10, 10), (5, 3, 20, 16)]
    a0 = packed_plane_wave(ctx, subs, nx, kh, po)
    sizes = [sx * sy * ctx.L for _, _, sx, sy in subs]
    a0[sizes[0] + 5] = np.nan
    a0d = torch.tensor(a0, dtype=torch.complex128, device=DEV)
    max_iter = 400
    sb, info = ctx.solve_batched_a0(subs, a0d, 1, use_graph=True, tol=1e-10, precision=precision,
                                    max_iter=max_iter, restart=50)
    st = [row[0]["status"] for row in info]
    print(f"  statuses {st}, iters {[row[0]['iters'] for row in info]}", flush=True)
    assert st == [0, -6, 0, 1], info
    assert info[3][0]["iters"] >= max_iter
    # the healthy systems match their lone solves
    for k in (0, 2):
        ox, oy, sx, sy = subs[k]
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * nx + ix).ravel()
        one = tmhip.Context(0)
        one.set_geometry(pos[idx], K, lmax)
        one.set_spheres(torch.tensor(radii[idx], dtype=torch.float64, device=DEV), wl.N_REL)
        s1, i1 = one.solve(one.plane_wave_rhs(kh, po), tol=1e-12)
        assert i1[0]["status"] == 0
        assert rel(host(sb[k]), host(s1)) < 1e-8
        one.close()
    # the context stays usable: a clean batch afterwards converges
    sb2, info2 = ctx.solve_batched([subs[0], subs[2]], kh, po, tol=1e-10, precision=precision)
    assert all(row[0]["status"] == 0 for row in info2), info2
    assert rel(host(sb2[0]), host(sb[0])) < 1e-8
    ctx.close()
