"""GPU position gradient (tm_grad_position, App. IV eq. "grad_pos_overlap")
against the CPU oracle's dense adjoint position gradient, whose analytic
derivative blocks and total are pinned on the CPU by central differences
(tests/test_oracle_position.py).  FP64 solves to 1e-13; the gradient is
compared within 1e-9 of its largest entry (solve error ~ cond * 1e-13)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from paper_2107_09879_amd import tmhip  # noqa: E402

pytestmark = pytest.mark.gpu
K = wl.K
DEV = torch.device("cuda", 0)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_position_gradient(ctx, kh, po, xd, parts=False):
    a0 = ctx.plane_wave_rhs(kh, po)
    s, info = ctx.solve(a0, tol=1e-13, precision="fp64")
    assert info[0]["status"] == 0
    z = np.array([torch.sum(ctx.detector_vector(xd, np.eye(3)[c]) * s[0]).item() for c in range(3)])
    Et = po[0] * np.exp(1j * K * kh[0] @ xd) + z
    w = np.conj(Et)
    v = ctx.detector_vector(xd, w)
    mu, info = ctx.adjoint_solve(v[None].contiguous(), tol=1e-13, precision="fp64")
    assert info[0]["status"] == 0
    g = host(ctx.grad_position(mu, s, a0, khat=kh, xd=xd, w=w[None]))[0]
    if not parts:
        return g
    gc = host(ctx.grad_position(mu, s))[0]
    gi = host(ctx.grad_position(mu, s, a0, khat=kh))[0] - gc
    gd = host(ctx.grad_position(mu, s, xd=xd, w=w[None]))[0] - gc
    return g, {"coupling": gc, "incident": gi, "detector": gd}


@pytest.mark.parametrize("nx,ny,lmax,inc", [(5, 4, 2, "x"), (4, 4, 3, "p10"), (4, 3, 4, "s10")])
def test_position_gradient_vs_oracle(nx, ny, lmax, inc):
    print(f"[case] position gradient {nx}x{ny} lmax={lmax} {inc}", flush=True)
    pos = wl.lattice_positions(nx, ny)
    radii = wl.uniform_radii(nx * ny, 0.12, 0.28, nx + 10 * lmax)
    kh, po = wl.incidence(inc)
    kh, po = np.atleast_2d(kh), np.atleast_2d(po)
    xd = np.array([0.55, 0.75, 2.3])
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device=DEV), wl.N_REL)
    g, parts = gpu_position_gradient(ctx, kh, po, xd, parts=True)
    O, gref, _, _, pref = oracle.objective_and_position_gradient_dense(
        pos, K, lmax, radii, wl.N_REL, kh[0], po[0], xd, parts=True)
    scale = np.abs(gref[:, :2]).max()
    for name in ("coupling", "incident", "detector"):
        err = np.abs(parts[name] - pref[name][:, :2]).max() / scale
        print(f"  {name}: max err {err:.2e} (part max {np.abs(pref[name][:, :2]).max():.3e})", flush=True)
        assert err < 1e-9, name
    assert np.abs(g - gref[:, :2]).max() < 1e-9 * scale
    ctx.close()


def test_position_gradient_argument_checks():
    ctx = tmhip.Context(0)
    ctx.set_geometry(wl.lattice_positions(3, 2), K, 2)
    ctx.set_spheres(torch.full((6,), 0.2, dtype=torch.float64, device=DEV), wl.N_REL)
    mu = torch.zeros(1, 6, ctx.L, dtype=torch.complex128, device=DEV)
    with pytest.raises(ValueError):
        ctx.grad_position(mu, mu, khat=[[0, 0, 1.0]])  # khat without a0
    with pytest.raises(ValueError):
        ctx.grad_position(mu, mu, xd=[0, 0, 2.0])  # xd without w
    with pytest.raises(tmhip.TmError) as e:
        ctx.grad_position(mu, mu, mu, khat=[[np.nan, 0, 1.0]])
    assert e.value.code == -6
    ctx.close()
