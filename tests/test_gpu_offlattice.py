"""Scatterers off the lattice (anywhere in the z = 0 plane): the on-the-fly
block matvec (translation blocks formed per pair from eq. "tran_coeff") and
the solve/readout built on it, against the CPU oracle's dense assembly
(blocks per ordered pair, the same construction the oracle always uses).
Tolerances as for the lattice path: FP64 operator 1e-12, complex64 2e-5,
solves at tol 1e-12 within 1e-10 of dense LU, readout 1e-11."""
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


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def jittered(nx, ny, amp, seed):
    """A perturbed lattice: every site moved in-plane by up to amp."""
    pos = wl.lattice_positions(nx, ny)
    pos[:, :2] += np.random.default_rng(seed).uniform(-amp, amp, (nx * ny, 2))
    return pos


def cluster(n, seed):
    """Random in-plane centres at least 0.5 apart."""
    g = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = g.uniform(0, 4.0, 2)
        if all(np.hypot(*(p - q)) > 0.5 for q in pts):
            pts.append(p)
    pos = np.zeros((n, 3))
    pos[:, :2] = pts
    return pos


CASES = [("jitter", 3), ("cluster", 2), ("jitter", 5), ("cluster", 1)]


def geometry(kind, lmax):
    if kind == "jitter":
        return jittered(7, 5, 0.05, lmax)
    return cluster(17, lmax)


@pytest.mark.parametrize("kind,lmax", CASES)
def test_offlattice_operator_and_solve(kind, lmax):
    print(f"[case] off-lattice {kind} lmax={lmax}", flush=True)
    pos = geometry(kind, lmax)
    N = len(pos)
    radii = np.random.default_rng(9).uniform(0.12, 0.2, N)
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    nx, ny, pitch = ctx.get_lattice()
    assert (nx, ny, pitch) == (N, 1, 0.0)
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device=DEV), wl.N_REL)
    L = ctx.L
    rng = np.random.default_rng(lmax)
    x = rng.normal(size=(2, N, L)) + 1j * rng.normal(size=(2, N, L))
    xd = torch.tensor(x, dtype=torch.complex128, device=DEV)
    A = oracle.coupling_dense(pos, K, lmax)
    ref = (A @ x.reshape(2, -1).T).T.reshape(2, N, L)
    refT = (A.T @ x.reshape(2, -1).T).T.reshape(2, N, L)
    assert rel(host(ctx.apply_operator(xd, "coupling", "fp64")), ref) < 1e-12
    assert rel(host(ctx.apply_operator(xd, "coupling", "mixed")), ref) < 2e-5
    assert rel(host(ctx.apply_operator(xd, "coupling_t", "fp64")), refT) < 1e-12
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    fa = host(ctx.apply_operator(xd, "adjoint", "mixed"))
    refa = x - (A.T @ (t[None] * x).reshape(2, -1).T).T.reshape(2, N, L)
    assert rel(fa, refa) < 2e-5
    kh, po = wl.incidences(["x", "p10"])
    a0 = ctx.plane_wave_rhs(kh, po)
    a0h = host(a0)
    for r in range(2):
        assert rel(a0h[r], oracle.plane_wave_coeffs(lmax, K, kh[r], po[r], pos)) < 1e-12
    B, _, T = oracle.system_dense(pos, K, lmax, t)
    s_ref = np.linalg.solve(B, T @ a0h.reshape(2, -1).T).T
    for prec in ("fp64", "mixed"):
        s, info = ctx.solve(a0, tol=1e-12, precision=prec)
        assert all(i["status"] == 0 for i in info), info
        assert rel(host(s).reshape(2, -1), s_ref) < 1e-10
    pts = np.array([[0.3, 0.2, 2.0], [1.5, 1.1, -0.9], [3.0, 2.0, 0.6]])
    E = host(ctx.near_field(s, torch.tensor(pts, device=DEV)))
    for r in range(2):
        assert rel(E[r], oracle.near_field(s_ref[r].reshape(N, L), pos, K, lmax, pts)) < 1e-11
    mu, info = ctx.adjoint_solve(xd[:1].contiguous(), tol=1e-12)
    assert rel(host(mu).reshape(-1), np.linalg.solve(B.T, x[0].ravel())) < 1e-10
    ctx.close()


def test_offlattice_rejects_lattice_only_calls_and_overlaps():
    pos = cluster(6, 1)
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, 2)
    ctx.set_spheres(torch.full((6,), 0.15, dtype=torch.float64, device=DEV), wl.N_REL)
    mu = torch.zeros(1, 6, ctx.L, dtype=torch.complex128, device=DEV)
    kh, po = wl.incidences(["x"])
    for call in (lambda: ctx.solve_batched([(0, 0, 2, 1)], kh, po),
                 lambda: ctx.grad_position(mu, mu),
                 lambda: ctx.apply_operator_noalloc(mu, torch.empty_like(mu)),
                 lambda: ctx.autotune(1, "mixed")):
        with pytest.raises(tmhip.TmError) as e:
            call()
        assert e.value.code == -3
    # two spheres whose centres are 0.5 apart cannot both have radius 0.3
    with pytest.raises(tmhip.TmError) as e:
        ctx.set_spheres(torch.full((6,), 0.3, dtype=torch.float64, device=DEV), wl.N_REL)
    assert e.value.code == -2
    pos2 = pos.copy()
    pos2[3] = pos2[1]
    with pytest.raises(tmhip.TmError) as e:
        ctx.set_geometry(pos2, K, 2)
    assert e.value.code == -2
    pos3 = pos.copy()
    pos3[2, 2] = 0.1
    with pytest.raises(tmhip.TmError) as e:
        ctx.set_geometry(pos3, K, 2)
    assert e.value.code == -3
    ctx.close()
