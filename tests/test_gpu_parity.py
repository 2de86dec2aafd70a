"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances (normwise relative unless stated):
  FP64 operator / tables ......... 1e-12  (sum of <= N*225 terms, rounding ~1e-16 each)
  complex64 operator ............. 2e-5   (FP32 table + input rounding ~6e-8, sums of
                                            ~1e4 terms with FP32 accumulation)
  FP64 solve at tol 1e-12 ........ 1e-10  (error <= cond(B) * residual, cond ~ 10)
  mixed solve refined to 1e-12 ... 1e-10
  mixed solve stopped at 1e-6 .... 1e-5
  readout / Mie / RHS (FP64) ..... 1e-11
"""
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
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def to_dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make_ctx(nx, ny, lmax, radii=None, seed=0, lo=0.15, hi=0.25):
    pos = wl.lattice_positions(nx, ny)
    if radii is None:
        radii = wl.uniform_radii(nx * ny, lo, hi, seed)
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    return ctx, pos, radii


def rand_vec(rng, R, N, L):
    return rng.normal(size=(R, N, L)) + 1j * rng.normal(size=(R, N, L))


# ----------------------------------------------------------------- operator
SHAPES = [(1, 1, 2), (5, 4, 2), (20, 18, 3), (37, 5, 3), (1, 9, 2), (33, 33, 3)]


@pytest.mark.parametrize("nx,ny,lmax", SHAPES)
def test_coupling_operator_fp64_and_c64(nx, ny, lmax):
    print(f"[case] coupling nx={nx} ny={ny} lmax={lmax}", flush=True)
    rng = np.random.default_rng(nx * 100 + ny)
    ctx, pos, radii = make_ctx(nx, ny, lmax)
    L = oracle.n_coeffs(lmax)
    x = rand_vec(rng, 2, nx * ny, L)
    lc = oracle.LatticeCoupling(nx, ny, wl.PITCH, K, lmax)
    ref = np.stack([lc.apply(x[r]) for r in range(2)])
    refT = np.stack([lc.apply(x[r], transpose=True) for r in range(2)])
    xd = to_dev(x)
    if nx * ny == 1:
        assert np.abs(host(ctx.apply_operator(xd, "coupling"))).max() == 0.0
        return
    y64 = host(ctx.apply_operator(xd, "coupling", "fp64"))
    y32 = host(ctx.apply_operator(xd, "coupling", "mixed"))
    assert rel(y64, ref) < 1e-12
    assert rel(y32, ref) < 2e-5
    yT = host(ctx.apply_operator(xd, "coupling_t", "fp64"))
    assert rel(yT, refT) < 1e-12
    # forward and adjoint operators: x - t A x, x - A^T (t x)
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    f = host(ctx.apply_operator(xd, "forward", "fp64"))
    assert rel(f, x - t[None] * ref) < 1e-12
    fa = host(ctx.apply_operator(xd, "adjoint", "mixed"))
    refa = np.stack([x[r] - lc.apply(t * x[r], transpose=True) for r in range(2)])
    assert rel(fa, refa) < 2e-5
    ctx.close()


def test_operator_is_deterministic():
    rng = np.random.default_rng(3)
    ctx, _, _ = make_ctx(24, 24, 3)
    xd = to_dev(rand_vec(rng, 1, 576, 30))
    a = host(ctx.apply_operator(xd, "forward", "mixed"))
    b = host(ctx.apply_operator(xd, "forward", "mixed"))
    assert np.array_equal(a, b)
    ctx.close()


# ----------------------------------------------------------------- set-up kernels
def test_lds_matvec_chains_on_a_user_stream_without_host_syncs():
    """The remainder-row (wide-tile) launch runs on the context's second
    stream.  It must follow earlier work on the caller's stream and precede
    later work there: two chained products on a private stream, with every
    LDS variant and a lattice whose height leaves two remainder rows, are
    synchronised only at the end."""
    print("[case] lds chain on a user stream", flush=True)
    nx, ny, lmax = 20, 18, 3
    rng = np.random.default_rng(2018)
    L = oracle.n_coeffs(lmax)
    x = rand_vec(rng, 1, nx * ny, L)
    lc = oracle.LatticeCoupling(nx, ny, wl.PITCH, K, lmax)
    ref1 = lc.apply(x[0])
    ref2 = lc.apply(ref1)
    # a second right-hand side: a call with R = 2 followed at once by one
    # with R = 1 re-cuts the work split while the first may still run
    xb = np.concatenate([x, rand_vec(rng, 1, nx * ny, L)])
    refb = lc.apply(xb[1])
    st = torch.cuda.Stream(device=DEV)
    out, outb = {}, {}
    with torch.cuda.stream(st):
        ctx, pos, radii = make_ctx(nx, ny, lmax)
        xd = to_dev(x)
        xbd = to_dev(xb)
        for prec in ("fp64", "mixed"):
            for v in (8, 9, 10):
                ctx.set_matvec_config(prec, v, 0)
                y1 = ctx.apply_operator(xd, "coupling", prec)
                y2 = ctx.apply_operator(y1, "coupling", prec)
                out[prec, v] = (y1, y2)
            yb2 = ctx.apply_operator(xbd, "coupling", prec)
            yb1 = ctx.apply_operator(xd, "coupling", prec)
            outb[prec] = (yb2, yb1)
    st.synchronize()
    for (prec, v), (y1, y2) in out.items():
        tol = 1e-12 if prec == "fp64" else 2e-5
        assert rel(y1.cpu().numpy()[0], ref1) < tol, (prec, v)
        assert rel(y2.cpu().numpy()[0], ref2) < 2 * tol, (prec, v)
    for prec, (yb2, yb1) in outb.items():
        tol = 1e-12 if prec == "fp64" else 2e-5
        assert rel(yb2.cpu().numpy()[0], ref1) < tol, prec
        assert rel(yb2.cpu().numpy()[1], refb) < tol, prec
        assert rel(yb1.cpu().numpy()[0], ref1) < tol, prec
    ctx.close()


def test_mie_and_plane_wave_match_oracle():
    ctx, pos, radii = make_ctx(7, 6, 3, lo=0.12, hi=0.28, seed=5)
    t, dt = ctx.get_tmatrix_diag()
    tr, dtr = oracle.mie_tmatrix_diag_many(3, K, radii, wl.N_REL)
    assert rel(host(t), tr) < 1e-12
    assert rel(host(dt), dtr) < 1e-11
    kh, po = wl.incidences(["x", "y", "p10", "s10"])
    a0 = host(ctx.plane_wave_rhs(kh, po))
    for r in range(4):
        assert rel(a0[r], oracle.plane_wave_coeffs(3, K, kh[r], po[r], pos)) < 1e-12
    ctx.close()


def test_lossy_sphere_mie():
    pos = wl.lattice_positions(3, 1)
    radii = np.array([0.1, 0.2, 0.25])
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, 3)
    m = 1.5 + 0.3j
    ctx.set_spheres(to_dev(radii, torch.float64), m)
    t, dt = ctx.get_tmatrix_diag()
    tr, dtr = oracle.mie_tmatrix_diag_many(3, K, radii, m)
    assert rel(host(t), tr) < 1e-12 and rel(host(dt), dtr) < 1e-11
    ctx.close()


@pytest.mark.parametrize("lmax,radius,m", [(1, 0.05, 2.0), (3, 0.25, 2.0), (2, 0.3, 1.5 + 0.3j)])
def test_tm_mie_single_sphere(lmax, radius, m):
    t, d = tmhip.mie(lmax, K, radius, m)
    for l in range(1, lmax + 1):
        a, b, da, db = oracle.mie_ab(l, K * radius, m)
        assert abs(t[0, l - 1] + b) <= 1e-12 * abs(b) + 1e-300
        assert abs(t[1, l - 1] + a) <= 1e-12 * abs(a) + 1e-300
        assert abs(d[0, l - 1] + K * db) <= 1e-11 * abs(K * db) + 1e-300
        assert abs(d[1, l - 1] + K * da) <= 1e-11 * abs(K * da) + 1e-300
    with pytest.raises(tmhip.TmError):
        tmhip.mie(7, K, radius, m)
    with pytest.raises(tmhip.TmError):
        tmhip.mie(lmax, K, -radius, m)


def _dense_t(radii, lmax, seed):
    """Mie diagonal plus a seeded full perturbation (0.1 of the largest |t|
    per sphere): a T that mixes every (p, l, m) of a scatterer."""
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    g = np.random.default_rng(seed)
    N, L = t.shape
    E = g.standard_normal((N, L, L)) + 1j * g.standard_normal((N, L, L))
    E *= (0.1 * np.abs(t).max(1) / np.sqrt(2 * L))[:, None, None]
    return np.stack([np.diag(t[i]) for i in range(N)]) + E


@pytest.mark.parametrize("nx,ny,lmax", [(4, 3, 2), (6, 5, 3)])
def test_dense_tmatrix_operator_and_solve(nx, ny, lmax):
    ctx, pos, radii = make_ctx(nx, ny, lmax, seed=17)
    Td = _dense_t(radii, lmax, 5)
    ctx.set_tmatrix_dense(to_dev(Td))
    B, A, T = oracle.system_dense(pos, K, lmax, Td)
    g = np.random.default_rng(2)
    N, L = nx * ny, ctx.L
    x = g.standard_normal((2, N, L)) + 1j * g.standard_normal((2, N, L))
    xf = x.reshape(2, -1)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        y = host(ctx.apply_operator(to_dev(x), "forward", prec)).reshape(2, -1)
        assert rel(y, xf - (T @ (A @ xf.T)).T) < tol
        y = host(ctx.apply_operator(to_dev(x), "adjoint", prec)).reshape(2, -1)
        assert rel(y, xf - (A.T @ (T.T @ xf.T)).T) < tol
    kh, po = wl.incidences(["x", "p10"])
    a0 = ctx.plane_wave_rhs(kh, po)
    s_ref = np.linalg.solve(B, T @ host(a0).reshape(2, -1).T).T
    for prec in ("fp64", "mixed"):
        s, info = ctx.solve(a0, tol=1e-12, precision=prec)
        assert all(i["status"] == 0 for i in info)
        assert rel(host(s).reshape(2, -1), s_ref) < 1e-10
    w = to_dev(x)
    mu, _ = ctx.adjoint_solve(w, tol=1e-12)
    assert rel(host(mu).reshape(2, -1), np.linalg.solve(B.T, xf.T).T) < 1e-10
    # what a dense T does not support
    for call in (lambda: ctx.get_tmatrix_diag(), lambda: ctx.grad_radius(mu, s, a0),
                 lambda: ctx.solve_batched([(0, 0, 2, 2)], kh, po)):
        with pytest.raises(tmhip.TmError) as e:
            call()
        assert e.value.code == -7
    ctx.close()


@pytest.mark.parametrize("lmax", [3, 6])
def test_dense_tmatrix_mblock_structure(lmax):
    """A dense T that is zero between different azimuthal orders m (a
    scatterer symmetric about the z axis, like the null-field cylinders) is
    applied from its m-blocks alone; the same T with one entry between
    different m takes the general apply.  Both against the oracle's dense
    operator, forward and adjoint, and a mixed solve at tol 1e-12 through the
    oracle's residual (and dense LU at lmax 3; at lmax 6 cond(B) is ~6e3, so
    the solution error is only bounded by cond(B) x 1e-12).  The within-m
    perturbation scales as sqrt(|t_n t_n'|), which keeps B well conditioned."""
    print(f"[case] dense T m-blocks lmax={lmax}", flush=True)
    nx, ny = 5, 3
    ctx, pos, radii = make_ctx(nx, ny, lmax, seed=21)
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    N, L = t.shape
    g = np.random.default_rng(8)
    E = g.standard_normal((N, L, L)) + 1j * g.standard_normal((N, L, L))
    a = np.sqrt(np.abs(t))
    E *= 0.3 * a[:, :, None] * a[:, None, :]
    m_of = np.array([m for (_, _, m) in oracle.index_list(lmax)])
    Tb = (np.stack([np.diag(t[i]) for i in range(N)]) + E) * (m_of[:, None] == m_of[None, :])[None]
    Tg = Tb.copy()
    Tg[4, 0, 1] = 1e-3 * np.abs(Tb[4]).max()  # (p,l,m) = (0,1,-1) <- (0,1,0)
    x = g.standard_normal((2, N, L)) + 1j * g.standard_normal((2, N, L))
    xf = x.reshape(2, -1)
    kh, po = wl.incidences(["x", "p10"])
    for name, Td in (("m-blocks", Tb), ("general", Tg)):
        ctx.set_tmatrix_dense(to_dev(Td))
        B, A, T = oracle.system_dense(pos, K, lmax, Td)
        for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
            y = host(ctx.apply_operator(to_dev(x), "forward", prec)).reshape(2, -1)
            assert rel(y, xf - (T @ (A @ xf.T)).T) < tol
            y = host(ctx.apply_operator(to_dev(x), "adjoint", prec)).reshape(2, -1)
            assert rel(y, xf - (A.T @ (T.T @ xf.T)).T) < tol
        a0 = ctx.plane_wave_rhs(kh, po)
        b = T @ host(a0).reshape(2, -1).T
        s, info = ctx.solve(a0, tol=1e-12, precision="mixed", max_iter=4000)
        sh = host(s).reshape(2, -1).T
        res = np.linalg.norm(B @ sh - b) / np.linalg.norm(b)
        print(f"  {name}: iters {[i['iters'] for i in info]}, oracle residual {res:.2e}", flush=True)
        assert all(i["status"] == 0 for i in info), info
        assert res < 1e-11
        if lmax == 3:
            assert rel(sh, np.linalg.solve(B, b)) < 1e-10
    ctx.close()


def test_dense_tmatrix_equal_to_diagonal():
    ctx, pos, radii = make_ctx(5, 4, 3, seed=9)
    kh, po = wl.incidences(["y"])
    a0 = ctx.plane_wave_rhs(kh, po)
    s_diag, _ = ctx.solve(a0, tol=1e-13)
    t, _ = ctx.get_tmatrix_diag()
    ctx.set_tmatrix_dense(torch.diag_embed(t).contiguous())
    s_dense, _ = ctx.solve(a0, tol=1e-13)
    assert rel(host(s_dense), host(s_diag)) < 1e-12
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)  # back to the diagonal path
    s_back, _ = ctx.solve(a0, tol=1e-13)
    assert rel(host(s_back), host(s_diag)) < 1e-13
    ctx.close()


# ----------------------------------------------------------------- solve
def _c1():
    pos, radii, kh, po, cfg = wl.config_inputs("c1")
    n = cfg["nx"]
    ctx, _, _ = make_ctx(n, n, cfg["lmax"], radii=radii)
    return ctx, pos, radii, kh, po, cfg


def test_solve_c1_fp64_and_mixed_vs_dense_lu():
    ctx, pos, radii, kh, po, cfg = _c1()
    lmax = cfg["lmax"]
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    a0r = oracle.plane_wave_coeffs(lmax, K, kh[0], po[0], pos)
    s_ref = oracle.solve_dense(pos, K, lmax, t, a0r)
    a0 = ctx.plane_wave_rhs(kh, po)
    s64, info = ctx.solve(a0, tol=1e-12, precision="fp64")
    assert info[0]["status"] == 0 and info[0]["rel_residual"] <= 1e-12
    assert rel(host(s64)[0], s_ref) < 1e-10
    smx, info = ctx.solve(a0, tol=1e-12, precision="mixed", inner_tol=1e-4)
    assert info[0]["status"] == 0 and info[0]["matvecs_lowp"] > 0
    assert rel(host(smx)[0], s_ref) < 1e-10
    sf, info = ctx.solve(a0, tol=1e-6, precision="mixed", inner_tol=1e-4)
    assert rel(host(sf)[0], s_ref) < 1e-5
    # far field and optical theorem through the GPU path
    dirs = np.array([[0, 0, 1.0], [0.6, 0, 0.8], [0, -0.6, -0.8]])
    F = host(ctx.far_field(s64, to_dev(dirs, torch.float64)))[0]
    Fr = oracle.far_field(s_ref, pos, K, lmax, dirs)
    assert rel(F, Fr) < 1e-10
    ctx.close()


def test_solve_multi_rhs_and_x0_and_adjoint():
    rng = np.random.default_rng(8)
    ctx, pos, radii = make_ctx(6, 5, 3, seed=8)
    t, _ = oracle.mie_tmatrix_diag_many(3, K, radii, wl.N_REL)
    B, A, T = oracle.system_dense(pos, K, 3, t)
    kh, po = wl.incidences(["x", "p10"])
    a0 = ctx.plane_wave_rhs(kh, po)
    s, info = ctx.solve(a0, tol=1e-12)
    a0h = host(a0)
    for r in range(2):
        ref = np.linalg.solve(B, (t * a0h[r]).ravel()).reshape(30, 30)
        assert rel(host(s)[r], ref) < 1e-10
    # warm start from the answer converges immediately
    s2, info2 = ctx.solve(a0, x0=s, tol=1e-10)
    assert info2[0]["iters"] == 0
    # adjoint (I - A^T T) mu = v
    v = rand_vec(rng, 1, 30, 30)
    mu, info = ctx.adjoint_solve(to_dev(v), tol=1e-12)
    Badj = np.eye(900) - A.T @ T
    assert rel(host(mu)[0], np.linalg.solve(Badj, v.ravel()).reshape(30, 30)) < 1e-10
    ctx.close()


# ----------------------------------------------------------------- readout + adjoint
@pytest.mark.parametrize("R,lmax", [(2, 3), (1, 2), (3, 3), (5, 1)])
def test_near_field_and_detector(R, lmax):
    rng = np.random.default_rng(4)
    ctx, pos, radii = make_ctx(6, 4, lmax)
    L = oracle.n_coeffs(lmax)
    s = rand_vec(rng, R, 24, L) * 0.1
    pts = np.array([[0.3, 0.3, 5.0], [1.0, -2.0, 0.7], [1.5, 0.9, -3.0], [0.6, 0.6, 0.45],
                    [0.0, 0.0, 0.5], [40.0, 30.0, 2.0]])
    E64 = host(ctx.near_field(to_dev(s), to_dev(pts, torch.float64), "fp64"))
    E32 = host(ctx.near_field(to_dev(s), to_dev(pts, torch.float64), "mixed"))
    for r in range(R):
        ref = oracle.near_field(s[r], pos, K, lmax, pts)
        assert rel(E64[r], ref) < 1e-11
        assert rel(E32[r], ref) < 1e-4
    xd = np.array([0.9, 1.1, 4.0])
    w = np.array([1.0 + 0.5j, -0.3j, 0.2])
    v = host(ctx.detector_vector(xd, w))
    vr = np.einsum('c,cil->il', w, oracle.detector_vectors(pos, K, lmax, xd))
    assert rel(v, vr) < 1e-12
    ctx.close()


def test_gradient_vs_oracle_adjoint():
    nx, ny, lmax = 4, 3, 2
    pos = wl.lattice_positions(nx, ny)
    radii = wl.uniform_radii(nx * ny, 0.12, 0.28, 21)
    kh, po = wl.incidence("x")
    xd = np.array([0.9, 0.6, 3.0])
    O, g_ref, s_ref, mu_ref = oracle.objective_and_gradient_dense(pos, K, lmax, radii, wl.N_REL,
                                                                  kh, po, xd)
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    a0 = ctx.plane_wave_rhs(kh, po)
    s, _ = ctx.solve(a0, tol=1e-13)
    vc = [ctx.detector_vector(xd, np.eye(3)[c]) for c in range(3)]
    z = np.array([np.sum(host(vc[c]) * host(s)[0]) for c in range(3)])
    Et = po * np.exp(1j * K * kh @ xd) + z
    w = ctx.detector_vector(xd, np.conj(Et))
    mu, _ = ctx.adjoint_solve(w[None].contiguous(), tol=1e-13)
    g = host(ctx.grad_radius(mu, s, a0))[0]
    assert rel(g, g_ref) < 1e-9
    ctx.close()


# ----------------------------------------------------------------- errors
def test_error_paths():
    ctx = tmhip.Context(0)
    pos = wl.lattice_positions(4, 4)
    # a centre off the z = 0 plane is outside the method's planar layout
    with pytest.raises(tmhip.TmError) as e:
        bad = pos.copy()
        bad[5, 2] += 0.01
        ctx.set_geometry(bad, K, 3)
    assert e.value.code == -3
    ctx.set_geometry(pos, K, 3)
    with pytest.raises(tmhip.TmError) as e:
        ctx.set_spheres(to_dev(np.full(16, 0.31), torch.float64), 2.0)
    assert e.value.code == -2
    r = np.full(16, 0.2)
    r[3] = np.nan
    with pytest.raises(tmhip.TmError) as e:
        ctx.set_spheres(to_dev(r, torch.float64), 2.0)
    assert e.value.code == -6
    ctx.set_spheres(to_dev(np.full(16, 0.2), torch.float64), 2.0)
    a0 = ctx.plane_wave_rhs(*wl.incidence("x"))
    s, info = ctx.solve(a0, tol=1e-14, max_iter=3)
    assert info[0]["status"] == 1 and info[0]["iters"] == 3
    ctx.close()


@pytest.mark.parametrize("variant", range(11))
def test_every_matvec_variant_matches_oracle(variant):
    """All kernel variants the autotuner may pick compute the same product."""
    print(f"[case] variant {variant}", flush=True)
    rng = np.random.default_rng(40 + variant)
    nx, ny, lmax = 29, 21, 3
    ctx, pos, radii = make_ctx(nx, ny, lmax)
    x = rand_vec(rng, 2, nx * ny, 30)
    lc = oracle.LatticeCoupling(nx, ny, wl.PITCH, K, lmax)
    ref = np.stack([lc.apply(x[r]) for r in range(2)])
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        for items in (0, 7, 300):
            ctx.set_matvec_config(prec, variant, items)
            y = host(ctx.apply_operator(to_dev(x), "coupling", prec))
            assert rel(y, ref) < tol, (prec, items)
    ctx.close()


def test_autotune_keeps_a_correct_configuration():
    rng = np.random.default_rng(77)
    ctx, pos, radii = make_ctx(40, 24, 3)
    x = rand_vec(rng, 1, 960, 30)
    ref = oracle.LatticeCoupling(40, 24, wl.PITCH, K, 3).apply(x[0])
    for prec, tol in (("mixed", 2e-5), ("fp64", 1e-12)):
        ms, (v, items) = ctx.autotune(1, prec)
        assert ms > 0 and 0 <= v < 11
        assert rel(host(ctx.apply_operator(to_dev(x), "coupling", prec))[0], ref) < tol
    ctx.close()


def test_progress_callback_reports_every_cycle():
    ctx, pos, radii = make_ctx(12, 10, 3, seed=4)
    kh, po = wl.incidences(["x"])
    a0 = ctx.plane_wave_rhs(kh, po)
    seen = []
    ctx.set_progress(lambda c, i, n, r: seen.append((c, i, n, r)))
    _, info = ctx.solve(a0, tol=1e-12, restart=10)
    assert info[0]["status"] == 0 and len(seen) == info[0]["cycles"] > 1
    assert [x[0] for x in seen] == list(range(len(seen)))
    assert all(x[2] == 1 for x in seen) and abs(seen[0][3] - 1.0) < 1e-12
    assert all(b[3] <= a[3] * (1 + 1e-12) for a, b in zip(seen, seen[1:]))
    seen.clear()
    _, binfo = ctx.solve_batched([(0, 0, 6, 5), (3, 2, 8, 7)], kh, po, restart=10, tol=1e-10)
    assert len(seen) == max(i["cycles"] for row in binfo for i in row)
    assert all(1 <= x[2] <= 2 for x in seen)
    # a long cycle also reports every 50 steps inside the cycle (Givens
    # estimates, non-increasing within the cycle)
    big, _, _ = make_ctx(20, 18, 3, seed=4)
    big.set_progress(lambda c, i, n, r: seen.append((c, i, n, r)))
    seen.clear()
    _, info = big.solve(big.plane_wave_rhs(kh, po), tol=1e-13, restart=300)
    inner = [x for x in seen if x[0] == 0 and x[1] > 0]
    # after steps 50, 100, ... of cycle 0, except a step that ends the solve
    # or the cycle (the next cycle reports at its start)
    assert len(inner) == (min(info[0]["iters"], 300) - 1) // 50
    assert all(x[1] % 50 == 0 for x in inner)
    assert all(b[3] <= a[3] * (1 + 1e-12) for a, b in zip(inner, inner[1:]))
    big.close()
    ctx.set_progress(None)
    seen.clear()
    ctx.solve(a0, tol=1e-8)
    assert not seen
    ctx.close()


# ----------------------------------------------------------------- batched subregions
SUBS = [(0, 0, 12, 9), (5, 3, 20, 16), (30, 20, 10, 10), (7, 7, 1, 1), (0, 0, 24, 20), (13, 2, 17, 5)]


@pytest.mark.parametrize("precision,use_graph,autotune",
                         [("fp64", False, False), ("fp64", True, False), ("mixed", True, False),
                          ("fp64", True, True), ("mixed", True, True)])
def test_batched_subregions_match_single_solves(precision, use_graph, autotune):
    """Every (subregion, rhs) of a batch equals the same subregion solved on
    its own (scatterers outside it ignored), for graph replay and eager runs,
    with the default launch configuration and with the batched autotuner's."""
    print(f"[case] batched {precision} graph={use_graph} autotune={autotune}", flush=True)
    nx, ny, lmax = 40, 30, 3
    pos = wl.lattice_positions(nx, ny)
    radii = wl.lens_radii(nx, ny)
    kh, po = wl.incidences(["x", "p10"])
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    assert ctx.batch_config(precision) == (0, 0)
    ctx.set_batch_autotune(autotune)
    sb, info = ctx.solve_batched(SUBS, kh, po, use_graph=use_graph, tol=1e-11, precision=precision,
                                 max_iter=20000)
    for k in range(len(SUBS)):
        print(f"[info] sub {k} {SUBS[k]}: {info[k]}", flush=True)
    if use_graph:
        assert ctx.batch_graph_used()
    pf, items = ctx.batch_config(precision)
    print(f"[info] batch config {precision}: prefetch {pf}, items {items}", flush=True)
    R = len(kh)
    if autotune:
        assert 1 <= pf <= (3 if precision == "mixed" else 2)
        assert items in [wg // (2 * R) for wg in (16384, 32768, 65536)]
    else:
        # the context's default kernels: FP64 table prefetch depth 2, complex64 depth 1
        assert (pf, items) == (1 if precision == "mixed" else 2, 32768 // (2 * R))
    for k, (ox, oy, sx, sy) in enumerate(SUBS):
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * nx + ix).ravel()
        single = tmhip.Context(0)
        single.set_geometry(pos[idx], K, lmax)
        single.set_spheres(to_dev(radii[idx], torch.float64), wl.N_REL)
        a0 = single.plane_wave_rhs(kh, po)
        s_ref, info1 = single.solve(a0, tol=1e-13, max_iter=40000)
        assert all(i["status"] == 0 for i in info1), info1
        for r in range(2):
            assert info[k][r]["status"] == 0 and info[k][r]["rel_residual"] <= 1e-11
            assert rel(host(sb[k])[r], host(s_ref)[r]) < 1e-9, (k, r)
        single.close()
    # a small subregion against the oracle's dense LU directly
    ox, oy, sx, sy = SUBS[0]
    ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
    idx = (iy * nx + ix).ravel()
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii[idx], wl.N_REL)
    s_or = oracle.solve_dense(pos[idx], K, lmax, t,
                              oracle.plane_wave_coeffs(lmax, K, kh[1], po[1], pos[idx]))
    assert rel(host(sb[0])[1], s_or) < 1e-9
    ctx.close()


# ----------------------------------------------------------------- full-size (100 x 100)
def test_full_size_c2_sampled_rows_and_solve():
    """100 x 100 lattice, lmax 3 (the benchmark workload): sampled rows of the
    FP64 and complex64 operators against the oracle's row-by-row product, and
    the converged mixed-precision and FP64 solves checked through the oracle's
    rows of B s - T a0 and against each other."""
    print("[case] full-size c2", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("c2")
    n, lmax = cfg["nx"], cfg["lmax"]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    rng = np.random.default_rng(2024)
    x = rand_vec(rng, 1, n * n, 30)
    rows = [0, 57, 4950, 5049, 9999]
    ref = oracle.rows_A(pos, K, lmax, x[0], rows)
    y64 = host(ctx.apply_operator(to_dev(x), "coupling", "fp64"))[0]
    y32 = host(ctx.apply_operator(to_dev(x), "coupling", "mixed"))[0]
    assert rel(y64[rows], ref) < 1e-12
    assert rel(y32[rows], ref) < 2e-5
    a0 = ctx.plane_wave_rhs(kh, po)
    smx, imx = ctx.solve(a0, tol=1e-8, precision="mixed")
    s64, i64 = ctx.solve(a0, tol=1e-10, precision="fp64")
    assert imx[0]["status"] == 0 and i64[0]["status"] == 0
    assert imx[0]["rel_residual"] <= 1e-8
    assert rel(host(smx)[0], host(s64)[0]) < 1e-6
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii[rows], wl.N_REL)
    b = t * host(a0)[0][rows]
    s = host(s64)[0]
    r_rows = s[rows] - t * oracle.rows_A(pos, K, lmax, s, rows) - b
    assert np.linalg.norm(r_rows) / np.linalg.norm(b) < 1e-6
    ctx.close()


def test_full_size_c5_sampled_rows():
    """300 x 300 lens tile, lmax 3, 2 RHS, in the launch configuration the
    tile benchmark times (both block-matvec precisions): sampled rows of the
    coupling operator against the oracle's row-by-row product."""
    print("[case] full-size c5", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("c5")
    n, lmax, R = cfg["nx"], cfg["lmax"], 2
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    ctx.set_matvec_config("mixed", 9, 32768 // (2 * R))
    ctx.set_matvec_config("fp64", 8, 16384 // (2 * R))
    x = rand_vec(np.random.default_rng(300), R, n * n, 30)
    y64 = host(ctx.apply_operator(to_dev(x), "coupling", "fp64"))
    y32 = host(ctx.apply_operator(to_dev(x), "coupling", "mixed"))
    # a corner, the last site, and sites in the last (4-row) band and the centre
    for r, rows in ((0, [0, n * n - 1]), (1, [n * (n - 3) + 150, n * 150 + 149])):
        ref = oracle.rows_A(pos, K, lmax, x[r], rows)
        assert rel(y64[r][rows], ref) < 1e-12, (r, rows)
        assert rel(y32[r][rows], ref) < 2e-5, (r, rows)
    ctx.close()


def test_full_size_c4_transposed_rows():
    """150 x 150 lattice, lmax 3 (the adjoint workload): sampled rows of the
    transposed coupling operator the adjoint solve applies."""
    print("[case] full-size c4", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("c4")
    n, lmax = cfg["nx"], cfg["lmax"]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    x = rand_vec(np.random.default_rng(150), 1, n * n, 30)
    rows = [0, n * 75 + 74, n * n - 1]
    ref = oracle.rows_A(pos, K, lmax, x[0], rows, transpose=True)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        y = host(ctx.apply_operator(to_dev(x), "coupling_t", prec))[0]
        assert rel(y[rows], ref) < tol, prec
    ctx.close()
