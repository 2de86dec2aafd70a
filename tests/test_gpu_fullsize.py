"""Full-size parity on the paths the benchmarks time, against the CPU oracle:
  * the 100 x 100 solve (FP64 at tol 1e-10, mixed refined to 1e-12) checked
    through oracle rows of B s - T a0, and the complex64-limited solve (tol
    1e-6) against the 1e-5 coefficient target;
  * the mixed solve on a 30 x 30 lattice against the oracle's own
    matrix-free FP64 GMRES;
  * the near field and its transpose past one LDS chunk of spheres and one
    tile of points, and at the 300 x 300 lens tile on sampled plane points;
  * the four smallest and four largest of the 48 lens subregions, batched at
    GMRES(200), each checked through oracle residual rows;
  * the 100 x 100 silicon-cylinder lattice at lmax 6 (dense null-field T) in
    its autotuned launch configurations: the coupling product on sampled rows
    and the forward operator on the centre row;
  * the jittered 100 x 100 lattice (off-lattice blocks formed per pair): the
    coupling product and its transpose on sampled rows.
Row residuals are ||s_rows - t A_rows s - t a0_rows|| / ||t a0_rows||."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from oracle.ebcm import cylinder_surface, ebcm_tmatrix  # noqa: E402
from paper_2107_09879_amd import tmhip  # noqa: E402

pytestmark = pytest.mark.gpu
K = wl.K
DEV = torch.device("cuda", 0)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def to_dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def row_residual(pos, lmax, t_rows, s, a0_rows, rows):
    b = t_rows * a0_rows
    r = s[rows] - t_rows * oracle.rows_A(pos, K, lmax, s, rows) - b
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_c2_solves_through_oracle_rows():
    print("[case] c2 solves vs oracle rows", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("c2")
    n, lmax = cfg["nx"], cfg["lmax"]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    a0 = ctx.plane_wave_rhs(kh, po)
    s64, i64 = ctx.solve(a0, tol=1e-10, precision="fp64")
    sref, iref = ctx.solve(a0, tol=1e-12, precision="mixed", max_iter=4000)
    s6, i6 = ctx.solve(a0, tol=1e-6, precision="mixed")
    for info in (i64, iref, i6):
        assert info[0]["status"] == 0, info
    rows = [0, 99, 57, 4950, 5049, 5050, 7777, 9900, 9999]
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii[rows], wl.N_REL)
    a0r = host(a0)[0][rows]
    r64 = row_residual(pos, lmax, t, host(s64)[0], a0r, rows)
    rref = row_residual(pos, lmax, t, host(sref)[0], a0r, rows)
    print(f"  row residual: fp64 (tol 1e-10) {r64:.2e}, mixed refined (1e-12) {rref:.2e}", flush=True)
    assert r64 < 1e-9
    assert rref < 1e-10
    # complex64 matvecs stopped at 1e-6: the 1e-5 coefficient target
    e6 = rel(host(s6)[0], host(sref)[0])
    print(f"  mixed tol 1e-6 vs refined: {e6:.2e}", flush=True)
    assert e6 < 1e-5
    ctx.close()


def test_mixed_solve_vs_oracle_matrix_free_gmres():
    print("[case] 30x30 mixed vs oracle GMRES", flush=True)
    nx = ny = 30
    lmax = 3
    pos = wl.lattice_positions(nx, ny)
    radii = wl.uniform_radii(nx * ny, 0.15, 0.25, 7)
    kh, po = wl.incidence("x")
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    s, info = ctx.solve(ctx.plane_wave_rhs(kh, po), tol=1e-12, precision="mixed")
    assert info[0]["status"] == 0
    t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii, wl.N_REL)
    a0 = oracle.plane_wave_coeffs(lmax, K, kh, po, pos)
    lc = oracle.LatticeCoupling(nx, ny, wl.PITCH, K, lmax)
    b = (t * a0).ravel()
    L = oracle.n_coeffs(lmax)
    sref = oracle.gmres(lambda x: x - (t * lc.apply(x.reshape(-1, L))).ravel(), b, tol=1e-13,
                        restart=100, maxiter=3000)
    sref = sref[0] if isinstance(sref, tuple) else sref
    e = rel(host(s)[0].ravel(), sref)
    print(f"  mixed (1e-12) vs oracle GMRES (1e-13): {e:.2e}", flush=True)
    assert e < 1e-10
    ctx.close()


def test_near_field_past_one_chunk_and_one_point_tile():
    """13 x 11 spheres (the last 32-sphere chunk ragged) and 300 points (more
    than one 256-point tile of the transposed map), two right-hand sides."""
    print("[case] near field 13x11, 300 points", flush=True)
    nx, ny, lmax, R = 13, 11, 3, 2
    pos = wl.lattice_positions(nx, ny)
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(wl.uniform_radii(nx * ny, 0.15, 0.25, 1), torch.float64), wl.N_REL)
    rng = np.random.default_rng(13)
    L = ctx.L
    s = (rng.normal(size=(R, nx * ny, L)) + 1j * rng.normal(size=(R, nx * ny, L))) * 0.1
    P = 300
    pts = np.stack([rng.uniform(-1.0, 8.2, P), rng.uniform(-1.0, 7.0, P), rng.uniform(0.5, 4.0, P)], -1)
    pts[:7, 2] *= -1.0  # a few below the plane
    ptd = to_dev(pts, torch.float64)
    E64 = host(ctx.near_field(to_dev(s), ptd, "fp64"))
    E32 = host(ctx.near_field(to_dev(s), ptd, "mixed"))
    for r in range(R):
        ref = oracle.near_field(s[r], pos, K, lmax, pts)
        scale = np.abs(ref).max()
        assert np.abs(E64[r] - ref).max() < 1e-11 * scale
        assert np.abs(E32[r] - ref).max() < 1e-4 * scale
    w = rng.normal(size=(R, P, 3)) + 1j * rng.normal(size=(R, P, 3))
    v = host(ctx.near_field_adjoint(ptd, to_dev(w)))
    for r in range(R):
        # transpose: sum_{p,c} w E = sum_{i,n} v s for every s
        ref = np.zeros((nx * ny, L), dtype=complex)
        for p in range(P):
            ref += np.einsum('c,cil->il', w[r, p], oracle.detector_vectors(pos, K, lmax, pts[p]))
        assert np.abs(v[r] - ref).max() < 1e-11 * np.abs(ref).max()
    ctx.close()


def test_c5_near_field_plane_sampled():
    """The 300 x 300 lens tile's near-field plane (z = 5 wavelengths over the
    footprint), mixed precision as the benchmark runs it, on 64 sampled plane
    points (corners, centre, random) for a seeded coefficient vector."""
    print("[case] c5 near field sampled", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("c5")
    n, lmax = cfg["nx"], cfg["lmax"]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    rng = np.random.default_rng(5)
    s = (rng.normal(size=(1, n * n, ctx.L)) + 1j * rng.normal(size=(1, n * n, ctx.L))) * 1e-3
    n_side, extent, z = cfg["plane"]
    plane = wl.near_field_plane(n_side, extent, z)
    pick = [0, n_side - 1, n_side * (n_side - 1), n_side * n_side - 1,
            n_side * (n_side // 2) + n_side // 2]
    pick += list(rng.choice(n_side * n_side, 64 - len(pick), replace=False))
    pts = plane[pick]
    E = host(ctx.near_field(to_dev(s), to_dev(pts, torch.float64), "mixed"))[0]
    ref = oracle.near_field(s[0], pos, K, lmax, pts)
    err = np.abs(E - ref).max() / np.abs(ref).max()
    print(f"  mixed near field vs oracle, 64 points over 9e4 spheres: {err:.2e}", flush=True)
    assert err < 1e-4
    ctx.close()


def test_c3_smallest_and_largest_subregions():
    """The 4 smallest and 4 largest of the 48 lens subregions, one batch at
    GMRES(200) in mixed precision to 1e-8, every system checked through oracle
    residual rows (a corner, the centre and a random site)."""
    print("[case] c3 4 smallest + 4 largest", flush=True)
    cfg = wl.CONFIGS["c3"]
    pos, radii, kh, po, _ = wl.config_inputs("c3")
    allsubs = [(ox, oy, sd, sd) for ox, oy, sd in wl.subregions(seed=cfg["seed"])]
    order = np.argsort([q[2] for q in allsubs])
    subs = [allsubs[i] for i in list(order[:4]) + list(order[-4:])]
    kh, po = kh[:1], po[:1]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, cfg["lmax"])
    ctx.set_spheres(to_dev(radii, torch.float64), wl.N_REL)
    sb, info = ctx.solve_batched(subs, kh, po, use_graph=True, tol=1e-8, restart=200,
                                 precision="mixed", max_iter=20000)
    rng = np.random.default_rng(48)
    lmax, nxf = cfg["lmax"], cfg["nx"]
    for k, (ox, oy, sx, sy) in enumerate(subs):
        assert info[k][0]["status"] == 0 and info[k][0]["rel_residual"] <= 1e-8, (k, info[k])
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * nxf + ix).ravel()
        p_k = pos[idx]
        rows = [0, (sy // 2) * sx + sx // 2, int(rng.integers(sx * sy))]
        t, _ = oracle.mie_tmatrix_diag_many(lmax, K, radii[idx][rows], wl.N_REL)
        a0r = oracle.plane_wave_coeffs(lmax, K, kh[0], po[0], p_k[rows])
        res = row_residual(p_k, lmax, t, host(sb[k])[0], a0r, rows)
        print(f"  subregion {k} {subs[k]}: iters {info[k][0]['iters']}, oracle row residual {res:.2e}",
              flush=True)
        assert res < 5e-8
    ctx.close()


def test_cyl6_cylinder_lattice_operator_sampled():
    """100 x 100 silicon cylinders at lmax 6 with the kernels the benchmark
    autotunes.  The coupling product of a vector living on 8 sites is checked
    on 32 target rows (corners, centre, the sources themselves, random) with
    the oracle's row routine over just those sites; the forward operator
    x - T A x of a dense random vector on the centre row with the oracle's
    full row of A and its null-field T of that cylinder."""
    print("[case] cyl6 operator sampled", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("cyl6")
    height, n_rel = cfg["cylinders"]
    n, lmax = cfg["nx"], cfg["lmax"]
    N = n * n
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    ctx.set_cylinders(to_dev(radii, torch.float64), height, n_rel)
    L = ctx.L
    rng = np.random.default_rng(66)
    src = [0, n - 1, N // 2 + n // 2, N - n, N - 1] + [int(v) for v in rng.choice(N, 3, replace=False)]
    xs = np.zeros((1, N, L), dtype=complex)
    xs[0, src] = rng.normal(size=(len(src), L)) + 1j * rng.normal(size=(len(src), L))
    rows = list(dict.fromkeys(src + [1, n, 2 * n + 3] + [int(v) for v in rng.choice(N, 32, replace=False)]))[:32]
    ref = []
    for j in rows:
        others = [i for i in src if i != j]
        sub = np.concatenate([xs[0, [j]] * 0.0, xs[0, others]])
        ref.append(oracle.rows_A(pos[[j] + others], K, lmax, sub, [0])[0])
    ref = np.array(ref)
    x = rng.normal(size=(1, N, L)) + 1j * rng.normal(size=(1, N, L))
    c = N // 2 + n // 2
    Tc = ebcm_tmatrix(lmax, K, n_rel, cylinder_surface(radii[c], height, 96))
    fref = x[0, c] - Tc @ oracle.rows_A(pos, K, lmax, x[0], [c])[0]
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        ms, conf = ctx.autotune(1, prec)
        y = host(ctx.apply_operator(to_dev(xs), "coupling", prec))[0]
        e = rel(y[rows], ref)
        f = host(ctx.apply_operator(to_dev(x), "forward", prec))[0, c]
        ef = rel(f, fref)
        print(f"  {prec} (variant {conf[0]}, items {conf[1]}): sampled rows {e:.2e}, "
              f"forward centre row {ef:.2e}", flush=True)
        assert e < tol
        assert ef < tol
    ctx.close()


def test_offl_jittered_lattice_operator_sampled():
    """The benchmark's jittered 100 x 100 lattice, where every translation
    block is formed on the fly: rows of A x and A^T x for a dense random x at
    corners, centre and random targets, both precisions, against the oracle's
    row routine."""
    print("[case] offl operator sampled", flush=True)
    pos, radii, kh, po, cfg = wl.config_inputs("offl")
    n, lmax = cfg["nx"], cfg["lmax"]
    N = n * n
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, K, lmax)
    assert ctx.get_lattice()[2] == 0.0
    L = ctx.L
    rng = np.random.default_rng(77)
    x = rng.normal(size=(1, N, L)) + 1j * rng.normal(size=(1, N, L))
    rows = [0, n - 1, N // 2 + n // 2, N - 1] + [int(v) for v in rng.choice(N, 2, replace=False)]
    ref = oracle.rows_A(pos, K, lmax, x[0], rows)
    refT = oracle.rows_A(pos, K, lmax, x[0], rows, transpose=True)
    xd = to_dev(x)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        y = host(ctx.apply_operator(xd, "coupling", prec))[0][rows]
        yT = host(ctx.apply_operator(xd, "coupling_t", prec))[0][rows]
        e, eT = rel(y, ref), rel(yT, refT)
        print(f"  {prec}: rows {e:.2e}, transposed rows {eT:.2e}", flush=True)
        assert e < tol
        assert eT < tol
    ctx.close()
