"""Benchmark: T-matrix multiple-scattering solve on one MI355X.

Workload (default): 100 x 100 lattice of n = 2.0 spheres (1e4 scatterers,
pitch 0.6 wavelengths, radii uniform in [0.15, 0.25] wavelengths, seed 2),
lmax = 3 (30 coefficients per sphere, 3e5 complex unknowns), x-polarised
plane wave at normal incidence.

One step = the whole hot path on device-resident inputs: translation-table
build, Mie T-matrices, plane-wave right-hand side, mixed-precision GMRES(50)
(complex64 matvec with FP32 accumulation, FP64 Arnoldi and FP64 iterative
refinement) to a 1e-8 FP64 true relative residual, and far-field readout.
The timed value is the time-to-solution per step (lower is better).

Also reported: the same solve in plain FP64 GMRES on the same GPU, the block
matvec's throughput against the matrix-core roofline (HIP events on the
library's stream around each block-matvec launch), and the CPU oracle timed
on the host cores (one FP64 matvec, extrapolated by the GPU's iteration count).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6   # TFLOP/s, MI355X dense FP64 matrix


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_names(variant, ctype):
    """Names of the kernels one block matvec of a variant launches (as the
    profiler prints them, template arguments included)."""
    if variant >= 8:
        # (columns groups per wave, displacement block) of the regular and the
        # wide tiles
        gx, reg, wide = (4, (16, 8), (16, 8)) if ctype == "float" else (2, (8, 16), (8, 16))
        pf = variant - 7 if ctype == "float" else min(variant - 7, 2)
        # regular tiles, then the wide-tile instance for the rows past the
        # last multiple of 16 (absent when the height is a multiple of 16)
        return [f"block_matvec_lds_kernel<{ctype}, {gx}, {b[0]}, {b[1]}, {pf}, {w}>"
                for b, w in ((reg, "false"), (wide, "true"))]
    gauss, pref, occ = variant & 1, (variant >> 1) & 1, 4 if variant & 4 else 2
    return [f"block_matvec_kernel<{ctype}, {str(bool(gauss)).lower()}, {str(bool(pref)).lower()}, {occ}>"]


def kernel_name(variant, ctype):
    return " + ".join(kernel_names(variant, ctype))


MATVEC_SOURCES = ("paper_2107_09879_amd/csrc/tm_matvec_lds.hip", "paper_2107_09879_amd/csrc/tm_matvec.hip")


def kernel_source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in MATVEC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernels, workload):
    """HBM bytes of one block matvec (the sum over its kernels) from the
    committed counter summary (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated
    against a plain copy), or None when a kernel has no row for this workload
    or the matvec sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "block_matvec_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    rows = {}
    with open(path) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[1] == workload and cells[2] == digest:
                try:
                    rows[cells[0]] = float(cells[3])
                except ValueError:
                    pass
    if not all(k in rows for k in kernels):
        return None
    return sum(rows[k] for k in kernels)


NF_SOURCE = "paper_2107_09879_amd/csrc/tm_basis.hip"
# FP32 VALU issue peak: 0.5 wave64 instructions per SIMD per cycle on 1024
# SIMDs at 2.4 GHz, in lane-instructions per second (FMA = one instruction)
PEAK_VALU_LANE_INSTR = 1024 * 0.5 * 64 * 2.4e9


def nf_valu_per_pair(kernel):
    """VALU lane-instructions per (point, sphere) pair of the near-field kernel
    from the committed counter summary, or None if the source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "near_field_c5_300x300_plane1000x1000.md")
    if not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, NF_SOURCE), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    with open(path) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 3 and cells[0] == kernel and cells[1] == digest:
                try:
                    return float(cells[2])
                except ValueError:
                    return None
    return None


def copy_calibration(torch, mib=512):
    """A plain copy of known size for the HBM counters: y = x * 1 over
    `mib` MiB of float32 reads `mib` MiB and writes `mib` MiB."""
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.mul(x, 1.0)
    torch.cuda.synchronize()
    del x, y


def tune_matvec(ctx, args, n_rhs):
    """Block-matvec kernel of each precision: fixed by --matvec-config, else
    autotuned on the context's geometry (set-up, outside any timed region)."""
    tuned = {}
    fixed = {}
    for spec in args.matvec_config:
        prec, v, items = spec.split(":")
        fixed[prec] = (int(v), int(items))
    for prec in ("mixed", "fp64"):
        if prec in fixed:
            ctx.set_matvec_config(prec, *fixed[prec])
            tuned[prec] = {"variant": fixed[prec][0], "items": fixed[prec][1], "fixed": True}
            log(f"[bench] {prec} matvec fixed: variant {fixed[prec][0]}, items {fixed[prec][1]}")
        elif not args.no_autotune:
            ms, conf = ctx.autotune(n_rhs, prec)
            tuned[prec] = {"block_matvec_ms": ms, "variant": conf[0], "items": conf[1]}
            log(f"[bench] autotune {prec}: {ms:.3f} ms, variant {conf[0]}, items {conf[1]}")
    return tuned


def isolated_matvec(ctx, n_rhs, reps):
    """Average block-matvec launch of each precision over `reps` back-to-back
    forward operators on a seeded random vector (HIP events on the library's
    stream), with the algorithmic FP32 / FP64 rate against the matrix peak."""
    import torch

    rng = np.random.default_rng(0)
    shape = (n_rhs, ctx.n, ctx.L)
    x = torch.tensor(rng.normal(size=shape) + 1j * rng.normal(size=shape), dtype=torch.complex128,
                     device="cuda")
    mv = {}
    for which, prec, peak in ((1, "mixed", PEAK_FP32_MFMA), (0, "fp64", PEAK_FP64_MFMA)):
        ctx.apply_operator(x, "forward", prec)
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(reps):
            ctx.apply_operator(x, "forward", prec)
        ctx.profile_enable(False)
        ms, launches, flops = ctx.profile_query(which)
        avg = ms / max(launches, 1) / 1e3
        tf = flops / avg / 1e12
        mv[prec] = {"avg_launch_ms": avg * 1e3, "tflops": tf, "peak_tflops": peak, "frac": tf / peak,
                    "flops_per_launch": flops, "launches": launches}
        log(f"[bench] {prec} block matvec: {avg*1e3:.3f} ms, {tf:.2f} TFLOP/s ({tf/peak:.1%} of {peak})")
    ctx.profile_reset()
    return mv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2",
                    help="workload: c1, c2 (default), c3 (batched subregions), c4 (adjoint and "
                         "gradients), c5 (300x300 tile), jinc (padding study), cyl6 (lmax-6 "
                         "silicon cylinders), offl (off-lattice blocks)")
    ap.add_argument("--matvec-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--subregions", type=int, default=0, help="c3: use only the first K subregions")
    ap.add_argument("--no-sequential", action="store_true",
                    help="c3: skip the one-subregion-at-a-time comparison")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="c3: keep the batched path's default launch configuration instead of "
                         "timing the candidates on the batch first")
    ap.add_argument("--restart", type=int, default=0,
                    help="c3, c5: GMRES restart length (default: the workload's, 50)")
    ap.add_argument("--tile-iters", type=int, default=300,
                    help="c5: Arnoldi steps of the bounded solve used for the extrapolation")
    ap.add_argument("--tile-rhs", type=int, default=-1,
                    help="c5: solve only this right-hand side (0 or 1) to the tolerance and time it")
    ap.add_argument("--tile-precision", default="mixed", choices=["mixed", "fp64"],
                    help="c5: precision of the --tile-rhs solve")
    ap.add_argument("--tile-max-iter", type=int, default=20000,
                    help="c5: Arnoldi steps allowed to the --tile-rhs solve (a multiple of the restart "
                         "ends it on a cycle boundary, where a later run can resume exactly)")
    ap.add_argument("--tile-x0", default="", help="c5: .npy start vector of the --tile-rhs solve")
    ap.add_argument("--tile-save", default="", help="c5: .npy file for the --tile-rhs solution")
    ap.add_argument("--cyl-max-iter", type=int, default=5000,
                    help="cyl6: Arnoldi steps allowed to the solve of each step")
    ap.add_argument("--offl-max-iter", type=int, default=5000,
                    help="offl: Arnoldi steps allowed to the solve of each step")
    ap.add_argument("--matvec-config", action="append", default=[], metavar="PREC:VARIANT:ITEMS",
                    help="fix the block-matvec kernel of a precision (mixed or fp64) instead of "
                         "autotuning it, e.g. mixed:9:16384")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; there is no multi-GPU path. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.config == "c3":
        return bench_batched(args)
    if args.config == "c4":
        return bench_adjoint(args)
    if args.config == "c5":
        return bench_tile(args)
    if args.config == "jinc":
        return bench_jinc_padding(args)
    if args.config == "cyl6":
        return bench_cylinders(args)
    if args.config == "offl":
        return bench_offlattice(args)

    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    dev = torch.device("cuda", 0)
    pos, radii, kh, po, cfg = wl.config_inputs(args.config)
    n = cfg["nx"]
    lmax = cfg["lmax"]
    N = n * n
    tol = cfg.get("tol", 1e-8)
    restart = cfg.get("restart", 50)
    log(f"[bench] config {args.config}: {cfg['name']}, N={N}, lmax={lmax}, R={len(kh)}")
    ctx = tmhip.Context(0)
    radii_d = torch.tensor(radii, dtype=torch.float64, device=dev)
    dirs = torch.tensor([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], dtype=torch.float64, device=dev)

    # set-up outside the timed region: kernel variant / work split per precision
    ctx.set_geometry(pos, wl.K, lmax)
    tuned = tune_matvec(ctx, args, len(kh))

    def step(precision):
        ctx.set_geometry(pos, wl.K, lmax)
        ctx.set_spheres(radii_d, wl.N_REL)
        a0 = ctx.plane_wave_rhs(kh, po)
        s, info = ctx.solve(a0, tol=tol, restart=restart, precision=precision, inner_tol=1e-4)
        F = ctx.far_field(s, dirs)
        return s, info, F

    for w in range(args.warmup):
        _, info, _ = step("mixed")
        log(f"[bench] warmup {w}: {info}")
    copy_calibration(torch)
    # timed region; the library records HIP events on its own stream around
    # every block-matvec launch, which gives the kernel's average duration
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        s, info, F = step("mixed")
        infos.append(info)
        log(f"[bench] step {k}: {info[0]}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.profile_enable(False)
    live = {}
    for which, prec, peak in ((1, "mixed", PEAK_FP32_MFMA), (0, "fp64", PEAK_FP64_MFMA)):
        ms, launches, flops = ctx.profile_query(which)
        if launches:
            avg = ms / launches / 1e3
            live[prec] = {"avg_launch_ms": avg * 1e3, "launches": launches, "flops_per_launch": flops,
                          "tflops": flops / avg / 1e12, "frac": flops / avg / 1e12 / peak}
    ctx.profile_reset()
    log(f"[bench] mixed time-to-solution {dt:.4f} s/step, info {infos[-1]}, matvec {live}")

    fp64 = None
    if not args.no_fp64:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s64, info64, _ = step("fp64")
        torch.cuda.synchronize()
        fp64 = {"time_to_solution_s": time.perf_counter() - t1, "info": info64[0]}
        log(f"[bench] fp64 time-to-solution {fp64['time_to_solution_s']:.4f} s, {info64[0]}")
        d = (s - s64).abs().pow(2).sum().sqrt() / s64.abs().pow(2).sum().sqrt()
        fp64["mixed_vs_fp64_rel_diff"] = float(d)

    # block-matvec throughput in isolation (same kernels, back to back)
    mv = isolated_matvec(ctx, len(kh), args.matvec_reps)

    # algorithmic bytes of one complex64 matvec: table + input + output
    L = ctx.L
    D = (2 * n - 1) ** 2
    alg_bytes = D * (L * L // 2) * 8 + 2 * N * L * 8
    dom = live.get("mixed", mv["mixed"])
    gbs = alg_bytes / (dom["avg_launch_ms"] / 1e3) / 1e9
    variant = ctx.get_matvec_config("mixed")[0]
    knames = kernel_names(variant, "float")
    if n % 16 == 0:
        knames = knames[:1]
    kname = " + ".join(knames)

    cpu = None
    if not args.no_cpu_baseline and args.config == "c2":
        cpu = cpu_baseline(pos, radii, kh, po, cfg, infos[-1][0])
    extra = {}

    out = {
        "metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
        "value": dt,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "scatterers": N, "lmax": lmax, "unknowns": N * L,
                   "rhs": len(kh), "tol": tol, "restart": restart, "precision": "mixed"},
        "solve_info": infos[-1][0],
        "autotuned": tuned,
        "fp64_gmres": fp64,
        "matvec_timed_region": live,
        "matvec_isolated": mv,
        "matvec_algorithmic_GBps": gbs,
        "roofline": {"bound": "mfma", "achieved": dom["tflops"], "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": dom["tflops"] / PEAK_FP32_MFMA,
                     # issued matrix-core flops (Gauss 3-product form, padded slots)
                     "mfma_issue_frac": dom["tflops"] * mfma_issue_ratio(lmax) / PEAK_FP32_MFMA,
                     "effective_ceiling_tflops": PEAK_FP32_MFMA / mfma_issue_ratio(lmax),
                     "traffic": measured_traffic(knames, cfg["name"]),
                     "kernel": kname, "avg_launch_ms": dom["avg_launch_ms"],
                     "flops_per_launch": dom["flops_per_launch"],
                     "kernel_source_digest": kernel_source_digest()},
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_tile(args):
    """300 x 300 lens tile (9e4 spheres, lmax 3, 2 RHS): translation-table
    build, block-matvec throughput in both precisions, a bounded
    mixed-precision solve (its residual history gives an extrapolated
    time-to-solution, labelled as such), and the scattered field on a
    1000 x 1000 plane 5 wavelengths above the lattice."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    pos, radii, kh, po, cfg = wl.config_inputs("c5")
    n, lmax, R = cfg["nx"], cfg["lmax"], len(kh)
    N = n * n
    ctx = tmhip.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_geometry(pos, wl.K, lmax)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device="cuda"), wl.N_REL)
    log(f"[bench] tile: N={N}, table build {t_table:.2f} s")
    fixed = {"mixed": (9, 32768 // (2 * R)), "fp64": (8, 16384 // (2 * R))}
    for spec in args.matvec_config:
        prec, v, items = spec.split(":")
        fixed[prec] = (int(v), int(items))
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.normal(size=(R, N, ctx.L)) + 1j * rng.normal(size=(R, N, ctx.L)),
                     dtype=torch.complex128, device="cuda")
    mv = {}
    for which, prec, peak in ((1, "mixed", PEAK_FP32_MFMA), (0, "fp64", PEAK_FP64_MFMA)):
        ctx.set_matvec_config(prec, *fixed[prec])
        ctx.apply_operator(x, "forward", prec)
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(3):
            ctx.apply_operator(x, "forward", prec)
        ctx.profile_enable(False)
        ms, launches, flops = ctx.profile_query(which)
        avg = ms / launches / 1e3
        mv[prec] = {"variant": fixed[prec][0], "items": fixed[prec][1], "avg_launch_ms": avg * 1e3,
                    "tflops": flops / avg / 1e12, "frac": flops / avg / 1e12 / peak, "rhs": R}
        log(f"[bench] tile {prec} block matvec ({R} RHS): {avg*1e3:.1f} ms, {flops/avg/1e12:.2f} TFLOP/s")
    ctx.profile_reset()
    del x
    hist = []
    t_start = [None]

    def progress(cycles, iters, n_live, worst):
        hist.append((time.perf_counter() - t_start[0], iters, worst))
        log(f"[bench] tile solve: cycle {cycles}, iters {iters}, residual {worst:.3e}")

    ctx.set_progress(progress)
    full = args.tile_rhs >= 0
    if full:  # one right-hand side to the tolerance (the solver treats them independently)
        kh, po = kh[args.tile_rhs:args.tile_rhs + 1], po[args.tile_rhs:args.tile_rhs + 1]
    a0 = ctx.plane_wave_rhs(kh, po)
    restart = args.restart or cfg["restart"]
    prec = args.tile_precision if full else "mixed"
    x0 = None
    if full and args.tile_x0:  # resume from a saved iterate (exact on a restart-cycle boundary)
        x0 = torch.tensor(np.load(args.tile_x0), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t_start[0] = time.perf_counter()
    s, info = ctx.solve(a0, x0=x0, tol=cfg["tol"], restart=restart, precision=prec,
                        max_iter=args.tile_max_iter if full else args.tile_iters)
    if full and args.tile_save:
        np.save(args.tile_save, s.cpu().numpy())
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t_start[0]
    ctx.set_progress(None)
    # residual decade rate over the second half of the bounded run (per RHS the
    # history restarts; use the last RHS's records)
    last = [h for h in hist if h[1] > 0][-max(2, len(hist) // 4):]
    extrap = None
    if len(last) >= 2 and last[-1][2] < last[0][2]:
        its = last[-1][1] - last[0][1]
        decades = np.log10(last[0][2] / last[-1][2])
        remaining = max(0.0, np.log10(last[-1][2] / cfg["tol"]))
        it_total = info[-1]["iters"] + remaining / decades * its
        sec_per_iter = t_solve / max(1, sum(i["iters"] for i in info))
        extrap = {"iters_per_rhs_est": it_total, "time_to_solution_s_est": it_total * sec_per_iter * R,
                  "sec_per_iteration": sec_per_iter, "basis": "extrapolated from the bounded run"}
    log(f"[bench] tile {'full' if full else 'bounded'} solve {t_solve:.1f} s, info {info}, "
        f"extrapolation {extrap}")
    nf = None if full else near_field_plane(ctx, s, cfg)
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": mv["mixed"]["avg_launch_ms"], "unit": "ms per c64 block matvec (2 RHS)",
           "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": mv["mixed"]["avg_launch_ms"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
           "data": "synthetic", "config": {"workload": cfg["name"], "scatterers": N, "lmax": lmax, "rhs": R,
                                           "restart": restart},
           "table_build_s": t_table, "matvec": mv,
           "bounded_solve": None if full else {"max_iter": args.tile_iters, "time_s": t_solve, "info": info},
           "solve_one_rhs": {"rhs": args.tile_rhs, "precision": prec, "resumed": bool(args.tile_x0),
                             "max_iter": args.tile_max_iter, "time_s": t_solve, "info": info}
           if full else None,
           "time_to_solution_extrapolated": None if full else extrap, "near_field": nf,
           "roofline": {"bound": "mfma", "achieved": mv["mixed"]["tflops"], "peak": PEAK_FP32_MFMA,
                        "unit": "TFLOP/s", "frac": mv["mixed"]["frac"], "traffic": None,
                        "kernel": kernel_name(fixed["mixed"][0], "float")}}
    print(json.dumps(out), flush=True)
    ctx.close()


def near_field_plane(ctx, s, cfg):
    """Scattered field on the n x n plane of the workload (FP32 basis, FP64
    phase reduction), timed with HIP events around the readout call."""
    import torch

    import workloads as wl

    n_side, extent, z = cfg["plane"]
    pts = torch.tensor(wl.near_field_plane(n_side, extent, z), dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.near_field(s, pts[:1024], "mixed")
    ev0.record()
    E = ctx.near_field(s, pts, "mixed")
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    R = s.shape[0]
    pairs = pts.shape[0] * ctx.n * R
    kernel = f"near_field_v2<float, {ctx.lmax}, {R}>"
    ipp = nf_valu_per_pair(kernel)
    roof = None
    if ipp is not None:
        achieved = pts.shape[0] * ctx.n * ipp / (ms * 1e-3)
        roof = {"bound": "alu", "kernel": kernel, "valu_lane_instr_per_pair": ipp,
                "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_INSTR / 1e12,
                "unit": "T VALU lane-instructions/s", "frac": achieved / PEAK_VALU_LANE_INSTR}
    log(f"[bench] near field {n_side}x{n_side}: {ms:.1f} ms, {pairs / ms / 1e6:.3g} G pair-rhs/s, "
        f"VALU issue {roof['frac'] if roof else None}")
    return {"points": pts.shape[0], "ms": ms, "pair_rhs_per_s": pairs / ms * 1e3,
            "max_abs": float(E.abs().max()), "roofline": roof}


def bench_cylinders(args):
    """100 x 100 lattice of silicon cylinders at lmax 6 (9.6e5 unknowns, dense
    null-field T per cylinder).  One step is the sphere workloads' step with
    the T-matrices built by the null-field kernel: translation table, T,
    plane-wave right-hand side, mixed-precision GMRES to 1e-8 and the far
    field.  Then the lmax-6 block matvec in isolation in both precisions."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    pos, radii, kh, po, cfg = wl.config_inputs("cyl6")
    n, lmax, R = cfg["nx"], cfg["lmax"], len(kh)
    height, n_rel = cfg["cylinders"]
    N = n * n
    tol = cfg["tol"]
    restart = args.restart or cfg["restart"]
    ctx = tmhip.Context(0)
    radii_d = torch.tensor(radii, dtype=torch.float64, device="cuda")
    dirs = torch.tensor([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], dtype=torch.float64, device="cuda")
    ctx.set_geometry(pos, wl.K, lmax)
    log(f"[bench] cylinders: N={N}, lmax={lmax}, L={ctx.L}, restart {restart}")
    tuned = tune_matvec(ctx, args, R)

    def progress(cycles, iters, n_live, worst):
        if cycles % 5 == 0:
            log(f"[bench] cycle {cycles}, iters {iters}, residual {worst:.2e}")

    ctx.set_progress(progress)

    def step(precision):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_geometry(pos, wl.K, lmax)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.set_cylinders(radii_d, height, n_rel)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        a0 = ctx.plane_wave_rhs(kh, po)
        s, info = ctx.solve(a0, tol=tol, restart=restart, precision=precision, inner_tol=1e-4,
                            max_iter=args.cyl_max_iter)
        F = ctx.far_field(s, dirs)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return s, info, F, {"table_s": t1 - t0, "tmatrix_s": t2 - t1, "rhs_solve_farfield_s": t3 - t2}

    for w in range(args.warmup):
        _, info, _, ph = step("mixed")
        log(f"[bench] warmup {w}: {info[0]}, {ph}")
    copy_calibration(torch)
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s, info, F, ph = step("mixed")
        log(f"[bench] step {k}: {info[0]}, {ph}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.profile_enable(False)
    live = {}
    for which, prec, peak in ((1, "mixed", PEAK_FP32_MFMA), (0, "fp64", PEAK_FP64_MFMA)):
        ms, launches, flops = ctx.profile_query(which)
        if launches:
            avg = ms / launches / 1e3
            live[prec] = {"avg_launch_ms": avg * 1e3, "launches": launches, "flops_per_launch": flops,
                          "tflops": flops / avg / 1e12, "frac": flops / avg / 1e12 / peak}
    ctx.profile_reset()
    ctx.set_progress(None)
    log(f"[bench] cylinders time-to-solution {dt:.3f} s/step, matvec {live}")
    mv = isolated_matvec(ctx, R, args.matvec_reps)
    dom = live.get("mixed", mv["mixed"])
    variant = ctx.get_matvec_config("mixed")[0]
    knames = kernel_names(variant, "float")
    if n % 16 == 0:
        knames = knames[:1]
    L = ctx.L
    alg_bytes = (2 * n - 1) ** 2 * (L * L // 2) * 8 + 2 * N * L * 8
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64+f64", "data": "synthetic",
           "config": {"workload": cfg["name"], "scatterers": N, "lmax": lmax, "unknowns": N * L,
                      "rhs": R, "tol": tol, "restart": restart, "precision": "mixed",
                      "scatterer": "silicon cylinder, null-field T"},
           "solve_info": info[0], "phases_s": ph, "autotuned": tuned,
           "matvec_timed_region": live, "matvec_isolated": mv,
           "matvec_algorithmic_GBps": alg_bytes / (dom["avg_launch_ms"] / 1e3) / 1e9,
           "roofline": {"bound": "mfma", "achieved": dom["tflops"], "peak": PEAK_FP32_MFMA,
                        "unit": "TFLOP/s", "frac": dom["tflops"] / PEAK_FP32_MFMA,
                        "mfma_issue_frac": dom["tflops"] * mfma_issue_ratio(lmax) / PEAK_FP32_MFMA,
                        "effective_ceiling_tflops": PEAK_FP32_MFMA / mfma_issue_ratio(lmax),
                        "traffic": measured_traffic(knames, cfg["name"]),
                        "kernel": " + ".join(knames), "avg_launch_ms": dom["avg_launch_ms"],
                        "flops_per_launch": dom["flops_per_launch"],
                        "kernel_source_digest": kernel_source_digest()}}
    print(json.dumps(out), flush=True)
    ctx.close()


OL_SOURCE = "paper_2107_09879_amd/csrc/tm_offlattice.hip"


def ol_valu_per_pair(kernel):
    """VALU lane-instructions per (target, source) pair and right-hand side of
    the off-lattice kernel from the committed counter summary, or None if the
    source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "offlattice_matvec_100x100_lmax3.md")
    if not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, OL_SOURCE), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    with open(path) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 3 and cells[0] == kernel and cells[1] == digest:
                try:
                    return float(cells[2])
                except ValueError:
                    return None
    return None


def bench_offlattice(args):
    """100 x 100 lattice with every site jittered in-plane (the 100 x 100
    workload's spheres): no two pairs share a displacement, so the translation
    blocks are formed on the fly per (target, source) pair.  One step = the
    lattice workload's step (geometry, Mie, RHS, mixed GMRES(50) to 1e-8, far
    field); then the off-lattice operator in isolation in both precisions,
    the complex64 one against the FP32 VALU issue peak."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    pos, radii, kh, po, cfg = wl.config_inputs("offl")
    n, lmax, R = cfg["nx"], cfg["lmax"], len(kh)
    N = n * n
    restart = args.restart or cfg["restart"]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, wl.K, lmax)
    if ctx.get_lattice()[2] != 0.0:
        raise RuntimeError("the jittered workload was taken for a lattice")
    radii_d = torch.tensor(radii, dtype=torch.float64, device="cuda")
    dirs = torch.tensor([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], dtype=torch.float64, device="cuda")
    log(f"[bench] off-lattice: N={N}, lmax={lmax}, restart {restart}")

    def progress(cycles, iters, n_live, worst):
        if cycles % 5 == 0:
            log(f"[bench] cycle {cycles}, iters {iters}, residual {worst:.2e}")

    ctx.set_progress(progress)

    def step():
        ctx.set_geometry(pos, wl.K, lmax)
        ctx.set_spheres(radii_d, wl.N_REL)
        a0 = ctx.plane_wave_rhs(kh, po)
        s, info = ctx.solve(a0, tol=cfg["tol"], restart=restart, precision="mixed", inner_tol=1e-4,
                            max_iter=args.offl_max_iter)
        F = ctx.far_field(s, dirs)
        return s, info, F

    for w in range(args.warmup):
        _, info, _ = step()
        log(f"[bench] warmup {w}: {info[0]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s, info, F = step()
        log(f"[bench] step {k}: {info[0]}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.set_progress(None)
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.normal(size=(R, N, ctx.L)) + 1j * rng.normal(size=(R, N, ctx.L)),
                     dtype=torch.complex128, device="cuda")
    op = {}
    for prec in ("mixed", "fp64"):
        ctx.apply_operator(x, "forward", prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.matvec_reps):
            ctx.apply_operator(x, "forward", prec)
        torch.cuda.synchronize()
        op[prec] = {"ms": (time.perf_counter() - t1) / args.matvec_reps * 1e3}
        log(f"[bench] off-lattice {prec} operator: {op[prec]['ms']:.2f} ms")
    kernel = (f"offlattice_small_kernel<float, {lmax}, false>" if lmax <= 3
              else f"offlattice_mid_kernel<float, {lmax}, false>")
    ipp = ol_valu_per_pair(kernel)
    roof = None
    if ipp is not None:
        achieved = N * (N - 1) * R * ipp / (op["mixed"]["ms"] * 1e-3)
        roof = {"bound": "alu", "kernel": kernel, "valu_lane_instr_per_pair": ipp,
                "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_INSTR / 1e12,
                "unit": "T VALU lane-instructions/s", "frac": achieved / PEAK_VALU_LANE_INSTR,
                "timing": "host clock around the operator (kernel + combine), device synchronised"}
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64+f64", "data": "synthetic",
           "config": {"workload": cfg["name"], "scatterers": N, "lmax": lmax, "unknowns": N * ctx.L,
                      "rhs": R, "tol": cfg["tol"], "restart": restart, "precision": "mixed"},
           "solve_info": info[0], "operator_isolated": op, "roofline": roof}
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_batched(args):
    """Overlapping square subregions (side 20-80 plus a 10-site buffer) of a
    300 x 300 lens layout, 4 right-hand sides each, solved as one batch
    (restart cycles replayed from a hipGraph) and, for comparison, one
    subregion at a time with the single-system solver (tables built outside
    the timed region).  --subregions K keeps the first K of the 48."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    cfg = wl.CONFIGS["c3"]
    pos, radii, kh, po, _ = wl.config_inputs("c3")
    subs = [(ox, oy, sd, sd) for ox, oy, sd in wl.subregions(seed=cfg["seed"])]
    if args.subregions:
        subs = subs[:args.subregions]
    R = len(kh)
    max_iter = 20000
    restart = args.restart or cfg["restart"]

    def progress(tag):
        last = [time.perf_counter()]

        def fn(cycles, iters, n_live, worst):
            now = time.perf_counter()
            if cycles % 10 == 0 or now - last[0] > 20.0:
                last[0] = now
                log(f"[bench] {tag}: cycle {cycles}, iters {iters}, live {n_live}, max residual {worst:.2e}")
        return fn

    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, wl.K, cfg["lmax"])
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device="cuda"), wl.N_REL)
    ctx.set_batch_autotune(not args.no_batch_autotune)
    res = {}
    precs = ["mixed"] if args.no_fp64 else ["mixed", "fp64"]
    for prec in precs:
        ctx.set_progress(progress(f"batched {prec}"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sb, info = ctx.solve_batched(subs, kh, po, use_graph=True, tol=cfg["tol"],
                                     restart=restart, precision=prec, max_iter=max_iter)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flat = [i for row in info for i in row]
        pf, items = ctx.batch_config(prec)
        res[prec] = {"time_s": dt, "graph": ctx.batch_graph_used(),
                     "launch": {"autotuned": not args.no_batch_autotune, "prefetch": pf,
                                "items_per_rhs_class": items},
                     "iters_max": max(i["iters"] for i in flat),
                     "iters_mean": float(np.mean([i["iters"] for i in flat])),
                     "converged": sum(i["status"] == 0 for i in flat), "systems": len(flat),
                     "max_rel_residual": max(i["rel_residual"] for i in flat),
                     "per_subregion": [{"box": list(q), "iters": [i["iters"] for i in row],
                                        "converged": all(i["status"] == 0 for i in row),
                                        "rel_residual": max(i["rel_residual"] for i in row)}
                                       for q, row in zip(subs, info)]}
        log(f"[bench] batched {prec}: {dt:.2f} s, {res[prec]['converged']}/{len(flat)} converged, "
            f"iters max {res[prec]['iters_max']} mean {res[prec]['iters_mean']:.0f}")
        for k, e in enumerate(res[prec]["per_subregion"]):
            if not e["converged"]:
                log(f"[bench] subregion {k} {e['box']} not converged: iters {e['iters']}, residual {e['rel_residual']:.2e}")
    ctx.set_progress(None)
    ctx.close()
    # the same systems one subregion at a time (R right-hand sides per solve)
    seq = {"time_s": 0.0, "table_build_s": 0.0, "iters_max": 0}
    for k, (ox, oy, sx, sy) in enumerate([] if args.no_sequential else subs):
        ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
        idx = (iy * cfg["nx"] + ix).ravel()
        one = tmhip.Context(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.set_geometry(pos[idx], wl.K, cfg["lmax"])
        torch.cuda.synchronize()
        seq["table_build_s"] += time.perf_counter() - t0
        one.set_spheres(torch.tensor(radii[idx], dtype=torch.float64, device="cuda"), wl.N_REL)
        one.set_progress(progress(f"subregion {k}"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a0 = one.plane_wave_rhs(kh, po)
        _, info = one.solve(a0, tol=cfg["tol"], restart=restart, precision="mixed",
                            max_iter=max_iter)
        torch.cuda.synchronize()
        seq["time_s"] += time.perf_counter() - t0
        seq["iters_max"] = max(seq["iters_max"], max(i["iters"] for i in info))
        log(f"[bench] subregion {k} ({sx}x{sy}) alone: {time.perf_counter() - t0:.2f} s, "
            f"iters {[i['iters'] for i in info]}")
        one.close()
    sites = sum(q[2] * q[3] for q in subs)
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": res["mixed"]["time_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": res["mixed"]["time_s"] * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
           "config": {"workload": cfg["name"], "subregions": len(subs), "sites": sites,
                      "rhs": R, "systems": len(subs) * R, "restart": restart},
           "batched": res, "sequential_mixed": None if args.no_sequential else seq,
           "batched_speedup_vs_sequential": None if args.no_sequential else seq["time_s"] / res["mixed"]["time_s"]}
    print(json.dumps(out), flush=True)


def bench_jinc_padding(args):
    """Padding study of App. II / Sec. 2 on one GPU: one jinc source below
    the centre of the 300 x 300 lens layout, solved on square subregions of
    growing side centred on it (all in one batched solve driven by the jinc
    expansion), and the scattered power (far field over the upper half space)
    and the near field 5 wavelengths above, each against the largest
    subregion."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    n, lmax = 300, 3
    pos = wl.lattice_positions(n, n)
    radii = wl.lens_radii(n)
    c0 = 149.5 * wl.PITCH
    halves = [2, 4, 6, 8, 12, 16, 24, 32, 48]
    subs = [(150 - h, 150 - h, 2 * h, 2 * h) for h in halves]
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, wl.K, lmax)
    ctx.set_spheres(torch.tensor(radii, dtype=torch.float64, device="cuda"), wl.N_REL)
    # far-field quadrature over the upper half space (Gauss-Legendre x trapezoid)
    xg, wg = np.polynomial.legendre.leggauss(48)
    th = np.arccos(0.5 * (xg + 1.0))  # cos(theta) in (0, 1)
    ph = np.arange(96) * 2 * np.pi / 96
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    wq = (0.5 * wg[:, None] * np.full(96, 2 * np.pi / 96)[None, :]).ravel()
    dirs_d = torch.tensor(dirs, dtype=torch.float64, device="cuda")
    g = np.linspace(-6.0, 6.0, 9)
    X, Y = np.meshgrid(c0 + g, c0 + g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 5.0)], -1)
    pts_d = torch.tensor(pts, dtype=torch.float64, device="cuda")
    rows = []
    total = 0.0
    for z0 in (-0.5, -3.0, -6.0):
        src = (c0, c0, z0, 1.0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a0 = ctx.jinc_rhs_batched(subs, [[[src]] for _ in subs])
        sb, info = ctx.solve_batched_a0(subs, a0, 1, use_graph=True, tol=1e-10, restart=200,
                                        precision="mixed", max_iter=20000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total += dt
        powers, fields = [], []
        for (ox, oy, sx, sy), s_k in zip(subs, sb):
            full = torch.zeros(1, n * n, ctx.L, dtype=torch.complex128, device="cuda")
            ix, iy = np.meshgrid(np.arange(ox, ox + sx), np.arange(oy, oy + sy))
            idx = torch.tensor((iy * n + ix).ravel(), device="cuda")
            full[0, idx] = s_k[0]
            F = ctx.far_field(full, dirs_d)[0].cpu().numpy()
            powers.append(float(np.sum(wq * np.sum(np.abs(F) ** 2, axis=1))))
            fields.append(ctx.near_field(full, pts_d)[0].cpu().numpy())
        ref_p, ref_e = powers[-1], fields[-1]
        for h, (sx_), p_, e_, inf in zip(halves, subs, powers, fields, info):
            rows.append({"z0": z0, "side": 2 * h, "side_wavelengths": 2 * h * wl.PITCH,
                         "scattered_power": p_,
                         "power_rel_err": abs(p_ - ref_p) / abs(ref_p),
                         "near_field_rel_err": float(np.linalg.norm(e_ - ref_e) / np.linalg.norm(ref_e)),
                         "iters": inf[0]["iters"], "converged": inf[0]["status"] == 0})
            log(f"[bench] jinc z0={z0}: side {2 * h:3d} ({2 * h * wl.PITCH:5.1f} wl) power {p_:.6e} "
                f"err {rows[-1]['power_rel_err']:.2e} near-field err {rows[-1]['near_field_rel_err']:.2e} "
                f"iters {inf[0]['iters']}")
        log(f"[bench] jinc z0={z0}: batched solve of {len(subs)} subregions {dt:.2f} s")
    ctx.close()
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": total, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": total * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
           "data": "synthetic",
           "config": {"workload": "jinc-source padding study on the 300x300 lens layout", "lmax": lmax,
                      "sides": [2 * h for h in halves], "source_heights": [-0.5, -3.0, -6.0],
                      "tol": 1e-10, "restart": 200},
           "padding_study": rows}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """150 x 150 lattice: forward solve, detector objective |E|^2 50 wavelengths
    above the centre, adjoint solve and radius gradient; central differences
    on a few seeded radii from warm-started FP64 solves."""
    import torch

    import workloads as wl
    from paper_2107_09879_amd import tmhip

    pos, radii, kh, po, cfg = wl.config_inputs("c4")
    xd = np.array(cfg["detector"])
    ctx = tmhip.Context(0)
    ctx.set_geometry(pos, wl.K, cfg["lmax"])
    for prec in ("mixed", "fp64"):
        ms, conf = ctx.autotune(1, prec)
        log(f"[bench] autotune {prec}: {ms:.3f} ms, variant {conf[0]}, items {conf[1]}")
    rd = torch.tensor(radii, dtype=torch.float64, device="cuda")
    tag = {"name": "forward"}

    def progress(cycles, iters, n_live, worst):
        if cycles % 10 == 0:
            log(f"[bench] {tag['name']}: cycle {cycles}, iters {iters}, residual {worst:.2e}")

    ctx.set_progress(progress)

    def objective(r_dev, tol, x0=None):
        ctx.set_spheres(r_dev, wl.N_REL)
        a0 = ctx.plane_wave_rhs(kh, po)
        s, info = ctx.solve(a0, x0=x0, tol=tol, precision="mixed", max_iter=20000)
        z = np.array([torch.sum(ctx.detector_vector(xd, np.eye(3)[c]) * s[0]).item() for c in range(3)])
        Et = po[0] * np.exp(1j * wl.K * kh[0] @ xd) + z
        return float(np.sum(np.abs(Et) ** 2)), s, a0, Et, info

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    O, s, a0, Et, info_f = objective(rd, 1e-12)
    w = ctx.detector_vector(xd, np.conj(Et))
    tag["name"] = "adjoint"
    mu, info_a = ctx.adjoint_solve(w[None].contiguous(), tol=1e-12, precision="mixed", max_iter=20000)
    g = ctx.grad_radius(mu, s, a0)[0].cpu().numpy()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    log(f"[bench] forward+adjoint+gradient {t_grad:.2f} s, O={O:.6e}, fwd {info_f[0]}, adj {info_a[0]}")
    # in-plane position gradient from the same two solutions (coupling, incident and detector
    # terms); the first call also builds the four FP64 derivative tables
    gpos = {}
    for key in ("first_call_s", "s"):
        if key == "s":
            ctx.profile_reset()
            ctx.profile_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.grad_position(mu, s, a0, khat=kh, xd=xd, w=np.conj(Et)[None])
        torch.cuda.synchronize()
        gpos[key] = time.perf_counter() - t1
    ctx.profile_enable(False)
    ms, launches, flops = ctx.profile_query(0)
    if launches:
        avg = ms / launches / 1e3
        gpos["derivative_matvecs"] = {"launches": launches, "avg_launch_ms": avg * 1e3,
                                      "tflops": flops / avg / 1e12,
                                      "frac": flops / avg / 1e12 / PEAK_FP64_MFMA}
    ctx.profile_reset()
    log(f"[bench] position gradient {gpos}")
    idx = np.random.default_rng(5).choice(len(radii), 20, replace=False)[: max(1, args.steps)]
    fd = []
    h = 1e-6
    for i in idx:
        vals = []
        for sg in (1, -1):
            r2 = rd.clone()
            r2[i] += sg * h
            tag["name"] = f"FD radius {i} {'+' if sg > 0 else '-'}"
            vals.append(objective(r2, 1e-13, x0=s)[0])
        fd.append((vals[0] - vals[1]) / (2 * h))
        log(f"[bench] FD radius {i}: adjoint {g[i]:.8e} fd {fd[-1]:.8e}")
    fd = np.array(fd)
    err = float(np.max(np.abs(fd - g[idx])) / np.max(np.abs(g)))
    out = {"metric": "time-to-solution at 1e-8 residual + translation-matvec GB/s, 1e4-1e5 scatterers",
           "value": t_grad, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": t_grad * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
           "data": "synthetic", "config": {"workload": cfg["name"], "scatterers": len(radii),
                                           "solves": "mixed precision, FP64 true residual 1e-12"},
           "objective": O, "forward": info_f[0], "adjoint": info_a[0],
           "fd_check": {"indices": idx.tolist(), "step": h, "max_err_rel_to_max_grad": err},
           "position_gradient": gpos}
    print(json.dumps(out), flush=True)
    ctx.close()


def host_cpu():
    """nproc (CPUs this process may run on) and the lscpu model name."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except Exception:
        nproc = os.cpu_count()
    model = None
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return {"nproc": nproc, "cpu_model": model}


def mfma_issue_ratio(lmax):
    """Issued matrix-core flops per algorithmic flop of the complex64 block
    matvec: per 16 target sites, displacement and class the kernel issues
    (S/16)^2 x 4 x 3 MFMA 16x16x4 instructions (complex products from three
    real products, S = padded class size) of 2048 flops each, against
    16 x (L/2)^2 x 8 algorithmic flops."""
    L = 2 * lmax * (lmax + 2)
    S = 16 * ((L // 2 + 15) // 16)
    hw = (S // 16) ** 2 * 4 * 3 * 2048
    alg = 16 * (L // 2) ** 2 * 8
    return hw / alg


def cpu_baseline(pos, radii, kh, po, cfg, gpu_info):
    """The oracle on the host cores: one FP64 matrix-free matvec at the full
    workload, timed, times the number of FP64-equivalent matvecs the GPU solve
    needed (extrapolated solve time)."""
    import oracle

    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    host = host_cpu()
    n = cfg["nx"]
    lmax = cfg["lmax"]
    t0 = time.perf_counter()
    lc = oracle.LatticeCoupling(n, n, 0.6, 2 * np.pi, lmax)
    t_setup = time.perf_counter() - t0
    L = oracle.n_coeffs(lmax)
    x = np.random.default_rng(1).normal(size=(n * n, L)) + 0j
    # bounded sample: every third displacement, scaled by the exact share of
    # (target, source) pairs it covers
    pairs = (n - np.abs(lc.dxy[:, 0])) * (n - np.abs(lc.dxy[:, 1]))
    keep = np.arange(len(lc.dxy)) % 3 == 0
    frac = pairs[keep].sum() / pairs.sum()
    lc.dxy, lc.blk = lc.dxy[keep], lc.blk[keep]
    t0 = time.perf_counter()
    lc.apply(x)
    t_mv = (time.perf_counter() - t0) / frac
    matvecs = gpu_info["matvecs_fp64"] + gpu_info["matvecs_lowp"]
    est = t_setup + t_mv * matvecs
    log(f"[bench] oracle: block setup {t_setup:.1f} s, one FP64 matvec {t_mv:.1f} s "
        f"(from a {frac:.1%} sample), x {matvecs} matvecs")
    return {"value": est, "unit": "s", "cores": cores, "kind": "oracle", **host,
            "sample": f"oracle FP64 matvec at this workload timed on every third lattice "
                      f"displacement ({frac:.1%} of the pairs) and scaled to one full matvec "
                      f"({t_mv:.2f} s), plus the per-displacement block setup ({t_setup:.2f} s), "
                      f"extrapolated to the {matvecs} matvecs the GPU solve used"}


if __name__ == "__main__":
    main()
