"""Host-side helpers of bench.py (no GPU): kernel naming and the gating of
the committed HBM-traffic figures by the matvec sources' digest."""
import subprocess
import sys

import bench

WL = "100x100 lattice, lmax 3 (3e5 unknowns)"


def test_kernel_names_follow_the_launch_configuration():
    assert bench.kernel_names(10, "float") == [
        "block_matvec_lds_kernel<float, 4, 16, 8, 3, false>",
        "block_matvec_lds_kernel<float, 4, 16, 8, 3, true>"]
    # the FP64 kernel caps the table prefetch depth at 2
    assert bench.kernel_names(10, "double") == bench.kernel_names(9, "double")
    assert bench.kernel_names(8, "double") == [
        "block_matvec_lds_kernel<double, 2, 8, 16, 1, false>",
        "block_matvec_lds_kernel<double, 2, 8, 16, 1, true>"]
    assert bench.kernel_names(5, "float") == ["block_matvec_kernel<float, true, false, 4>"]


def _write_summary(root, rows):
    d = root / "profiles"
    d.mkdir()
    lines = ["| kernel | workload | source digest | HBM bytes per launch |", "|---|---|---|---:|"]
    lines += [f"| {k} | {w} | {g} | {b} |" for k, w, g, b in rows]
    (d / "block_matvec_hbm_traffic.md").write_text("\n".join(lines) + "\n")


def test_traffic_is_summed_per_matvec_and_gated_by_digest(tmp_path, monkeypatch):
    reg, wide = bench.kernel_names(10, "float")
    _write_summary(tmp_path, [(reg, WL, "d1", 3.0e9), (wide, WL, "d1", 2.0e8),
                              (reg, "other workload", "d1", 1.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "d1")
    assert bench.measured_traffic([reg, wide], WL) == 3.2e9
    # a kernel without a row, another workload, or changed sources: no figure
    assert bench.measured_traffic(bench.kernel_names(8, "float"), WL) is None
    assert bench.measured_traffic([reg, wide], "other workload") is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "d2")
    assert bench.measured_traffic([reg, wide], WL) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
