"""Host-side tools without a GPU: profiling summaries, training-problem
recipes, and the bench's argument contract."""
import csv
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2010_10232_amd import learned  # noqa: E402
from paper_2010_10232_amd import profiling  # noqa: E402


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_summary_calibration_and_hash(tmp_path):
    # copy of 256 MiB reads 0.5x on FETCH_SIZE and 1x on WRITE_SIZE; the kernel
    # reads 1000 KiB and writes 300 KiB per launch on average
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    _write_counters(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0), ("__amd_rocclr_copyBuffer", 3.0),
                                      ("void hh::arnoldi_reg_kernel<4>(...)", 900.0),
                                      ("void hh::arnoldi_reg_kernel<4>(...)", 1100.0),
                                      ("void hh::op_kernel<3, 3, 0, 1, double>(...)", 7.0)])
    _write_counters(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0),
                                      ("void hh::arnoldi_reg_kernel<4>(...)", 300.0)])
    s = profiling.summarize(str(f), str(w), "arnoldi_reg_kernel", 256)
    assert s["n_fetch"] == 2 and s["n_write"] == 1
    assert abs(s["f_fetch"] - 0.5) < 1e-12 and abs(s["f_write"] - 1.0) < 1e-12
    assert abs(s["traffic"] - 1024.0 * (1000.0 / 0.5 + 300.0)) < 1e-6
    out = tmp_path / "arnoldi_x_traffic.md"
    profiling.write_summary(str(out), "arnoldi_reg_kernel", "x", "cmd", s)
    got = profiling.read_summary(str(out))
    assert got is not None and abs(got[0] - s["traffic"]) < 1.0 and got[1] == "arnoldi_reg_kernel"
    # a summary taken from other sources is not reported
    text = out.read_text().replace(profiling.source_hash(), "0" * 64)
    out.write_text(text)
    assert profiling.read_summary(str(out)) is None
    assert profiling.read_summary(str(tmp_path / "missing.md")) is None


def test_traffic_summary_grid_filter(tmp_path):
    # one kernel template on two levels (grid sizes 26112 and 6656): only the
    # finest level's dispatches count; the calibration copy counts whatever its grid
    def write(path, counter, rows):
        with open(path, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for name, g, v in rows:
                w.writerow({"Kernel_Name": name, "Grid_Size": g, "Counter_Name": counter, "Counter_Value": v})
    op = "void hh::op_direct_kernel<3, 3, 0, 1, double>(...)"
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    write(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072, 131072.0), (op, 26112, 600.0), (op, 26112, 800.0),
                            (op, 6656, 5000.0)])
    write(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 131072, 262144.0), (op, 26112, 400.0), (op, 6656, 9000.0)])
    s = profiling.summarize(str(f), str(w), "op_direct_kernel<3, 3, 0", 256, grid=26112)
    assert s["n_fetch"] == 2 and s["n_write"] == 1
    assert abs(s["traffic"] - 1024.0 * (700.0 / 0.5 + 400.0)) < 1e-6
    every = profiling.summarize(str(f), str(w), "op_direct_kernel<3, 3, 0", 256)
    assert every["n_fetch"] == 3 and every["traffic"] > s["traffic"]


def test_kernel_table_of_one_phase(tmp_path):
    # dispatches after the last training kernel only
    t = tmp_path / "trace.csv"
    with open(t, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, a, b in [("op_a", 0, 10), ("wgrad_kernel<32>", 20, 120), ("op_a", 130, 140),
                           ("wgrad_kernel<8>", 150, 200), ("fused", 210, 250), ("op_a", 260, 266), ("fused", 270, 300)]:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": b})
    rows = profiling.stats_from_trace(str(t), "wgrad_kernel")
    assert [r["Name"] for r in rows] == ["fused", "op_a"]
    assert rows[0]["Calls"] == "2" and float(rows[0]["TotalDurationNs"]) == 70.0
    assert abs(float(rows[0]["Percentage"]) - 100.0 * 70 / 76) < 1e-9
    out = tmp_path / "t.md"
    profiling.write_stats(None, "phase", "cmd", str(out), rows=rows)
    assert "| `fused` | 2 | 0.000 | 0.04 |" in out.read_text()
    # a kernel name the host's c++filt may not read (a bf16 parameter)
    nm = profiling._demangle("_ZN2hh16cnn_fused_kernelIfEEviiPKNS_2cxIT_EEPKdiPKfPKDF16bS9_S5_S2_PS3_i")
    assert "hh::cnn_fused_kernel" in nm and not nm.startswith("_Z")


def test_kernel_stats_table(tmp_path):
    p = tmp_path / "stats.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                                           "MinNs", "MaxNs", "StdDev"])
        w.writeheader()
        for i in range(25):
            w.writerow({"Name": f"void hh::k{i}(int)", "Calls": 2, "TotalDurationNs": 2000.0 * (25 - i),
                        "AverageNs": 1000.0 * (25 - i), "Percentage": 4.0, "MinNs": 1.0, "MaxNs": 2.0,
                        "StdDev": 0.0})
    out = tmp_path / "t.md"
    profiling.write_stats(str(p), "T", "cmd", str(out), top=18)
    lines = out.read_text().splitlines()
    rows = [ln for ln in lines if ln.startswith("| `")]
    assert len(rows) == 18 and rows[0].startswith("| `hh::k0`")
    assert any(ln.startswith("| (7 more kernels) | 14 |") for ln in lines)


def test_training_specs_seeded_and_in_range():
    a = learned.training_specs(n_problems=4, seed=7)
    b = learned.training_specs(n_problems=4, seed=7)
    assert [s["n_el"] for s in a] == [s["n_el"] for s in b]
    for s, t in zip(a, b):
        assert np.array_equal(s["k_elem"], t["k_elem"]) and s["x0"] == t["x0"]
        k = s["k_elem"]
        assert k.shape == (s["n_el"], s["n_el"])
        # k = kbar (1 + 0.3 g), g clipped to [-1, 1]; kbar within the draw range
        assert k.min() >= 0.7 * 100.0 / 0.7 - 1e-9 and k.max() <= 1.3 * 500.0 / 1.3 + 1e-9
        assert s["n_el"] <= 640
        # k_max h stays at or below the target resolution
        assert k.max() / s["n_el"] <= 0.625 + 1e-12


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_learned_specs_never_the_test_problem():
    bench = _bench_module()
    for name in ("mp2a_k100_p3_160", "grf_k300_p4_960", "wedge_k150_p3_480", "mp1b_k50_p2_80"):
        w = bench.WORKLOADS[name]
        specs = bench.learned_specs(w)
        again = bench.learned_specs(w)
        assert len(specs) == 2
        for s, t in zip(specs, again):
            assert s["x0"] == t["x0"] and s["n_el"] == w["n_el"] and s["p"] == w["p"]
            assert len(s["x0"]) == w["dim"]
            if "k_elem" in s:
                assert np.array_equal(s["k_elem"], t["k_elem"])
                assert not np.array_equal(s["k_elem"], bench.k_field(w))
            else:
                assert s["k"] == w["k"] and s["x0"] != tuple(w["x0"])


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_field_specs_span_k_100_500_on_the_application_grid():
    from paper_2010_10232_amd import workloads as W
    specs = learned.field_specs(48, 4, n_problems=3)
    test_field = W.grf_k(48, kbar=300.0, seed=0)
    for s in specs:
        k = s["k_elem"]
        assert s["n_el"] == 48 and s["p"] == 4 and k.shape == (48, 48)
        assert k.min() >= 100.0 - 1e-9 and k.max() <= 500.0 + 1e-9
        assert not np.array_equal(k / s["kbar"], test_field / 300.0)
        assert all(0.3 <= v <= 0.7 for v in s["x0"])


def test_bench_and_full_size_references_share_the_workload_options():
    """The full-size oracle references are taken with the options the bench times."""
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_full_size as MF
    bench = _bench_module()
    for name in ("grf_k300_p4_960", "wedge_k150_p2_480", "wedge_k150_p3_480", "wedge_k150_p4_480"):
        assert bench.WORKLOADS[name]["opts"] == MF.WORKLOADS[name]["opts"], name


def test_committed_traffic_summaries_match_the_current_sources():
    """Every HBM-traffic summary under profiles/ was taken on the sources it names:
    read_summary hands its figure to the bench only while their hash is unchanged,
    so a kernel edit without new counter runs shows up here rather than as a silent
    null in the bench line."""
    import glob
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md")))
    assert paths
    for path in paths:
        got = profiling.read_summary(path)
        assert got is not None, os.path.basename(path)
        assert got[0] > 0 and got[1]


def test_kernel_launches_by_shape(tmp_path):
    """--per-grid: one row per kernel and launch shape, only after the phase marker."""
    p = tmp_path / "trace.csv"
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Workgroup_Size_Y",
              "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    rows = [("hh::k(int)", 0, 100, 256, 2560), ("setup_end", 200, 210, 64, 64)]
    t = 1000
    for grid, dur in ((2560, 3000), (2560, 5000), (2560, 4000), (512, 700), (2560, 9000)):
        rows.append(("hh::k(int)", t, t + dur, 256, grid))
        t += 10000
    rows.append(("hh::other(int)", t, t + 50, 256, 256))
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for name, s, e, wg, grid in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e, "Workgroup_Size_X": wg,
                        "Workgroup_Size_Y": 1, "Workgroup_Size_Z": 1, "Grid_Size_X": grid, "Grid_Size_Y": 1,
                        "Grid_Size_Z": 1})
    got = profiling.grid_rows(str(p), "setup_end", r"hh::k\(")
    assert [(r["workgroups"], r["calls"]) for r in got] == [(10, 4), (2, 1)]
    assert got[0]["avg_us"] == 5.25 and got[0]["median_us"] == 5.0
    assert got[0]["min_us"] == 3.0 and got[0]["max_us"] == 9.0 and got[1]["avg_us"] == 0.7
    out = tmp_path / "g.md"
    profiling.write_grid_table(got, "T", "cmd", str(out))
    assert "| `hh::k` | 10 | 256 | 4 | 5.25 | 5.00 | 3.00 | 9.00 |" in out.read_text()
