"""Host-side helpers of bench.py (no GPU): the kernel-code identity that keys
the stored counter figures, and the one-iteration baseline configuration."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2002_12115_amd import hj  # noqa: E402


def test_code_identity_ignores_comments_and_layout_only():
    a = 'int f(int x) { // twice\n  return 2 * x; /* doubled */ }\nconst char* s = "// kept";\n'
    b = 'int f(int x)\n{\n    return 2 * x;   // note\n}\nconst char* s = "// kept";'
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(a) != bench.code_only(a.replace("2 * x", "3 * x"))
    assert bench.code_only(a) != bench.code_only(a.replace('"// kept"', '"// changed"'))
    assert "'/'" in bench.code_only("char c = '/'; // slash")


def test_kernel_hash_covers_the_kernel_sources():
    assert len(bench.kernel_hash()) == 16
    assert all(os.path.exists(os.path.join(ROOT, p)) for p in bench.KERNEL_SOURCES)


def test_one_iteration_baseline_config():
    c = bench.one_iteration_config(hj, "f64", (130, 130, 258))
    assert (c["tsteps"], c["kernel"], c["bj"], c["vec"], c["ichunk"]) == (1, hj.KERNEL_MARCH, 4, 2, 2)
    c = bench.one_iteration_config(hj, "f32", (20, 30, 40))
    assert (c["tsteps"], c["bj"], c["vec"], c["ichunk"]) == (1, 8, 4, 1)


def test_roofline_counts_each_array_once_per_pass():
    # 8 M cells, two iterations per launch, FP64, 0.1 ms per launch
    r = bench.roofline(8, 8_000_000, 2, 0.1, None)
    assert r["algorithmic_bytes_per_launch"] == 14 * 8 * 8_000_000
    assert abs(r["achieved"] - 14 * 8 * 8e6 / 1e-4 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / bench.PEAK_HBM_GBPS) < 1e-12
    assert r["lattice_updates_per_launch"] == 16_000_000
    assert abs(r["per_update_equiv_gbps"] - 2 * r["achieved"]) < 1e-6
    assert r["measured_gbps"] is None and r["measured_frac"] is None
    m = bench.roofline(8, 8_000_000, 2, 0.1, 1.08 * 14 * 8 * 8_000_000)
    assert abs(m["traffic_over_algorithmic"] - 1.08) < 1e-12
    assert abs(m["measured_frac"] - 1.08 * m["frac"]) < 1e-12


def _counter_csv(path, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_ingest_counters_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    """Counter bytes are the per-dispatch mean, scaled by what the counter read
    for the copy kernel over a known size, times the launches per pass; the
    entry carries the profiled run's configuration and the kernel-code key."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    kern = "void hj::wide_kernel<double, 8, false, true>(hj::Grid<double>, ...)"
    copy = "hj::copy_kernel(unsigned int __vector(4) const*, ...)"
    # 1 GiB copy: FETCH reads half (64 B per 128 B request), WRITE reads all
    _counter_csv(str(tmp_path / "f" / "host" / "fetch_counter_collection.csv"),
                 [(kern, "FETCH_SIZE", 100.0), (kern, "FETCH_SIZE", 300.0), (copy, "FETCH_SIZE", 524288.0)])
    _counter_csv(str(tmp_path / "w" / "host" / "write_counter_collection.csv"),
                 [(kern, "WRITE_SIZE", 50.0), (kern, "WRITE_SIZE", 50.0), (copy, "WRITE_SIZE", 1048576.0)])
    cfg = {"kernel": 1, "bj": 8, "vec": 2, "ichunk": 32, "tsteps": 2}
    (tmp_path / "run.json").write_text("noise\n" + __import__("json").dumps({"config": {"kernel_config": cfg}}) + "\n")
    e = bench.ingest_counters("medium_f64", "wide_kernel<double, 8", str(tmp_path / "f"), str(tmp_path / "w"),
                              str(tmp_path / "run.json"), 1 << 30, per_pass=3)
    assert e["fetch_bytes"] == 200 * 1024 * 2 * 3 and e["write_bytes"] == 50 * 1024 * 3
    assert e["bytes_per_launch"] == e["fetch_bytes"] + e["write_bytes"]
    assert e["config"] == cfg and e["kernel_hash"] == bench.kernel_hash() and e["dispatches"] == [2, 2]
    assert bench.load_traffic("medium_f64", cfg) == e["bytes_per_launch"]
    assert bench.load_traffic("medium_f64", dict(cfg, bj=4)) is None
