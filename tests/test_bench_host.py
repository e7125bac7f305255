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
