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
