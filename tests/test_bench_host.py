"""Host-side checks of bench.py's bookkeeping (no GPU needed): the hash that
keys the stored traffic counters to the kernel code ignores comments and
whitespace but not code, and it matches the stored counters' hash."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_tokens_ignore_comments_and_spacing():
    a = 'int a = 1; // one\n/* two\n lines */\nconst char* s = "x // y";\n'
    b = 'int a = 1;\n\n// a changed comment\n// on two lines\nconst char* s =   "x // y";'
    assert bench.code_tokens(a, "//") == bench.code_tokens(b, "//")
    # code, and comment markers inside string literals, still count
    assert bench.code_tokens(a, "//") != bench.code_tokens(a.replace("= 1", "= 2"), "//")
    assert bench.code_tokens(a, "//") != bench.code_tokens(a.replace('"x // y"', '"x"'), "//")
    p = 'x = ["-O3"]  # flags\ns = "a # b"\n'
    assert bench.code_tokens(p, "#") == bench.code_tokens('x = ["-O3"]\n# other\ns = "a # b"', "#")
    assert bench.code_tokens(p, "#") != bench.code_tokens(p.replace("-O3", "-O2"), "#")


def test_stored_traffic_matches_the_kernel_code():
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["kernel_hash"] == bench.kernel_hash()
    assert t["algorithmic_bytes_per_launch"] == 2 * 256 * 4096 * 1024
    assert 0 < t["hbm_bytes_per_launch"] < t["algorithmic_bytes_per_launch"]
