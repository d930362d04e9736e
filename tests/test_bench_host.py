"""Host-side checks of bench.py's bookkeeping (no GPU needed): the hash that
keys the stored counter profile to the kernel code ignores comments and
whitespace but not code, and it matches the stored profile's hash; the
roofline takes the nearer of the VALU-issue and HBM roofs; FP32 errors are
measured against the flow speed."""
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


def test_stored_counters_match_the_kernel_code():
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["kernel_hash"] == bench.kernel_hash()
    k = t["kernels"]["k_march2/fp64"]
    assert k["algorithmic_bytes_per_launch"] == 2 * 256 * 4096 * 1024
    assert 0 < k["hbm_bytes_per_launch"] < k["algorithmic_bytes_per_launch"]
    assert k["valu_insts_per_launch"] > 0
    for key in ("k_march/fp64", "k_march2/fp32", "k_march/fp32"):
        assert t["kernels"][key]["hbm_bytes_per_launch"] > 0


def test_roofline_takes_the_nearer_roof(monkeypatch, tmp_path):
    # a launch of 0.25 ms moving 1.0e9 bytes (4 TB/s, half the HBM peak) and
    # issuing 1.2e8 VALU instructions (0.78 of the VALU issue peak): VALU-bound
    ctr = {"kernel_hash": bench.kernel_hash(), "kernels": {"k_march2/fp64": {
        "hbm_bytes_per_launch": 1.0e9, "valu_insts_per_launch": 1.2e8}}}
    f = tmp_path / "c.json"
    f.write_text(json.dumps(ctr))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    res = {"steps_per_launch": 2, "nodes": 4096 * 1024, "kernel_ms_avg": 0.125, "clock_mhz": 2000.0}
    r = bench.roofline(res, "fp64")
    assert r["bound"] == "alu" and abs(r["frac"] - 1.2e8 / 0.25e-3 / bench.VALU_PEAK) < 1e-3
    assert abs(r["hbm_measured"]["frac"] - 0.5) < 1e-3
    assert abs(r["hbm_effective"]["GBs"] - 2 * 256 * 4096 * 1024 / 0.25e-3 / 1e9) < 0.1
    # the clock estimate is reported, nothing is derived from it
    assert r["core_clock_mhz_estimate"] == 2000.0 and set(r["valu"]) == {"insts_per_launch", "per_s", "frac"}
    # with few VALU instructions the HBM roof is the nearer one
    ctr["kernels"]["k_march2/fp64"]["valu_insts_per_launch"] = 1.0e7
    f.write_text(json.dumps(ctr))
    assert bench.roofline(res, "fp64")["bound"] == "hbm"
    # counters of other code are not used
    ctr["kernel_hash"] = "0" * 16
    f.write_text(json.dumps(ctr))
    r = bench.roofline(res, "fp64")
    assert r["traffic"] is None and r["valu"] is None and "note" in r


def test_macro_errors_use_the_flow_speed():
    import numpy as np
    ref = (np.ones((2, 3)), np.full((2, 3), 0.1), np.zeros((2, 3)), np.ones((2, 3)))
    got = (ref[0], ref[1] + 1e-6, ref[2], ref[3])
    e = bench.macro_errors(got, ref, 1.4)
    assert abs(e["ux"][1] - 1e-5) < 1e-12 and e["uy"][1] == 0.0
    # a fluid at rest falls back to the sound speed
    still = (ref[0], np.zeros((2, 3)), ref[2], ref[3])
    e = bench.macro_errors((ref[0], still[1] + 1e-6, ref[2], ref[3]), still, 1.4)
    assert abs(e["ux"][1] - 1e-6 / 1.4 ** 0.5) < 1e-12


def test_fetch_bytes_are_scaled_by_the_initialisation_kernel(tmp_path):
    """FETCH_SIZE is scaled so that the FP64 initialisation of the
    4096 x 1024 grid reads its 32 B per node; WRITE_SIZE by the plain
    copy's writes.  Synthetic counter files: the copy reads 1/2.667 of its
    bytes on FETCH_SIZE and the initialisation 1/2 of its own."""
    import csv
    import bench

    def write(d, rows):
        os.makedirs(os.path.join(d, "x"))
        with open(os.path.join(d, "x", "pmc_counter_collection.csv"), "w", newline="") as fh:
            w = csv.writer(fh)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writerows(rows)

    gib, nodes = 1 << 30, 4096 * 1024
    pair = "void (anonymous namespace)::k_march2<0, double>(double const*, double*)"
    init = "void (anonymous namespace)::k_init<double>(double*)"
    write(tmp_path / "f", [(1, "copy", "FETCH_SIZE", gib / 1024 / 2.667), (2, init, "FETCH_SIZE", 32 * nodes / 1024 / 2),
                           (3, pair, "FETCH_SIZE", 300000.0)])
    write(tmp_path / "w", [(1, "copy", "WRITE_SIZE", gib / 1024), (2, init, "WRITE_SIZE", 128 * nodes / 1024),
                           (3, pair, "WRITE_SIZE", 500000.0)])
    write(tmp_path / "s", [(3, pair, "SQ_INSTS_VALU", 1e8), (3, pair, "SQ_WAVES", 1936.0),
                           (3, pair, "GRBM_GUI_ACTIVE", 4e6)])
    out = bench.summarize_profile(tmp_path / "f", tmp_path / "w", tmp_path / "s", tmp_path / "o.json")
    assert abs(out["fetch_calibration"]["fetch_factor"] - 2.0) < 1e-12
    assert abs(out["copy_calibration"]["fetch_factor"] - 2.667) < 1e-9
    assert out["fetch_calibration"]["write_over_expected"] == 1.0
    k = out["kernels"]["k_march2/fp64"]
    assert k["fetch_bytes_per_launch"] == round(300000.0 * 1024 * 2.0)
    assert k["write_bytes_per_launch"] == round(500000.0 * 1024)


def test_summarize_counters_means_per_dispatch(tmp_path):
    """--summarize-counters: each counter summed over a dispatch's rows,
    then averaged over the dispatches of each step kernel; other kernels
    (a copy) are left out."""
    import csv
    import bench

    d = tmp_path / "s"
    os.makedirs(d / "x")
    pair = "void (anonymous namespace)::k_march2<0, double>(double const*, double*)"
    one = "void (anonymous namespace)::k_march<0, double>(double const*, double*)"
    with open(d / "x" / "pmc_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows([(1, pair, "SQ_WAVES", 1000.0), (1, pair, "SQ_WAVES", 936.0), (2, pair, "SQ_WAVES", 1936.0),
                     (1, pair, "SQ_WAIT_ANY", 5.0), (2, pair, "SQ_WAIT_ANY", 7.0),
                     (3, one, "SQ_WAVES", 992.0), (4, "copy", "SQ_WAVES", 64.0)])
    out = bench.summarize_counters([d])
    assert set(out) == {"k_march2<0, double>", "k_march<0, double>"}
    assert out["k_march2<0, double>"]["SQ_WAVES"] == 1936.0
    assert out["k_march2<0, double>"]["SQ_WAIT_ANY"] == 6.0
    assert out["k_march2<0, double>"]["dispatches"] == 2
    assert out["k_march<0, double>"]["SQ_WAVES"] == 992.0
