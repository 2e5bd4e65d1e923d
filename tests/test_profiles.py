"""The committed profiler summaries: each states the commands that produced it, and those commands
run committed files only (bench.py under rocprofv3, the program directly after `--`); each HBM
counter summary has its machine-readable twin with sane calibration factors."""
import glob
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def commands(text: str) -> list:
    m = re.search(r"```\n(.*?)\n```", text, re.S)
    assert m, "no command block"
    return [line for line in m.group(1).splitlines() if line.strip()]


def test_every_summary_names_the_commands_that_made_it():
    assert PROFILES
    for p in PROFILES:
        lines = commands(open(p).read())
        prof = [c for c in lines if "rocprofv3" in c]
        assert prof, p
        for c in lines:
            assert "_work" not in c, (p, c)
        for c in prof:
            after = c.split(" -- ", 1)[1].split()
            assert after[0] in ("python3", "python") and after[1].endswith("bench.py"), (p, c)
            assert os.path.exists(os.path.join(ROOT, "bench.py"))


def test_counter_summaries_are_calibrated_against_a_copy():
    for j in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.json"))):
        d = json.load(open(j))
        assert os.path.exists(j[:-5] + ".md"), j
        assert 1.9 < d["fetch_scale"] < 2.1 and 0.95 < d["write_scale"] < 1.05, j
        assert d["traffic_bytes"] > d["algorithmic_bytes"] > 0, j   # halo re-reads only add
        assert d["code_sha256"] and len(d["code_sha256"]) == 64, j


def test_alu_side_of_the_roofline_comes_from_the_committed_counters():
    """bench.py's roofline.alu: FP32 flops from the committed VALU mix (64 lanes x (add + mul +
    2 fma) per issued instruction) over the launch time, and the VALU issue rate against one wave64
    instruction per SIMD every 4 cycles at 2.4 GHz; both between 0 and 1 of their peaks."""
    import importlib.util
    import sys
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    def trace_mean_us(workload):   # the field kernel's mean launch time in that workload's trace
        for p in PROFILES:
            t = open(p).read()
            if "--kernel-trace" in t and f"--workload {workload} " in t:
                for line in t.splitlines():
                    if line.startswith("| `void lbk::k_fused"):
                        return float(line.split("|")[4])
        raise AssertionError(f"no kernel trace of {workload}")

    for j in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_sq_counters.json"))):
        d = json.load(open(j))
        shape = {"threads": d["launch"]["threads"], "seg_rows": d["launch"]["seg_rows"]}
        a = b.counted_alu(d["workload"], shape, trace_mean_us(d["workload"]))
        if d["code_sha256"] != b.kernel_code_digest():
            assert a is None, j
            continue
        c = d["counters"]
        assert a["fp32_flops_per_launch"] == 64 * (c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"]
                                                   + 2 * c["SQ_INSTS_VALU_FMA_F32"]), j
        assert 0 < a["frac"] < a["frac_of_nonpacked"] < 1 and 0 < a["valu_issue"]["frac"] < 1, (j, a)
        assert b.VALU_ISSUE_PEAK_G == 614.4
