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
