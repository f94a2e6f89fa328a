"""The committed profile summaries: each one names the command that made it,
and that command runs files of this repository only (bench.py with a
workload it knows, or the peaks program), so a reader can rerun it."""
import glob
import json
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2310_10750_amd import synth  # noqa: E402

SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def _commands(text):
    """Command lines inside fenced blocks."""
    out = []
    for block in re.findall(r"```\n(.*?)```", text, flags=re.S):
        out += [ln.strip() for ln in block.splitlines() if ln.strip()]
    return out


def test_there_are_summaries():
    assert len(SUMMARIES) >= 8


@pytest.mark.parametrize("path", SUMMARIES, ids=[os.path.basename(p) for p in SUMMARIES])
def test_summary_names_a_rerunnable_command(path):
    text = open(path).read()
    cmds = _commands(text)
    assert cmds, "no command in %s" % path
    for c in cmds:
        assert "rocprofv3" in c or "nlch_peaks" in c, c
        if "rocprofv3" in c:
            # the profiled program follows "--" directly and is the benchmark
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] == "python3" and prog[1] == "$R/bench.py", c
            m = re.search(r"--workload (\w+)", c)
            assert m, c
            synth.workload(m.group(1), nsteps=1)  # a workload bench.py knows
            assert "--pmc" not in c or ("--sys-trace" not in c and "--kernel-trace" not in c), c
        else:
            exe = c.split("&&")[-1].split()
            assert any(os.path.basename(t) == "nlch_peaks" for t in exe), c
    assert os.path.exists(os.path.join(ROOT, "paper_2310_10750_amd", "peaks", "peaks.hip"))


def test_traffic_json_commands_are_counter_passes():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for e in d.values():
        cmds = list(e.get("commands", [])) + ([e["lds_command"]] if "lds_command" in e else [])
        assert cmds
        for c in cmds:
            assert "rocprofv3 --pmc" in c and "$R/bench.py" in c, c
