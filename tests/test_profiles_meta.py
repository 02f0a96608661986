"""The committed profile summaries (CPU): each gives the command that made it,
and that command runs committed files only."""
import glob
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_profile_summaries_name_their_commands():
    mds = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert mds
    for p in mds:
        text = open(p).read()
        cmds = re.findall(r"```\n(.*?)```", text, flags=re.S)
        assert cmds, p
        for block in cmds:
            for line in [x for x in block.strip().splitlines() if x.strip()]:
                assert "rocprofv3" in line or "bench.py" in line, (p, line)
                assert "_work" not in line, (p, line)
                for script in re.findall(r"\$GRAFT_REPO_ROOT/(\S+\.py)", line):
                    assert os.path.exists(os.path.join(ROOT, script)), (p, script)


def test_counter_files_carry_the_kernel_hash():
    for p in glob.glob(os.path.join(ROOT, "profiles", "edge_pass_*_counters.json")):
        d = json.load(open(p))
        assert len(d["kernel_hash"]) == 16 and d["hbm_bytes_per_launch"] > 0, p
