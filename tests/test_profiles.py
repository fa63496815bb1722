"""The committed rocprofv3 summaries describe the kernels as they are: each names
the sha256 of the kernel source it was taken on, which must be the current one,
and gives the command that made it (committed files only)."""
import glob
import json
import os
import re

from paper_2208_13770_amd.profile_summary import kernel_hash

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_step_kernel_traffic_taken_on_the_current_source():
    t = json.load(open(os.path.join(PROFILES, "k_step_M2_traffic.json")))
    assert t["kernel_sha256_16"] == kernel_hash()
    assert "k_step" in t["kernel"] and t["bytes_per_launch"] > 0
    for cmd in t["commands"].values():
        assert "rocprofv3 --pmc" in cmd and "bench.py" in cmd and "_work" not in cmd


def test_summaries_name_the_current_source_and_their_command():
    mds = glob.glob(os.path.join(PROFILES, "*.md"))
    assert mds
    for path in mds:
        text = open(path).read()
        m = re.search(r"Kernel source sha256\[:16\]: ([0-9a-f]{16})", text)
        assert m and m.group(1) == kernel_hash(), path
        cmds = re.findall(r"Command: `([^`]*)`", text)
        assert cmds, path
        for c in cmds:
            assert "rocprofv3" in c and "_work" not in c, (path, c)
