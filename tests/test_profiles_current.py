"""The committed rocprofv3 summaries were taken on the current kernels: every
summary under profiles/ that names the hash of the sources it was taken on
matches those sources as they are now (the one-fluid step's code, or the
general step's headers), so a kernel change cannot leave a stale profile
behind."""
import glob
import hashlib
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_0442_amd", "csrc")


def _general_hash():
    h = hashlib.sha256()
    for f in ("lb2d_common.hpp", "lb2d_device.hpp", "lb2d_full.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def test_profiles_match_the_current_sources():
    import bench
    current = {bench.source_hash(), _general_hash()}
    seen = 0
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for h in re.findall(r"source:\s*([0-9a-f]{16})", open(path).read()):
            seen += 1
            assert h in current, f"{os.path.basename(path)} was taken on other sources ({h})"
    assert seen >= 8
