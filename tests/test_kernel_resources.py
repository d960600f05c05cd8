"""Build-time check of the HIP kernels (no GPU needed): hipcc's resource report must show no
private (scratch) memory in any kernel, so no kernel spills registers to HBM or keeps a
stack, and the hot kernels keep the occupancy they were designed for."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# kernel name fragment -> minimum waves per SIMD
MIN_OCCUPANCY = {"k_link_tiled": 5, "k_count": 8, "k_scatter": 8, "k_compress": 8}


def resources():
    from paper_2510_26851_amd import build as B

    out = {}
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_2510_26851_amd", "csrc", "*.hip"))):
        r = subprocess.run([HIPCC, *B.HIPFLAGS, "-c", src, "-o", os.devnull,
                            "-Rpass-analysis=kernel-resource-usage"],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        name = None
        for line in r.stderr.splitlines():
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                out[name] = {}
                continue
            m = re.search(r"(ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
            if m and name:
                out[name][m.group(1).split()[0]] = int(m.group(2))
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_no_scratch_and_hot_kernel_occupancy():
    res = resources()
    assert res, "no kernels reported"
    spills = {k: v["ScratchSize"] for k, v in res.items() if v.get("ScratchSize", 0)}
    assert not spills, spills
    for frag, occ in MIN_OCCUPANCY.items():
        hits = [v["Occupancy"] for k, v in res.items() if frag in k]
        assert hits and min(hits) >= occ, (frag, hits)
