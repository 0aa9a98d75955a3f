"""Build-level checks that need no GPU: the all-pairs repulsion kernel must
keep two waves per SIMD in every instantiation (at one wave per SIMD the
1M-point launch runs about 15 % slower), read from the compiler's own
resource-usage report of the gfx950 build."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_all_pairs_kernel_keeps_two_waves_per_simd(tmp_path):
    src = os.path.join(ROOT, "paper_2605_13928_amd", "csrc", "klgrad.hip")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src), "-c", src, "-o",
           str(tmp_path / "klgrad.o"), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    report = r.stderr
    occ = {}
    name = None
    for line in report.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"Occupancy \[waves/SIMD\]: (\d+)", line)
        if m and name:
            occ[name] = int(m.group(1))
    rep = {k: v for k, v in occ.items() if "rep_sym_kernel" in k}
    assert len(rep) == 9, sorted(occ)  # ZROW x superblock size {256, 512, 1024} x fused attraction
    assert all(v >= 2 for v in rep.values()), rep
