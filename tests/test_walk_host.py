"""Culling walk (Section 3.2), host build: the library's hierarchical walk
(`vrt_cullwalk.h`, every cell-skip level) against the oracle's plain walk.

The walk header is compiled for the host with hipcc and linked with the
oracle's C source; `tests/walk_host_check.hip` draws random blocker fields,
start voxels, eyes and limits and counts mismatches of the blocking count.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and shutil.which("gcc")), reason="needs hipcc and gcc")
def test_walk_matches_oracle(tmp_path):
    orc = tmp_path / "oracle.o"
    exe = tmp_path / "walk_check"
    subprocess.run(["gcc", "-O2", "-c", os.path.join(ROOT, "oracle", "vrt_oracle.c"), "-o", str(orc)], check=True)
    subprocess.run([HIPCC, "-O2", "--offload-host-only", "-x", "hip",
                    "-I" + os.path.join(ROOT, "paper_2510_09081_amd", "csrc"),
                    os.path.join(ROOT, "tests", "walk_host_check.hip"), "-x", "none", str(orc), "-o", str(exe)],
                   check=True, capture_output=True)
    for seed in (1, 2):
        r = subprocess.run([str(exe), str(seed), "3000"], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and "bad=0" in r.stdout, r.stdout[-2000:]
