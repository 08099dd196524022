"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (CPU only).

- The oracle (plain C) built with gcc's sanitizers and loaded into a Python
  process that calls every entry point on small inputs of the parity tests'
  shapes (tests/sanitize_oracle_run.py): any out-of-bounds access, overflow of
  a signed integer, shift out of range or misaligned load aborts the run.
- The culling walk's host build checked against the oracle's walk
  (tests/walk_host_check.hip), both compiled with clang's sanitizers; the
  device pass is not built (host-only compilation).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"


def _gcc_runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(not (shutil.which("gcc") and _gcc_runtime("libasan.so")), reason="needs gcc with libasan")
def test_oracle_under_asan_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-shared", "-fPIC", "-o", str(lib), os.path.join(ROOT, "oracle", "vrt_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, LD_PRELOAD=_gcc_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_oracle_run.py"), str(lib)],
                       capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.rstrip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and ROCm clang")
def test_walk_host_under_asan_ubsan(tmp_path):
    orc = tmp_path / "oracle.o"
    exe = tmp_path / "walk_check_san"
    san = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
    subprocess.run([CLANG, "-O1", "-g", "-std=gnu11", "-ffp-contract=off", *san, "-c",
                    os.path.join(ROOT, "oracle", "vrt_oracle.c"), "-o", str(orc)], check=True, capture_output=True)
    host_san = [a for f in san for a in ("-Xarch_host", f)]
    subprocess.run([HIPCC, "-O1", "-g", "--offload-host-only", "-x", "hip", *host_san,
                    "-I" + os.path.join(ROOT, "paper_2510_09081_amd", "csrc"),
                    os.path.join(ROOT, "tests", "walk_host_check.hip"), "-x", "none", str(orc), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe), "3", "3000"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert r.returncode == 0 and "bad=0" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
