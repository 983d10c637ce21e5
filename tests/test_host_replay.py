"""The library's index arithmetic replayed on the host under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU).

``tests/host_replay/replay.cpp`` is compiled with g++ together with the
library's planner (``csrc/plan.cpp``) and the index headers its kernels use
(``csrc/xform_index.hpp``, ``csrc/sk_index.hpp``; the HIP headers compile in
host mode).  It plans random contractions (every group kind, s, t or v = 0,
charge tables, subgroup modes, complex operands, every precision, fused and
three-step paths) plus the workloads' shapes, walks every access of the
transforms, the fused product's table offsets and load addresses, and the
stream-K and split-K partitions, and checks bounds, alignment, one write per
destination element and exact coverage.  Any failure, or any sanitizer report,
fails the test.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_08056_amd", "csrc")
ROCM_INCLUDE = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")


@pytest.mark.timeout(900)
def test_host_replay_under_sanitizers(tmp_path):
    gxx = shutil.which(os.environ.get("CXX", "g++"))
    if gxx is None or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "replay")
    build = [gxx, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE,
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             os.path.join(ROOT, "tests", "host_replay", "replay.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "400"], capture_output=True, text=True, timeout=800, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 failures" in r.stdout
    # the interleaved split-bf16 planes (forced wide tiles) were walked too
    m = re.search(r"(\d+) interleaved split-bf16 plane transforms", r.stdout)
    assert m and int(m.group(1)) > 0, r.stdout
    m = re.search(r"(\d+) split-bf16 plans reading U in place", r.stdout)
    assert m and int(m.group(1)) > 0, r.stdout
