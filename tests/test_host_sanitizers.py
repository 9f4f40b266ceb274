"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (no
GPU): network builder, path finder (trials, reconfiguration, spatial
candidates), slicing and planner (budgets, term groups, checkpointing,
batches, MPO and state observables, geometric tensor plans, channel gates)
and the documented error paths, driven by csrc/host_check.cpp and built
with g++ (the host sources need no HIP)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_10091_amd", "csrc")
SOURCES = ["network.cpp", "path.cpp", "plan.cpp", "slice.cpp", "capi_host.cpp", "host_check.cpp"]
FLAGS = ["-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
         "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(["g++", *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        "-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True, text=True, timeout=600)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    exe = str(tmp_path / "host_check_asan")
    subprocess.run(["g++", *FLAGS, *objs, "-o", exe, "-lpthread"],
                   check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host check ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
