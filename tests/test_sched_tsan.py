"""The request scheduler's host threads under ThreadSanitizer: the scheduler
source built for the CPU against a host stand-in of the HIP runtime (streams
are worker threads, events complete in stream order), with client threads
submitting, polling, waiting for and cancelling requests. No data race may be
reported and every request must end OK or cancelled, with its precoder written
before an OK result is published."""

import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_scheduler_threads_are_race_free():
    d = os.path.join(HERE, "sched_tsan")
    csrc = os.path.join(ROOT, "paper_2305_13925_amd", "csrc")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "sched_tsan")
        cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-I", d, "-I", os.path.join(ROOT, "include"),
               os.path.join(d, "driver.cpp"), os.path.join(d, "mock_hip.cpp"), os.path.join(csrc, "sched.cpp"),
               os.path.join(csrc, "tuner.cpp"), "-o", exe, "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
