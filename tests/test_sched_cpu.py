"""Admission policy of the request scheduler (host C++), built with g++ and run
on the CPU."""

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_sched_policy_host_checks():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sched_policy_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                        os.path.join(HERE, "sched_policy_check.cpp"), "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    assert "sched policy ok" in out
