"""Build libjacpcg.so for gfx950 with hipcc (in-tree).

    python -m paper_2305_13925_amd.build [--jobs N] [--debug]

Every .hip and .cpp file under csrc/ is compiled to an object in _build/ and
linked into paper_2305_13925_amd/libjacpcg.so. Packed-FP32 instructions are
disabled for all device code.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libjacpcg.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-std=c++17", "-fPIC", "-Wall", "-Werror", "-Wno-unused-result",
          f"-I{os.path.join(os.path.dirname(PKG), 'include')}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-file code generation choices. The FP64 kernels keep their matrix-core
# accumulators in ordinary VGPRs: with accumulation registers the compiler
# copied every accumulator between the two register files once per loop
# iteration, and waited for the products before each copy.
PER_FILE = {"refine.hip": ["-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form=1"]}


def _compile(src, opt):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, *PER_FILE.get(os.path.basename(src), []), opt, "-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature name and says so.
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return obj


def build(jobs=None, debug=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    opt = "-O1" if debug else "-O3"
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, opt), srcs))
    tmp = LIB + ".tmp"
    # roctx (rocprofiler-sdk) for the named host-side ranges of each phase
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
