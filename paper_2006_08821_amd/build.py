"""Build the EMU shared library (HIP for gfx950 + host C++) in-tree.

    python -m paper_2006_08821_amd.build      # writes paper_2006_08821_amd/libemu.so

Host sources are compiled with g++, HIP sources with hipcc for gfx950; the
shared library is linked with hipcc.  Every call rebuilds from source.

HIP code is compiled with `-ffp-contract=on`: a multiply is fused into an add
only within one source expression, chosen by the front end.  With the default
(`fast`) the back end picks which product of `a*b + c*d` to fuse per inlining
context, so the single-mesh and batched wrappers of one device body could
round differently.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libemu.so")

HOST_SRC = ["host_setup.cpp", "api_host.cpp"]
HIP_SRC = ["kernels.hip", "api.hip", "serve.hip"]
ARCH = os.environ.get("EMU_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = "/opt/rocm/lib"  # roctx ranges (rocprofiler-sdk-roctx)


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    out_dir = tempfile.mkdtemp(prefix="emu_build_")
    try:
        jobs = []
        objs = []
        for s in HOST_SRC:
            o = os.path.join(out_dir, s + ".o")
            objs.append(o)
            jobs.append(["g++", "-std=c++17", "-O3", "-fPIC", "-mavx2", "-mfma", "-pthread",
                         "-Wall", "-Wno-unused-function", "-c", os.path.join(CSRC, s), "-o", o])
        for s in HIP_SRC:
            o = os.path.join(out_dir, s + ".o")
            objs.append(o)
            jobs.append([hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
                         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                         "-munsafe-fp-atomics", "-ffp-contract=on", "-c", os.path.join(CSRC, s), "-o", o])
        with ThreadPoolExecutor(max_workers=4) as ex:
            logs = list(ex.map(_run, jobs))
        if verbose:
            for lg in logs:
                if lg.strip():
                    print(lg)
        tmp_lib = LIB + ".tmp"
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp_lib] + objs +
             ["-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-lpthread"])
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(out_dir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
