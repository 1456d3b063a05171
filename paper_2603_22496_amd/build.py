"""Builds the in-tree native artefacts.

  libkk.so      C-ABI library: host half (kk_host.cpp, g++, FP64 with no contraction) and
                gfx950 kernels (*.hip, hipcc)
  phantom/_rfsim.so  forward model of the synthetic input generator (gcc)

Every call compiles (no up-to-date check); objects go to a scratch directory and the
shared libraries are replaced atomically.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkk.so")

HIP_SOURCES = ["kk_beamform.hip", "kk_fft.hip", "kk_decompose.hip", "kk_ensemble.hip", "kk_complete.hip",
               "kk_static.hip"]
HOST_SOURCES = ["kk_host.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-fno-gpu-rdc",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
              "-Wall", "-Wno-sign-compare"]


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build_libkk(verbose: bool = False, extra_hip_flags=()) -> str:
    tmp = tempfile.mkdtemp(prefix="kkbuild_")
    try:
        jobs = [["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(tmp, src + ".o")]
                for src in HOST_SOURCES]
        jobs += [[HIPCC, *HIP_FLAGS, *extra_hip_flags, "-c", os.path.join(CSRC, src), "-o", os.path.join(tmp, src + ".o")]
                 for src in HIP_SOURCES]
        objs = [j[-1] for j in jobs]
        with ThreadPoolExecutor(max_workers=min(len(jobs), max(1, min(8, os.cpu_count() or 1)))) as ex:
            for out in ex.map(_run, jobs):
                if verbose and out.strip():
                    print(out)
        tmp_lib = os.path.join(tmp, "libkk.so")
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib, "-lgomp"])
        shutil.copy2(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


def build_all(verbose: bool = False) -> None:
    from .phantom import build_rfsim
    build_rfsim(force=True)
    build_libkk(verbose=verbose)


if __name__ == "__main__":
    build_all(verbose=True)
    print("built", LIB)
