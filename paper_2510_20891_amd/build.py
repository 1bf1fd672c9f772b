"""Build libemri.so (HIP kernels for gfx950 + the C ABI) in place.

    python -m paper_2510_20891_amd.build

Every source is compiled with hipcc for gfx950 only; objects go to
paper_2510_20891_amd/_build and the shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libemri.so")
ARCH = "gfx950"

HIP_SOURCES = ["status.cpp", "sft.hip", "score.hip", "mixed.hip", "topk.hip", "api.hip", "batched.hip", "search.hip", "harmonics.hip", "chirp.hip", "rescore.hip"]
HOST_SOURCES = ["basis.cpp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _common_flags() -> list[str]:
    return ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-I", INCLUDE, "-I", CSRC]


def _hip_cmd(src: str, obj: str) -> list[str]:
    # packed FP32 VALU forms are disabled for all device code
    return [_hipcc(), f"--offload-arch={ARCH}", *_common_flags(),
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-x", "hip", "-c", src, "-o", obj]


def _host_cmd(src: str, obj: str) -> list[str]:
    return ["g++", *_common_flags(), "-c", src, "-o", obj]


def _run(cmd: list[str]) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    work = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        work.append((_hip_cmd(os.path.join(CSRC, src), obj), obj))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        work.append((_host_cmd(os.path.join(CSRC, src), obj), obj))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, cmd) for cmd, _ in work]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[o for _, o in work]])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
