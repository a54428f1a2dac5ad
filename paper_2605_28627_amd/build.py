"""Build of the HIP library libdgx.so for gfx950 (in-tree).

Each kernel translation unit is compiled by hipcc into an object (the
residual kernels once per polynomial degree, in parallel), then everything
is linked into paper_2605_28627_amd/libdgx.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgx.so")
CHECK_LIB = os.path.join(HERE, "libdgx_pointwise_check.so")
BUILD = os.path.join(HERE, "_build")
DEGREES = range(1, 8)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


def _compile(src, obj, extra=()):
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, defines=(), out: str | None = None, build_dir: str | None = None) -> str:
    """Compile and link libdgx.so (defines: extra -D options, e.g. tuning switches)."""
    bdir = build_dir or BUILD
    os.makedirs(bdir, exist_ok=True)
    dflags = tuple(f"-D{d}" for d in defines)
    units = [(os.path.join(CSRC, "dgx_host.cpp"), os.path.join(bdir, "dgx_host.o"), dflags),
             (os.path.join(CSRC, "dgx_launch.hip"), os.path.join(bdir, "dgx_launch.o"), dflags)]
    for n in DEGREES:
        units.append((os.path.join(CSRC, "dgx_inst.hip"), os.path.join(bdir, f"dgx_inst_N{n}.o"),
                      (f"-DDGX_INST_N={n}",) + dflags))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(*u), units))
    target = out or LIB
    tmp = target + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, target)
    if out is None:
        build_pointwise_check()
    return target


def build_pointwise_check() -> str:
    """Host build of the point physics and its VJPs, for the CPU test suite."""
    tmp = CHECK_LIB + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-I", os.path.join(HERE, "..", "include"), os.path.join(CSRC, "dgx_pointwise_check.cpp"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host build of the point physics failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CHECK_LIB)
    return CHECK_LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build())
