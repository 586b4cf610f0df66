"""Build libswscan.so (HIP for gfx950) from csrc/ with hipcc.

Every translation unit is compiled in parallel into _build/, then linked into
the package directory.  ``build()`` always recompiles (it is the "does it
build" check); ``build(incremental=True)`` skips up-to-date objects.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswscan.so")
# the VALU issue-rate probe (a measurement aid) is a library of its own
PROBE_SRC = "valu_probe.hip"
PROBE_LIB = os.path.join(HERE, "libswprobe.so")
ARCH = "gfx950"

SOURCES = ["sw_shared_i16.hip", "sw_shared_i32.hip", "sw_pair_i16.hip", "sw_pair8_i16.hip",
           "sw_pair_i32.hip",
           "sw_launch.hip", "sw_runtime.cpp", "sw_devplan.cpp", "sw_starts.cpp", "sw_trace.hip", "sw_api.cpp", "sw_server.cpp", "sw_tune.cpp",
           "sw_noalloc.hip", "sw_swap.hip", "sw_trplan.hip"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         # packed FP32 VALU forms are kept out of every code object
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall", "-Wno-unused-function"]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "sw.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, incremental: bool, hdr_mtime: float) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) >= max(os.path.getmtime(path), hdr_mtime):
        return obj
    cmd = ["hipcc", "-x", "hip"] + FLAGS + ["-c", path, "-o", obj + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(obj + ".tmp", obj)
    return obj


def build(incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hdr = _headers_mtime()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs) + 1, max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental, hdr), srcs + [PROBE_SRC]))
    _link(objs[-1:], PROBE_LIB, [])
    objs = objs[:-1]
    _link(objs, LIB, ["-lpthread"])
    return LIB


def _link(objs, lib, extra):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + extra
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, lib)


if __name__ == "__main__":
    inc = "--incremental" in sys.argv
    print(build(incremental=inc))
