"""Builds libsmcrt.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsmcrt.so")
SOURCES = [os.path.join(CSRC, f) for f in ("api.cpp", "walk.hip", "voxel.hip", "accel.hip", "static_run.hip", "serve.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("layout.h", "launch.h", "walk_common.h", "voxel_model.h")] + [
    os.path.join(os.path.dirname(HERE), "include", "smcrt.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


PROBE_SRC = os.path.join(CSRC, "atomic_ceiling.hip")
PROBE = os.path.join(HERE, "atomic_ceiling")


def build_probe(verbose=False):
    """The FP64 atomic-throughput microbenchmark (a measurement tool, not
    part of the library)."""
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", PROBE, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    return PROBE


def build(verbose=False, extra=()):
    cmd = ["hipcc", *FLAGS, *extra, "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(ln for ln in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in ln)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
    print(build_probe(verbose=True))
