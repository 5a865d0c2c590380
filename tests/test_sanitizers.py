"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU (no GPU code is sanitized or run):

- the FP64 oracle built by gcc with both sanitizers, driven through its
  Python interface over runs, traces, the voxel model and voxelisation of
  every scene family, a vessel network and the random scenes;
- the library's host code (scene builder and validation, table packing,
  acceleration records, the request scheduler) built by hipcc with the
  sanitizers on the host side only, driving the host-side ABI tests and the
  packing of every scene through the device-less scheduler;
- a planted heap overflow in a scratch C file, which the same set-up must
  report, so that a clean run means something.

Each run is a child process with the sanitizer runtime preloaded; any
report ends it with a non-zero status."""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_08035_amd", "csrc")
SOURCES = ["api.cpp", "walk.hip", "voxel.hip", "accel.hip", "static_run.hip", "serve.hip"]

# sanitizer flags for hipcc: host side only (device code is built plain)
HOST_SAN = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
       "OMP_NUM_THREADS": "2"}


def _gcc_asan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc's AddressSanitizer runtime not found")
    return rt


def _child(code, preload, extra_env=None):
    env = dict(os.environ, LD_PRELOAD=preload, **ENV, **(extra_env or {}))
    return subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, capture_output=True, text=True,
                          timeout=900, cwd=ROOT)


def _reported(r):
    return r.returncode != 0 or "ERROR: AddressSanitizer" in r.stderr or "runtime error:" in r.stderr


@pytest.fixture(scope="module")
def oracle_san(tmp_path_factory):
    rt = _gcc_asan()
    out = str(tmp_path_factory.mktemp("san") / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fPIC", "-shared", "-o", out, os.path.join(ROOT, "oracle", "smcrt_oracle.c"), "-lm"],
                   check=True)
    return rt, out


def test_oracle_runs_clean_under_asan_and_ubsan(oracle_san):
    rt, lib = oracle_san
    r = _child(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import oracle.build as b
        b.LIB = {lib!r}
        b.is_stale = lambda: False
        from oracle import oracle as orc
        from paper_2112_08035_amd import workloads as W
        import numpy as np
        assert orc.lib()._name == {lib!r}
        for name, mk in W.WORKLOADS.items():
            d = mk(n_grid=8)
            orc.run(d, 1, 300)
            orc.trace(d, 1, 0, 50)
            orc.voxelize(d)
        d = W.vessel_scene(3, 1.0, n_caps=100, n_grid=8)
        orc.run(d, 1, 200)
        orc.run(d, 1, 200, voxel=True)
        for s in range(12):
            d = W.random_scene(s, n_grid=8)
            orc.run(d, 2, 200)
            orc.trace(d, 2, 1, 40)
            orc.segment_bound(d, 0, np.zeros(3), np.array([0.0, 0.0, 1.0]))
        print("clean")
    """, rt)
    assert not _reported(r) and "clean" in r.stdout, r.stderr[-4000:]


def test_planted_heap_overflow_is_reported(oracle_san, tmp_path):
    rt, _ = oracle_san
    src, lib = tmp_path / "planted.c", tmp_path / "libplanted.so"
    src.write_text("#include <stdlib.h>\n"
                   "int planted(int n) { int* a = malloc(sizeof(int) * n); a[n - 1] = 1;\n"
                   "  int s = a[n]; free(a); return s; }\n")
    subprocess.run(["gcc", "-O0", "-g", "-fsanitize=address", "-fPIC", "-shared", "-o", str(lib), str(src)], check=True)
    r = _child(f"""
        import ctypes
        print(ctypes.CDLL({str(lib)!r}).planted(16))
    """, rt)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, (r.returncode, r.stderr[-2000:])


def test_host_library_runs_clean_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not os.path.exists(hipcc) or not rts:
        pytest.skip("hipcc or clang's AddressSanitizer runtime not found")
    lib = str(tmp_path / "libsmcrt_san.so")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared", "-shared-libsan",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN
    cmd += ["-o", lib] + [os.path.join(CSRC, f) for f in SOURCES]
    subprocess.run(cmd, check=True, capture_output=True)
    env = {"SMCRT_LIB": lib}
    # the host-side ABI tests
    r = _child(f"""
        import sys
        import pytest
        sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", {os.path.join(ROOT, "tests", "test_abi_cpu.py")!r}]))
    """, rts[0], env)
    assert not _reported(r), (r.stdout[-3000:], r.stderr[-3000:])
    # every scene built, packed and scheduled by the device-less server
    r = _child(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        from paper_2112_08035_amd import smcrt as S, workloads as W
        assert S.LIB_PATH == {lib!r}
        descs = [mk(n_grid=8) for mk in W.WORKLOADS.values()]
        descs += [W.vessel_scene(3, 1.0, n_caps=200, n_grid=8), W.vessel_scene(4, 1.0, n_caps=50, n_grid=8)]
        descs += [W.random_scene(s, n_grid=8) for s in range(12)]
        descs += [dict(W.slab_scene(8), relax=1.9), dict(W.sphere_scene(8), segment=True)]
        sv = S.Server(device=-1, hbm_budget_bytes=1 << 30, epoch_packets=1000)
        ids = [sv.submit(S.Scene(d), i, 2000)[0] for i, d in enumerate(descs)]
        for rid in ids:
            sv.wait(rid, 60.0)
        assert all(sv.poll(r)[0] == "DONE" for r in ids)
        sv.close()
        print("clean")
    """, rts[0], env)
    assert not _reported(r) and "clean" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
