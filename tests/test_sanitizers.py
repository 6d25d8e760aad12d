"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU.

* The oracle (oracle/oracle.c) with gcc and a driver of exactly known cases
  (tests/native/oracle_sanitize.c).
* The library's host code: csrc/*.hip built by hipcc with the sanitizers on
  the host side only (-Xarch_host), the per-S pair-GEMM kernels replaced by
  host stand-ins, linked with a driver that calls the entry points with
  arguments their checks reject before any GPU call
  (tests/native/runtime_sanitize.cpp).  No GPU is needed.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2510_04795_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, "%s\n%s%s" % (" ".join(cmd), p.stdout[-4000:], p.stderr[-4000:])
    return p


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-fopenmp", "-ffp-contract=off", "-fno-fast-math", os.path.join(NATIVE, "oracle_sanitize.c"), "-o", exe,
         "-lm"])
    p = run([exe], env=dict(ENV, OMP_NUM_THREADS="4"))
    assert "all checks passed" in p.stdout


def hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
def test_host_runtime_under_sanitizers(tmp_path):
    srcs = [s for s in sorted(glob.glob(os.path.join(CSRC, "*.hip"))) if "pairgemm_s" not in os.path.basename(s)]
    srcs += [os.path.join(NATIVE, "runtime_sanitize.cpp"), os.path.join(NATIVE, "pair_stubs.cpp")]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Wno-unused-result", "-Wno-unused-value", "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run([hipcc()] + flags + ["-x", "hip", "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "runtime_san")
    # the link pulls in the host sanitizer runtimes; device code is built without them
    run([hipcc(), "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined"] + objs + ["-o", exe])
    p = run([exe], env=ENV)
    assert "all checks passed" in p.stdout
