"""Sanitizer builds of the host code (CPU only): the FP64 oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, and the library's host layer (descriptor validation, workspace layout,
chunking, schedules, optimiser options) built with the host sanitizers (device code unchanged)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_oracle_clean_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
                    "-lm"])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "ERROR" not in out and "runtime error" not in out, out


def test_library_host_layer_clean_under_asan_ubsan(tmp_path):
    # every library source is compiled with the sanitizers on its host code only (each flag after
    # -Xarch_host; the gfx950 device code is unchanged), then linked by the host compiler with a
    # driver that exercises descriptor validation, layout, chunking, schedules and option checks
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not shutil.which("g++"):
        pytest.skip("hipcc or g++ missing")
    csrc = os.path.join(ROOT, "paper_2604_08463_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for src in ("cs_api", "cs_prep", "cs_eval", "cs_maps", "cs_kmeans", "cs_optim"):
        obj = str(tmp_path / f"{src}.o")
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *host_san,
                                       "-I", inc, "-I", csrc, "-c", os.path.join(csrc, src + ".hip"), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out
    exe = str(tmp_path / "host_driver")
    rc, out = _run(["g++", "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-I", inc,
                    "-o", exe, os.path.join(HERE, "host_driver.cpp"), *objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, out
    # the HIP runtime's own allocations at exit are not this code's: leak detection off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "all checks held" in out and "runtime error" not in out, out
