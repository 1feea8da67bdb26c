"""The host runtime (csrc/hm_runtime.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code, linked with the device objects of
the in-tree build, runs tests/host_sanitizer_driver.cpp: the C ABI's host-only
paths (workspace sizing, every argument check before a HIP call, status and
error strings, NULL handles). Runs on the CPU; device code is not
instrumented (no GPU sanitizer on this hardware)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2308_13476_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_2308_13476_amd", "_lib")
DEVICE_OBJECTS = ["hm_level.o", "hm_setup.o", "hm_tail.o", "hm_krylov.o"]


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    objs = [os.path.join(LIBDIR, o) for o in DEVICE_OBJECTS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("device objects not built (run __graft_entry__.build())")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    rt = tmp_path / "hm_runtime_san.o"
    drv = tmp_path / "driver.o"
    exe = tmp_path / "driver"
    subprocess.run([hipcc, "-x", "hip", "-c", os.path.join(CSRC, "hm_runtime.cpp"), "-o", str(rt)] + common + san,
                   check=True, capture_output=True)
    subprocess.run([hipcc, "-c", os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp"), "-o", str(drv),
                    "-std=c++17", "-O1", "-g", "-I", os.path.join(ROOT, "include")] + san, check=True,
                   capture_output=True)
    subprocess.run([hipcc, str(drv), str(rt)] + objs + ["-o", str(exe), "--offload-arch=gfx950"] + san,
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", HIP_VISIBLE_DEVICES="")
    res = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, (res.returncode, res.stderr[-4000:])
