"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer.

1. The library's host runtime (tt_channel.cpp, tt_server.cpp, tt_io.cpp:
   arena, admission and release, tap windows, Jakes anchor tables,
   descriptor building for every apply form and launch schedule, the serving
   loop, the host IQ pipeline) linked against a CPU model of the HIP runtime
   whose kernel launches check every descriptor and every span a kernel would
   touch (tests/host_model).  The driver also checks that every allocation
   is returned.
2. The FP64 oracle, built from the same source with both sanitizers, under
   its own pin tests (loaded through TT_ORACLE_LIB with the ASan runtime
   preloaded).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_08217_amd", "csrc")
MODEL = os.path.join(ROOT, "tests", "host_model")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _clean(out: str):
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]


def test_host_runtime_under_asan_ubsan(tmp_path):
    _need("g++")
    exe = str(tmp_path / "host_model")
    srcs = [os.path.join(CSRC, f) for f in ("tt_channel.cpp", "tt_server.cpp", "tt_io.cpp")]
    srcs += [os.path.join(MODEL, f) for f in ("hip_model.cpp", "driver.cpp")]
    cmd = (["g++", "-std=c++17", "-w", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + SAN + srcs + ["-o", exe, "-lpthread"])
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    _clean(out)
    assert "0 allocations live, 0 failures" in out, out[-4000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    _need("gcc")
    so = str(tmp_path / "libtt_oracle_asan.so")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared"] + SAN +
                   [os.path.join(ROOT, "oracle", "tt_oracle.c"), "-o", so, "-lm"],
                   check=True, capture_output=True, timeout=300)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), asan
    env = dict(os.environ, TT_ORACLE_LIB=so, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"],
                       capture_output=True, text=True, timeout=900, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    _clean(out)
    assert " passed" in out, out[-2000:]
