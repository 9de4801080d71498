"""The library's host code (plan building, batch and autotuner argument
handling) built with AddressSanitizer and UndefinedBehaviorSanitizer and run
through tests/host_sanitize_driver.cpp: host-only plans over many geometries,
grids, tilings and flags with their tables checked, and the argument checks of
every entry point.  No GPU is used; the device launchers are stubs that abort."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_14906_amd", "csrc")
SOURCES = ["hodmas_host.cpp", "hodmas_batch.cpp", "hodmas_tune.cpp"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the ROCm headers")
def test_host_code_under_asan_and_ubsan(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = []
    for src in SOURCES + [os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")]:
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(tmp_path / (os.path.basename(path) + ".o"))
        subprocess.run(["g++"] + flags + ["-c", path, "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-fsanitize=address,undefined"] + objs +
                   ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
                    "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout)
    print(res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
