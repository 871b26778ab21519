"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle over every regime and edge of the model, and the
library's host side (descriptor validation, workspace plans, threshold
tables, the gap lookup), each built with gcc/g++ -fsanitize=address,undefined
and run to completion with sanitizer errors fatal."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1603_09255_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1", "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "oracle", "spegg_oracle.c"),
                                     os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    r = run([exe], env=ENV)
    assert "oracle sanitizer driver ok" in r.stdout


def test_library_host_code_clean_under_sanitizers(tmp_path):
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not installed")
    kobj = os.path.join(ROOT, "_build", "kernels.hip.o")
    if not os.path.exists(kobj):
        from paper_1603_09255_amd.build import build
        build()
    objs = []
    flags = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
             "-I" + CSRC] + SAN
    for src in [os.path.join(CSRC, f) for f in ("tables.cpp", "spegg_capi.cpp", "spegg_server.cpp")] + \
               [os.path.join(HERE, "host_driver.cpp")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run(["g++"] + flags + ["-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    # the device kernels (and their launchers) come unsanitized from the
    # library's own build; no call of the driver reaches them
    run(["g++", "-fsanitize=address,undefined"] + objs + [kobj, "-L/opt/rocm/lib", "-lamdhip64",
                                                           "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = run([exe], env=ENV)
    assert "host sanitizer driver ok" in r.stdout
