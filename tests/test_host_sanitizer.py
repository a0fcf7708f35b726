"""The library's host side under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): rpod_abi.cpp and warm_abi.cpp compiled host-only with both
sanitizers, linked against host stand-ins for the HIP runtime calls and the
kernel launchers (tests/host_sanitizer/stubs.cpp), and driven through the C
ABI (tests/host_sanitizer/driver.cpp): the autotuner in every storage type,
plain, batched, centred, adaptive and warm plans. Any sanitizer report, a
failing call, a malformed launch record or a leaked stream, event or graph
fails the test."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = [os.path.join(ROOT, "paper_2504_15350_amd", "csrc", "rpod_abi.cpp"),
           os.path.join(ROOT, "paper_2504_15350_amd", "csrc", "warm_abi.cpp"),
           os.path.join(HERE, "host_sanitizer", "stubs.cpp"),
           os.path.join(HERE, "host_sanitizer", "driver.cpp")]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="hipcc / clang++ not installed")
def test_host_side_is_clean_under_asan_and_ubsan(tmp_path):
    flags = ["-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out
    exe = str(tmp_path / "driver")
    link = subprocess.run([CLANG, "-fsanitize=address,undefined", *objs, "-o", exe], capture_output=True, text=True)
    assert link.returncode == 0, link.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=str(tmp_path))
    report = run.stdout + run.stderr
    assert run.returncode == 0 and "PASSED" in run.stdout, report[-4000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-4000:]
    shutil.rmtree(tmp_path, ignore_errors=True)
