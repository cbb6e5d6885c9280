"""Sanitizer builds of the host code (CPU only): the FP64 oracle under
AddressSanitizer + UndefinedBehaviorSanitizer (tests/cpu/oracle_sanitize.cpp
drives every entry point on a small instance), and the serving scheduler
(csrc/admission.h, driven by tests/cpu/sched_test.cpp with mock jobs) under
ASan + UBSan and under ThreadSanitizer.  ThreadSanitizer uses the LLVM
runtime of the ROCm toolchain: GCC 11's does not intercept
pthread_cond_clockwait (std::condition_variable::wait_until), which makes it
report impossible races (two threads holding one mutex)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPU = os.path.join(ROOT, "tests", "cpu")
CSRC = os.path.join(ROOT, "paper_2507_19276_amd", "csrc")
ASAN_UBSAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _build_run(compiler, flags, sources, timeout=300):
    exe = os.path.join(tempfile.mkdtemp(), "san")
    subprocess.run([compiler, "-std=c++17", "-O1", "-g", "-pthread"] + flags + sources + ["-o", exe], check=True,
                   capture_output=True, timeout=600)
    return subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=ENV)


def test_oracle_asan_ubsan():
    r = _build_run("g++", ASAN_UBSAN + ["-fopenmp", "-ffp-contract=off"],
                   [os.path.join(CPU, "oracle_sanitize.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp")])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]


def test_scheduler_asan_ubsan():
    r = _build_run("g++", ASAN_UBSAN + ["-I", CSRC], [os.path.join(CPU, "sched_test.cpp")])
    assert r.returncode == 0 and "fifo done=30 inorder=1" in r.stdout, r.stderr[-4000:]


def test_scheduler_tsan():
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        clang = shutil.which("clang++")
    if clang is None:
        pytest.skip("no clang++ with a ThreadSanitizer runtime")
    r = _build_run(clang, ["-fsanitize=thread", "-I", CSRC], [os.path.join(CPU, "sched_test.cpp")])
    assert r.returncode == 0 and "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "fifo done=30 inorder=1" in r.stdout
