"""The library's host-only code (layout-graph builder with several scan
threads, validation, simplification and split, recovery, tallies, the
server's range allocator) built with g++ under AddressSanitizer +
UndefinedBehaviorSanitizer and under ThreadSanitizer, driven by
tests/native/host_checks.cpp; the sanitizers turn any finding into a
non-zero exit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_14335_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "native", "host_checks.cpp"),
           os.path.join(CSRC, "frontend.cpp"), os.path.join(ROOT, "workload", "layoutgen.c")]


def build_and_run(tmp_path, flags, env_extra, sources=None, expect="host checks passed",
                  cxx=None):
    gxx = cxx or shutil.which("g++")
    if gxx is None or not os.path.exists(gxx):
        pytest.skip("compiler not found")
    exe = str(tmp_path / "host_checks")
    objs = []
    for src in sources or SOURCES:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        lang = ["-x", "c", "-std=c11"] if src.endswith(".c") else ["-x", "c++", "-std=c++17"]
        subprocess.run([gxx] + lang + ["-O1", "-g", "-fno-omit-frame-pointer", "-c", src,
                                       "-o", obj, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                       "-I", os.path.join(ROOT, "workload"),
                                       "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"] + flags,
                       check=True, capture_output=True, text=True)
        objs.append(obj)
    subprocess.run([gxx] + objs + ["-o", exe, "-lpthread", "-lm"] + flags, check=True,
                   capture_output=True, text=True)
    env = dict(os.environ)
    env.update(env_extra)
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert expect in out.stdout


def test_host_code_under_asan_ubsan(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                  {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})


def test_host_code_under_tsan(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=thread"],
                  {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})


SERVE_SOURCES = [os.path.join(ROOT, "tests", "native", "serve_double.cpp"),
                 os.path.join(CSRC, "serve_core.cpp"), os.path.join(CSRC, "frontend.cpp")]


# GCC 11's ThreadSanitizer does not intercept pthread_cond_clockwait, which
# libstdc++ uses for timed condition waits, and then reports a false double
# lock; the clang of the ROCm toolchain (host code only) intercepts it.
CLANG = "/opt/rocm/llvm/bin/clang++"


def test_server_core_under_tsan(tmp_path):
    """The server's scheduling core (tickets, workers, admission, ticks,
    shutdown) with a host-only double of its device executor, under
    ThreadSanitizer."""
    build_and_run(tmp_path, ["-fsanitize=thread"],
                  {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"},
                  sources=SERVE_SOURCES, expect="serve double passed", cxx=CLANG)


def test_server_core_under_asan_ubsan(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                  {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"},
                  sources=SERVE_SOURCES, expect="serve double passed")
