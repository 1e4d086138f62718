"""The host-side suites against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the library's host sources (planning, packing, extraction, layer
setup, the C-ABI argument checks): a heap overflow, use after free, signed
overflow, bad shift or divide by zero in that code fails here, on the CPU.
The sanitized library is built next to the regular one by the package build."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "_build_san", "libhe.so")
SUITES = ["tests/test_host_layer.py", "tests/test_plan_counts.py", "tests/test_abi.py"]


def _runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_sanitized_library_is_instrumented():
    if not os.path.exists(SAN_LIB):
        pytest.skip("sanitized library not built (paper_2409_16675_amd.build.build_sanitized())")
    blob = open(SAN_LIB, "rb").read()
    assert b"__asan_report_load8" in blob and b"__ubsan_handle_divrem_overflow" in blob


def test_host_suites_under_asan_and_ubsan():
    rt = _runtime()
    if not os.path.exists(SAN_LIB) or rt is None:
        pytest.skip("sanitized library or sanitizer runtime absent")
    env = dict(os.environ, LD_PRELOAD=rt, HE_LIBRARY=SAN_LIB, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = subprocess.run([sys.executable, "-c", "from paper_2409_16675_amd import he; print(he.LIB_PATH)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and probe.stdout.strip() == SAN_LIB, probe.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + SUITES,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert " passed" in r.stdout
