"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only, no device).

* The library's host code that runs without a device -- the sequence
  compiler (compile_sequence, plan_slices, assign_shape_slots,
  narrow_rotations) and the K-t spin-spacing calculator (ps_kt_extent) --
  built with g++ -fsanitize=address,undefined into tests/host_sanitize.cpp,
  a driver that feeds them seeded random sequences, valid and corrupted,
  and checks the compiler's output invariants.
* The C oracle built the same way and loaded (through PS_ORACLE_LIB, with
  the ASan runtime preloaded) by its own pin tests in a subprocess.

Any sanitizer report aborts the run (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1305_6861_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs the host compilers")


def test_compiler_and_kt_calculator_under_sanitizers(tmp_path):
    exe = tmp_path / "host_sanitize"
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_sanitize.cpp"), os.path.join(CSRC, "compile.cpp"),
           os.path.join(CSRC, "kt.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), "3000"], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert " 0 failures" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    from oracle import build as ob
    lib = str(tmp_path / "liboracle_san.so")
    ob.build(out=lib, extra_flags=SAN)
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.exists(libasan), libasan
    env = dict(os.environ, LD_PRELOAD=libasan, PS_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    tests = ["tests/test_oracle_pins.py", "tests/test_oracle_coils.py", "tests/test_oracle_trajectory.py",
             "tests/test_oracle_snapshots.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_the_harness_catches_a_planted_overflow(tmp_path):
    """The same flags and preload catch a heap overflow in a library loaded
    through ctypes (so a clean run above means something)."""
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\n"
                   "int overflow(int n) { int *a = malloc(4 * n); a[n] = 1; int r = a[0]; free(a); return r; }\n")
    lib = tmp_path / "liboverflow.so"
    subprocess.run(["gcc", "-shared", "-fPIC", *SAN, str(src), "-o", str(lib)], check=True, capture_output=True)
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0")
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).overflow(8)"
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
