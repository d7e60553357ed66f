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


@pytest.fixture(scope="module")
def kernel_objects(tmp_path_factory):
    """The library's kernel sources built by hipcc as for the library (linked
    into the served-loop driver, never run there)."""
    from paper_1305_6861_amd import build as lb
    d = tmp_path_factory.mktemp("kernels")
    objs, procs = [], []
    for src in ("kernels.hip", "calib.hip"):
        obj = str(d / (src + ".o"))
        procs.append(subprocess.Popen([lb.HIPCC, *lb.COMMON, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")[-3000:]
    return objs


def _served_loop_binary(tmp_path, sanitize, objs):
    """tests/host_sched_sanitize.cpp linked with the library's host sources
    built by g++ with the given sanitizer flags."""
    host = ["api.cpp", "server.cpp", "batch.cpp", "compile.cpp", "tune.cpp", "kt.cpp", "kt_engine.cpp", "plan.cpp"]
    exe = str(tmp_path / "host_sched")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-w", *sanitize, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_sched_sanitize.cpp"),
           *[os.path.join(CSRC, h) for h in host], *objs, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(not os.path.exists("/opt/rocm/lib/libamdhip64.so"), reason="needs the HIP runtime to link")
@pytest.mark.parametrize("kind", ["thread", "address"])
def test_served_loop_under_sanitizers(tmp_path, kind, kernel_objects):
    """The served loop's locking and bookkeeping: four client threads submit,
    poll, wait (with and without time-outs), cancel and release 120 requests
    on a scheduler-test context while a fifth reads the server counters and
    one iteration fails by design.  ThreadSanitizer: no data race; ASan and
    UBSan: no memory error.  (A suppression covers the double-lock report
    that gcc 11's ThreadSanitizer gives for a condition-variable wait with a
    time-out: libstdc++ waits through pthread_cond_clockwait there, which
    that ThreadSanitizer does not intercept, so it misses the unlock.)"""
    flags = (["-fsanitize=thread"] if kind == "thread"
             else ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])
    exe = _served_loop_binary(tmp_path, flags, kernel_objects)
    supp = tmp_path / "tsan.supp"
    supp.write_text("mutex:ps_wait\n")
    env = dict(os.environ, TSAN_OPTIONS=f"halt_on_error=1 suppressions={supp}",
               ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for _ in range(3):
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        print(r.stdout, r.stderr[-3000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert " 0 problems" in r.stdout


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
