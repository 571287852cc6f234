"""The sparse solvers' host code under sanitizers (CPU only).

tests/sanitize/host_driver.cpp factors and solves seeded 27-point block
systems with the host multifrontal (complex128 and complex64 factors, single
and block solves, 3-D with three unknowns per point and 2-D with two) and runs
the threaded symbolic phase of the GPU factor, checking residuals and the
elimination order.  It is built with clang++ from the library's own sources
(host_solver.cpp, nd_tree.cpp, gpu_symbolic.cpp) twice:

* AddressSanitizer + UndefinedBehaviorSanitizer (no recovery; leaks checked,
  the OpenMP runtime's own allocation suppressed);
* ThreadSanitizer, with the OpenMP runtime's synchronisation made visible to
  it through the Archer tool library and the target-clone dispatch turned
  off (its resolvers would run before the sanitizer's runtime).

Either build reporting anything fails the test.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_02297_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ARCHER = "/opt/rocm/llvm/lib/libarcher.so"
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")] + \
          [os.path.join(CSRC, f) for f in ("host_solver.cpp", "nd_tree.cpp", "gpu_symbolic.cpp")]
COMMON = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-march=x86-64-v3", "-Wno-pass-failed",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not available")]


def _build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    r = subprocess.run([CLANG] + COMMON + flags + SOURCES + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, args, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, env=e, timeout=600)
    print(r.stdout[-2000:])
    return r


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = _build(tmp_path, "host_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    supp = os.path.join(ROOT, "tests", "sanitize", "lsan.supp")
    r = _run(exe, [12, 47], {"ASAN_OPTIONS": "detect_leaks=1", "LSAN_OPTIONS": f"suppressions={supp}",
                             "UBSAN_OPTIONS": "print_stacktrace=1", "OMP_NUM_THREADS": "4"})
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ALL OK" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(ARCHER), reason="Archer (OpenMP annotations for TSan) not available")
def test_host_code_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, "host_tsan", ["-fsanitize=thread", "-DLS_NO_TARGET_CLONES"])
    r = _run(exe, [14, 47], {"OMP_TOOL_LIBRARIES": ARCHER, "TSAN_OPTIONS": "ignore_noninstrumented_modules=1",
                             "OMP_NUM_THREADS": "8"})
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ALL OK" in r.stdout
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
