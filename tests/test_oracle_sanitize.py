"""The FP64 oracle (plain C) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on small grids through a C driver
(tests/oracle_sanitize_driver.c): no out-of-bounds access, use after free,
leak or undefined behaviour on any path of the grid step.  CPU only; the
sanitizer runtime is linked statically.  The same driver also runs under
ThreadSanitizer, built with clang against the LLVM OpenMP runtime, for the
oracle's OpenMP loops."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-static-libasan",
           os.path.join(ROOT, "oracle", "rrmhd_oracle.c"),
           os.path.join(ROOT, "oracle", "rrmhd3d_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


_CLANG = "/opt/rocm/llvm/bin/clang"
_OMPLIB = "/opt/rocm/llvm/lib"
_ARCHER = os.path.join(_OMPLIB, "libarcher.so")

# a positive control: two threads of an OpenMP loop update one variable
# without synchronisation, which the sanitizer must report
_RACY = r"""
#include <stdio.h>
int main(void) {
  double s = 0.0;
#pragma omp parallel for
  for (int i = 0; i < 4096; ++i) s += (double)i;
  printf("%g\n", s);
  return 0;
}
"""


def _tsan_build(srcs, exe):
    cmd = [_CLANG, "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=thread", *srcs, "-lm",
           "-o", exe, f"-Wl,-rpath,{_OMPLIB}"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def _tsan_run(exe):
    # the LLVM OpenMP runtime with its Archer tool supplies the runtime's
    # synchronisation to the sanitizer (barriers, task and lock semantics);
    # reports from inside the uninstrumented runtime library are dropped
    env = dict(os.environ, OMP_NUM_THREADS="4", OMP_TOOL_LIBRARIES=_ARCHER,
               TSAN_OPTIONS="ignore_noninstrumented_modules=1 halt_on_error=1 exitcode=66")
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.skipif(not (os.path.exists(_CLANG) and os.path.exists(_ARCHER)),
                    reason="clang with the LLVM OpenMP runtime and Archer not available")
def test_oracle_under_thread_sanitizer(tmp_path):
    """The oracle's OpenMP loops (the 2D and 3D grid steps, the 3D init and
    moments) built with ThreadSanitizer and run through the same driver on
    four threads: no data race.  The same build of a loop with an
    unsynchronised shared sum is reported, so the set-up does see races."""
    racy_src = tmp_path / "racy.c"
    racy_src.write_text(_RACY)
    racy = str(tmp_path / "racy")
    _tsan_build([str(racy_src)], racy)
    r = _tsan_run(racy)
    assert r.returncode == 66 and "data race" in r.stderr, r.stdout + r.stderr

    exe = str(tmp_path / "oracle_tsan")
    _tsan_build([os.path.join(ROOT, "oracle", "rrmhd_oracle.c"),
                 os.path.join(ROOT, "oracle", "rrmhd3d_oracle.c"),
                 os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")], exe)
    r = _tsan_run(exe)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr, r.stderr
