"""AddressSanitizer + UndefinedBehaviorSanitizer on the host code (CPU).

* The FP64 oracle, compiled with gcc -fsanitize=address,undefined into
  oracle/sanitize_driver.c, which runs every oracle function on small and
  edge-case inputs and checks identities it must satisfy.
* The library's host layer (argument validation, tuning table, error text),
  built with host-side ASan + UBSan (paper_2009_11742_amd.build
  .build_sanitized) and loaded in a child process with the clang ASan
  runtime preloaded, running the C-ABI tests of test_abi_cpu.py (none of
  which touch a GPU).
Any sanitizer report fails the run (halt on the first error).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "oracle sanitizer driver: ok" in r.stdout


def test_host_layer_under_asan_ubsan(tmp_path):
    from paper_2009_11742_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.build_sanitized(str(tmp_path / "san"))
    rt = build.asan_runtime()
    assert rt, "clang ASan runtime not found"
    env = dict(os.environ, ROM_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "passed" in r.stdout and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
