"""The oracle's CPU pins run clean under AddressSanitizer and UBSan (no GPU).

The oracle source is built once more with -fsanitize=address,undefined (any
finding aborts) and the pin modules run in a child process that loads that
build (``WANDQS_ORACLE_LIB``) with the ASan runtime preloaded.  The finest
linear-wake resolution is left out to bound the time; it runs the same code
as the coarser ones.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["test_oracle_mg.py", "test_oracle_slice.py", "test_oracle_adjoint.py",
        "test_oracle_tangent.py", "test_oracle_threads.py"]


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("g++") is None or _runtime("libasan.so") is None,
                    reason="g++ with the ASan runtime is not available")
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                    "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", lib,
                    os.path.join(ROOT, "oracle", "wandqs_oracle.cpp")], check=True)
    env = dict(os.environ, LD_PRELOAD=_runtime("libasan.so"), WANDQS_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "-k", "not linear_wake_closed_form and not under_asan"] + \
          [os.path.join(ROOT, "tests", f) for f in PINS]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    print(r.stdout.strip().splitlines()[-1])
