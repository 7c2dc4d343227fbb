"""The library's host code runs clean under AddressSanitizer and UBSan (no GPU).

Every source of libwandqs.so is built once more, the host side instrumented
with -fsanitize=address,undefined (any finding aborts; the device side is
compiled as usual and never launched here), and the host-side ABI tests run in
a child process that loads that build (``WANDQS_LIB``) with clang's ASan
runtime preloaded: configuration validation, workspace sizing and layout, the
init path up to its HIP failure, and the exported symbol table.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2012_00881_amd"))
import build as B  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _asan_runtime():
    if not os.path.exists(B.HIPCC):
        return None
    p = subprocess.run([B.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_asan_runtime() is None, reason="hipcc with clang's ASan runtime is not available")
def test_host_code_under_asan_ubsan(tmp_path):
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-I", os.path.join(ROOT, "include"), "-I", B.CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([B.HIPCC] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(compile_one, B.sources()))
    lib = str(tmp_path / "libwandqs_asan.so")
    subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN[:4] + ["-o", lib] + objs,
                   check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), WANDQS_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:alloc_dealloc_mismatch=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_lib_abi.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
    print(r.stdout.strip().splitlines()[-1])
