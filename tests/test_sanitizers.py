"""The oracle and the library's host code (argument validation, constant
folding, workspace carving, the molecular-data reader, plan set-up) under
AddressSanitizer and UndefinedBehaviorSanitizer: each is rebuilt with the
sanitizers into a temporary directory and the CPU tests that exercise it run
in a child process that preloads the sanitizer runtime. No GPU code runs."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(tests, env_extra, preload):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", *tests, "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


def test_oracle_under_asan_and_ubsan(tmp_path):
    import oracle

    lib = oracle.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    preload = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    _run(["tests/test_oracle_pins.py", "tests/test_oracle_levels.py",
          "tests/test_oracle_post.py"], {"IRIS_ORACLE_LIB": lib}, preload)


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2607_01338_amd import build

    runtimes = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/"
                                "libclang_rt.asan-x86_64.so"))
    if not runtimes:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    lib = build.build_host_sanitized(str(tmp_path / "libiris_rt_san.so"))
    _run(["tests/test_abi.py"], {"IRIS_RT_LIBRARY": lib}, runtimes[-1])
