"""AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only): the oracle's
pins against the oracle built with both sanitizers, and the ABI's host-side
validation against the library built with them on its host code.  Every
finding aborts the child process, so a pass means none was reported."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run(env_extra, test_file):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", test_file], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    return r.stdout


@pytest.mark.skipif(_gcc_runtime("libasan.so") is None, reason="gcc's ASan runtime missing")
def test_oracle_pins_under_asan_and_ubsan():
    import oracle
    lib = oracle.build_sanitized()
    out = _run({"ORACLE_LIB": lib, "LD_PRELOAD": _gcc_runtime("libasan.so")},
               "tests/test_oracle_pins.py")
    assert " passed" in out


def test_host_validation_under_asan_and_ubsan():
    from paper_2512_06715_amd import build_san
    try:
        rt = build_san.asan_runtime()
    except RuntimeError:
        pytest.skip("clang's ASan runtime missing")
    lib = build_san.build()
    out = _run({"PDHG_LIB": lib, "LD_PRELOAD": rt}, "tests/test_abi_host.py")
    assert " passed" in out
