"""Host code under sanitizers, on the CPU: the server's arena allocator and
admission rule (a C++ driver against a reference model and a fake clock),
the plans' autotune cache file, and the oracle's pin suite against an
AddressSanitizer + UBSan build of the oracle."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g"]


def _gxx_runtime(name):
    path = subprocess.check_output(["g++", f"-print-file-name={name}"], text=True).strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_arena_and_admission_under_sanitizers(tmp_path):
    exe = str(tmp_path / "arena_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", *SAN, "-I", os.path.join(ROOT, "paper_2511_16298_amd", "csrc"),
                           os.path.join(HERE, "native", "arena_test.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "OK"


def test_tune_cache_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tunecache_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", *SAN, "-I", os.path.join(ROOT, "paper_2511_16298_amd", "csrc"),
                           os.path.join(HERE, "native", "tunecache_test.cpp"), "-o", exe])
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "OK"


def test_oracle_pins_under_sanitizers(tmp_path):
    asan = _gxx_runtime("libasan.so")
    if asan is None:
        pytest.skip("libasan runtime not found")
    import oracle
    lib = str(tmp_path / "liboracle_san.so")
    oracle.build(out=lib, extra=SAN)
    env = dict(os.environ, SS_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
