"""Host code under sanitizers (no device): the CPU oracle, the block
scheduler of host-memory matching and the host worker pool of the copies,
each driven by a harness in tests/sanitize/ and built with gcc/g++ with
AddressSanitizer and UndefinedBehaviorSanitizer (the pool also with
ThreadSanitizer).  A sanitizer report makes the harness exit non-zero."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ASAN_UBSAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _build_and_run(tmp_path, compiler, flags, sources, name, env=None):
    exe = str(tmp_path / name)
    r = subprocess.run([compiler, *flags, "-o", exe, *sources], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run([exe], capture_output=True, text=True, env=e, timeout=300)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, \
        (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", ["-std=c11", *ASAN_UBSAN, "-ffp-contract=off", "-fopenmp"],
                         [os.path.join(SAN, "oracle_harness.c"), os.path.join(ROOT, "oracle", "cashash_oracle.c"),
                          os.path.join(ROOT, "oracle", "geometry_oracle.c"), "-lm"], "oracle_harness",
                         env={"OMP_NUM_THREADS": "2"})
    assert "oracle harness ok" in out


def test_scheduler_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", ["-std=c++17", *ASAN_UBSAN],
                         [os.path.join(SAN, "sched_harness.cpp")], "sched_harness")
    assert "scheduler harness ok" in out



def test_host_pool_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", ["-std=c++17", *ASAN_UBSAN],
                         [os.path.join(SAN, "pool_harness.cpp"), "-lpthread"], "pool_harness_asan")
    assert "pool harness ok" in out


def test_host_pool_under_tsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", ["-std=c++17", "-O1", "-g", "-fsanitize=thread"],
                         [os.path.join(SAN, "pool_harness.cpp"), "-lpthread"], "pool_harness_tsan")
    assert "pool harness ok" in out
