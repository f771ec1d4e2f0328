"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C code: rebuilt with -fsanitize=address,undefined (every
  report fatal) and its pin tests re-run against that build in a child
  Python process with the sanitizer runtimes preloaded.
* The library's host-side footprint check (host_geom.hpp, the geometry of
  set_footprint / mppi_check_footprint): a fuzz driver built with the same
  sanitizers by g++.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["tests/test_oracle_geometry.py", "tests/test_oracle_cost.py",
                "tests/test_oracle_rng_rollout.py", "tests/test_oracle_hybrid.py",
                "tests/test_oracle_mlp.py", "tests/test_oracle_cloud.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _sanitizer_env(extra):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(extra)
    return env


def test_oracle_tests_pass_under_sanitizers():
    from oracle import oracle
    san = oracle.build_sanitized()
    env = _sanitizer_env({"EXACT_MPPI_ORACLE_LIB": san})
    probe = ("from oracle import oracle; oracle.lib(); "
             "print(any('liboracle_san.so' in l for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "True", r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", *ORACLE_TESTS, "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, out


def test_host_footprint_check_under_sanitizers(tmp_path):
    exe = tmp_path / "footprint_check_fuzz"
    src = os.path.join(ROOT, "tests", "host", "footprint_check_fuzz.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
                    "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "violations 0" in r.stdout
