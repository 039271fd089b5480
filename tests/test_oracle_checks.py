"""CPU checks of the oracle's own builds (no GPU):

* a write-counting build (ORACLE_VARIANT=count) against the amplitude write
  counts the paper states per algorithm (Table "alg_summary_table" and each
  algorithm's cost statement), which a wrong loop range or a doubled pass
  would change;
* an AddressSanitizer + UndefinedBehaviorSanitizer build (ORACLE_VARIANT=asan)
  running every oracle pin, and a deliberately undersized buffer passed to it
  that the sanitizer must report (so a clean run means something).

Each runs in a subprocess that loads the chosen build."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _env(variant, asan=False):
    env = dict(os.environ)
    env["ORACLE_VARIANT"] = variant
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    if asan:
        sys.path.insert(0, ROOT)
        from oracle import build
        lib = build.asan_runtime()
        if not lib:
            pytest.skip("the sanitizer runtime is not available")
        env["LD_PRELOAD"] = lib
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def _build(variant):
    sys.path.insert(0, ROOT)
    from oracle import build
    build.build(variant=variant)


def test_write_counts_match_the_paper():
    _build("count")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_write_counts.py")],
                       env=_env("count"), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "write counts ok" in r.stdout


def test_oracle_pins_under_sanitizers():
    _build("asan")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider"],
                       env=_env("asan", asan=True), capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_sanitizer_build_reports_an_overflow():
    """A 2^10-amplitude buffer passed as an 11-qubit state: the sanitizer
    build must stop at the first access past its end."""
    _build("asan")
    code = (
        "import ctypes as C, numpy as np, oracle\n"
        "L = oracle.lib()\n"
        "assert oracle.build.lib_path('asan') in L._name\n"
        "psi = np.zeros(1 << 10, np.complex128)\n"
        "m = np.eye(2, dtype=np.complex128)\n"
        "t = np.array([10], np.int32)\n"
        "L.oracle_apply_gate(psi.ctypes.data, 11, None, 0, t.ctypes.data, 1, m.ctypes.data)\n"
        "print('no report')\n")
    r = subprocess.run([sys.executable, "-c", code], env=_env("asan", asan=True), capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode != 0, r.stdout + r.stderr
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
