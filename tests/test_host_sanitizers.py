"""The host code of libqsim built with AddressSanitizer and
UndefinedBehaviorSanitizer (libqsim_asan.so; the device code is unchanged)
running the C-ABI checks and the host logic (recording, fusion, tile
planning and packing, batch recording with gadget decompositions) on the
CPU, in a subprocess with the sanitizer runtime preloaded."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def san_env():
    sys.path.insert(0, ROOT)
    from oracle import build as obuild
    from paper_2311_01512_amd import build as lbuild
    rt = obuild.asan_runtime()
    if not rt:
        pytest.skip("the sanitizer runtime is not available")
    lib = lbuild.build(sanitize=True)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0", "QS_LIB": lib,
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "PYTHONPATH": ROOT + os.pathsep + env.get("PYTHONPATH", "")})
    return env


def test_abi_checks_under_sanitizers(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], env=san_env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]


def test_host_logic_under_sanitizers(san_env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_logic_checks.py")], env=san_env,
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "host logic ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
