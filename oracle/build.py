"""Compile the C oracle into oracle/liboracle.so (gcc, FP64, no fast-math).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg load the result.  Two more variants serve the CPU tests:
liboracle_count.so counts every amplitude write (-DORACLE_COUNT_WRITES), and
liboracle_asan.so is built by the ROCm clang with AddressSanitizer and
UndefinedBehaviorSanitizer (clang instruments the complex-typed loads and
stores of the OpenMP loops, which this gcc's AddressSanitizer leaves
unchecked); load it with the runtime of asan_runtime() preloaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
ROCM_CLANG = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
VARIANTS = {
    "plain": (LIB, []),
    "count": (os.path.join(HERE, "liboracle_count.so"), ["-DORACLE_COUNT_WRITES"]),
    "asan": (os.path.join(HERE, "liboracle_asan.so"),
             ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]),
}


def asan_runtime():
    """Path of the shared AddressSanitizer runtime the sanitizer build needs
    preloaded, or None."""
    r = subprocess.run([ROCM_CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def lib_path(variant="plain"):
    return VARIANTS[variant][0]


def build(verbose=False, variant="plain"):
    out, extra = VARIANTS[variant]
    cc = ["gcc"]
    if variant == "asan":
        cc = [ROCM_CLANG, "-shared-libsan", "-Wl,-rpath," + os.path.join(os.path.dirname(os.path.dirname(ROCM_CLANG)), "lib")]
    cmd = cc + ["-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
                "-Wno-unused-parameter"] + extra + [SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
