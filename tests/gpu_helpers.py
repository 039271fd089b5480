"""Helpers shared by the GPU parity tests."""
import numpy as np

TOL = {"c128": 1e-12, "c64": 1e-5}


def amp_err(got, want):
    """max_i |got_i - want_i| / max_i |want_i| (normalised max-abs error)."""
    want = np.asarray(want)
    scale = np.abs(want).max()
    if scale == 0:
        scale = 1.0
    return float(np.abs(np.asarray(got) - want).max() / scale)


def scalar_tol(prec, magnitude=1.0):
    return TOL[prec] * max(1.0, abs(magnitude))


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
