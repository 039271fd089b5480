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


def progress(request, msg):
    """Print past pytest's output capture (long oracle runs inside fixtures
    report their progress as they go)."""
    capman = request.config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        print(f"[oracle] {msg}", flush=True)
        return
    with capman.global_and_fixture_disabled():
        print(f"[oracle] {msg}", flush=True)


def run_oracle_ops(request, state, ops, density=False, label="", every_s=20.0):
    """oracle.run_ops, reporting progress about every `every_s` seconds."""
    import time

    import oracle
    t0 = last = time.perf_counter()
    for i, op in enumerate(ops):
        oracle.run_ops(state, [op], density=density)
        now = time.perf_counter()
        if now - last > every_s:
            progress(request, f"{label}: {i + 1}/{len(ops)} ops, {now - t0:.0f} s")
            last = now
    progress(request, f"{label}: {len(ops)} ops in {time.perf_counter() - t0:.1f} s")
    return state
