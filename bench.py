"""Throughput of the 28-qubit random-circuit workload on one MI355X.

A step is one application of the 500-gate circuit (Haar 1-qubit gates,
2-target Haar gates with 0-3 controls, Pauli gadgets exp(i theta P) of weight
1-28) to a 2^28-amplitude statevector resident in HBM.  Paths timed:

* fused complex64: the library's autotuner picks plain passes, dense
  k-qubit blocks (FP32 MFMA for 4-6 qubits) or tile steps (many operators
  per HBM pass), generic or compiled per step.  This is the headline
  `value`.
* plain complex128: one pass per gate (the paper's per-gate method).
* fused complex128: the autotuned complex128 tile steps.

`value` is logical amplitude-updates/s (plain per-gate accounting: 2^(N-s)
per s-controlled gate, 2^N per gadget, credited alike to every path).  The
timed region is `--steps` applications with every pass bracketed by HIP
events on the qureg's stream; the roofline's per-launch average comes from
those events.  Each path's state after one application from the
counter-hashed state is compared with the oracle's (the CPU baseline run,
the whole circuit on the host cores).  The default line also carries the
14-qubit density-matrix workload and the 512-circuit batch as sub-objects.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=28)
    ap.add_argument("--gates", type=int, default=500)
    ap.add_argument("--fuse-candidates", default="0,4,5,10,11,12,13",
                    help="fusion widths the autotuner tries: 0 plain, 2-6 dense blocks, 8-14 LDS tiles")
    ap.add_argument("--cpu-runs", type=int, default=1,
                    help="runs of the oracle over the whole circuit for the CPU baseline (median taken)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (CPU baseline and the error against the oracle)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="headline only: skip the density-matrix and batched sub-lines")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware-counter collection: one torch copy of 2 GiB "
                         "(the calibration kernel of known traffic), then one application of the "
                         "28-qubit circuit (with --workload sv34 the 34-qubit one, with density14 the "
                         "14-qubit density circuit) compiled at "
                         "--probe-fuse-k in --probe-precision")
    ap.add_argument("--probe-fuse-k", type=int, default=12)
    ap.add_argument("--probe-precision", default="c64", choices=["c64", "c128"])
    ap.add_argument("--probe-specialize", action="store_true",
                    help="compile the probe circuit's tile steps into a kernel each first")
    ap.add_argument("--no-specialize", action="store_true",
                    help="keep the generic tile-step kernel (no run-time compilation)")
    ap.add_argument("--batch-precision", default="c64", choices=["c64", "c128"],
                    help="state precision of the batch512 workload")
    ap.add_argument("--workload", default="circuit28", choices=["circuit28", "density14", "batch512", "sv34"],
                    help="circuit28 (default, the headline): 28-qubit 500-gate circuit; density14: 14-qubit "
                         "density matrix; batch512: 512 circuits with energies and gradients; sv34: 34 qubits")
    return ap.parse_args()


SPECIALIZED_TILE = "qs_step_* (tile steps compiled per step at run time)"


def kernel_name(info, real, specialized=False):
    k = info["kernel"]
    if k == "tile" and specialized:
        return f"{SPECIALIZED_TILE}<{real}>"
    if k == "gadget_pairs":
        return f"k_gadget_pairs<{real}>"
    if k == "gadget_diag":
        return f"k_gadget_diag<{real}>"
    if k == "dense_mfma":
        return f"k_dense_mfma<{info['num_targs']}>"
    if k == "tile":
        return f"k_tile_step<{real}>"
    return f"k_gate<{real}, {info['num_targs']}>"


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (profiles/traffic.json), or None when there is
    none or one of the kernel's sources changed since the counters were
    taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}@{workload}")
    if not rec:
        return None
    for name, prefix in rec["sources"].items():
        src = open(os.path.join(ROOT, name), "rb").read()
        if hashlib.sha256(src).hexdigest()[:len(prefix)] != prefix:
            return None
    return rec["bytes_per_launch"]


def time_steps(circ, q, steps, torch):
    """Seconds per application, HIP events on the qureg's stream."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(q.stream)
    for _ in range(steps):
        circ.apply(q)
    b.record(q.stream)
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / steps


def pass_kinds(circ, q):
    """Per pass of a compiled circuit: (kernel name, amplitudes it reads and
    writes once, flops)."""
    n = 2 * q.num_qubits if q.density else q.num_qubits     # index bits
    real = "float" if q.precision == "c64" else "double"
    out = []
    for i in range(circ.stats()["num_passes"]):
        info = circ.pass_info(i)
        name = kernel_name(info, real, circ.specialized > 0)
        amps = 1 << (n - info["num_ctrls"])
        if info["kernel"] == "tile":
            amps = 1 << n          # one read and one write of the whole state per step
        flops = 8 * (1 << info["num_targs"]) * amps if info["kernel"].startswith("dense") else 0
        out.append((name, amps, flops))
    return out


def line_amps(ops, n, amp_bytes):
    """Per operator of a plain (one pass per operator) circuit: amplitudes of
    the 128-byte lines its kernel must read and write.  A control on a qubit
    inside a line (the 3 (complex128) or 4 (complex64) lowest) selects half
    of every line, so it does not shrink the set of lines touched."""
    low = 3 if amp_bytes == 16 else 4
    out = []
    for op in ops:
        hi = [c for c in op.get("ctrls", ()) if c >= low] if op["op"] == "unitary" else []
        out.append(1 << (n - len(hi)))
    return out


def timed_region(circ, q, steps, torch, lines=None):
    """The timed region: `steps` applications of the circuit, each pass
    bracketed by HIP events on the qureg's stream (the stream the kernels
    are launched on).  Returns (seconds per application over the whole
    region, kernel -> [launches, total ms, amplitudes, flops] summed over
    every pass of every application)."""
    kinds = pass_kinds(circ, q)
    npass = len(kinds)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(npass)]
          for _ in range(steps)]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(q.stream)
    for s_ in range(steps):
        for i in range(npass):
            ev[s_][i][0].record(q.stream)
            circ.apply_passes(q, i, 1)
            ev[s_][i][1].record(q.stream)
    b.record(q.stream)
    b.synchronize()
    out = {}
    for s_ in range(steps):
        for i, ((name, amps, flops), (e0, e1)) in enumerate(zip(kinds, ev[s_])):
            c = out.setdefault(name, [0, 0.0, 0, 0, 0])
            c[0] += 1
            c[1] += e0.elapsed_time(e1)
            c[2] += amps
            c[3] += flops
            c[4] += lines[i] if lines else amps
    return a.elapsed_time(b) * 1e-3 / steps, out


def time_passes(circ, q, torch):
    """One application pass by pass, each bracketed by HIP events; returns
    kernel -> [launches, total ms, amplitudes touched, flops]."""
    return timed_region(circ, q, 1, torch)[1]


def per_kernel_table(kinds, amp_bytes):
    """Per kernel: launches, average ms, GB/s of the algorithmic bytes (the
    amplitudes the plain method updates, read and written once) and, where
    they differ, of the 128-byte lines the kernel must move (controls on
    qubits inside a line select half of every line)."""
    out = {}
    for k, v in kinds.items():
        d = {"launches": v[0], "avg_ms": v[1] / v[0], "GBps": 2 * amp_bytes * v[2] / (v[1] * 1e-3) / 1e9,
             "TFLOPs": (v[3] / (v[1] * 1e-3) / 1e12) if v[3] else None}
        if len(v) > 4 and v[4] != v[2]:
            d["GBps_lines"] = 2 * amp_bytes * v[4] / (v[1] * 1e-3) / 1e9
        out[k] = d
    return out


def roofline(kinds, amp_bytes, workload):
    name, v = max(kinds.items(), key=lambda kv: kv[1][1])
    launches, ms, amps, flops = v[:4]
    avg_s = ms * 1e-3 / launches
    if name.startswith("k_dense_mfma<6>"):
        achieved = flops / launches / avg_s / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MFMA_F32_PEAK_TFLOPS, "traffic": measured_traffic(name, workload),
                "kernel": name, "avg_launch_ms": avg_s * 1e3, "flops_per_launch": flops / launches}
    bytes_per_launch = 2 * amp_bytes * amps / launches
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, workload),
            "kernel": name, "avg_launch_ms": avg_s * 1e3, "bytes_per_launch": bytes_per_launch}


def host_cpu():
    """Host CPU as the oracle sees it: usable cores and the model name."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(ops, n, seed, runs):
    """The oracle (plain per-gate complex128 on the host cores, OpenMP) on
    the whole circuit from the counter-hashed state the GPU paths start
    from; the median of `runs` runs.  Returns (baseline record, the oracle's
    final state)."""
    import statistics
    import oracle
    updates = 0
    for op in ops:
        updates += (1 << n) if op["op"] == "gadget" else (1 << (n - len(op["ctrls"])))
    times = []
    psi = None
    for _ in range(runs):
        psi = oracle.hashed_state(n, seed)
        t0 = time.perf_counter()
        oracle.run_ops(psi, ops)
        times.append(time.perf_counter() - t0)
    dt = statistics.median(times)
    cpu = host_cpu()
    rec = {"value": updates / dt, "unit": "amplitude-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"the whole {len(ops)}-gate {n}-qubit circuit, plain per-gate complex128, from the "
                     f"counter-hashed state (seed {seed}); median of {runs} run(s): "
                     + ", ".join(f"{t:.1f} s" for t in times),
           "nproc": cpu["nproc"], "cpu_model": cpu["model"], "seconds": times}
    return rec, psi


def batch_vs_oracle(keep):
    """The batch's energies of a sample of circuits (the smallest, the
    largest and two between) against the oracle's, and the gradient of the
    smallest against the oracle's exact parameter-shift rule, on the host."""
    import numpy as np
    import oracle
    probs, e, g = keep["probs"], keep["energies"], keep["grads"]
    ns = [p["num_qubits"] for p in probs]
    order = sorted(range(len(probs)), key=lambda i: (ns[i], i))
    sample = sorted({order[0], order[len(order) // 3], order[2 * len(order) // 3], order[-1]})
    offs = np.concatenate([[0], np.cumsum([len(p["angles"]) for p in probs])])
    t0 = time.perf_counter()
    e_err = 0.0
    for i in sample:
        p = probs[i]
        psi = oracle.run_ops(oracle.zero_state(p["num_qubits"]), p["ops"])
        want = oracle.sv_expec_pauli_sum(psi, p["codes"], p["coeffs"]).real
        e_err = max(e_err, abs(e[i] - want) / max(1.0, float(np.abs(p["coeffs"]).sum())))
    i0 = order[0]
    p = probs[i0]
    m = len(p["angles"])
    gw = oracle.param_shift_gradient(p["num_qubits"], p["ops"], p["codes"], p["coeffs"], m)
    g_err = float(np.abs(g[offs[i0]:offs[i0] + m] - gw).max() / max(1.0, float(np.abs(gw).max())))
    return {"max_energy_err": float(e_err), "max_grad_err": g_err,
            "sample": f"energies of circuits {sample} (N = {[ns[i] for i in sample]}), scaled by the sum of "
                      f"|coefficients|; the {m} gradients of circuit {i0} (N = {ns[i0]}) against the exact "
                      f"parameter-shift rule, scaled by their largest magnitude",
            "seconds": time.perf_counter() - t0}


def streaming_ceiling(qs, q, torch, reps=5):
    """The fastest in-house streaming kernel on this state: a Pauli-X gadget
    on the highest qubit (k_gadget_pairs: each thread reads and writes a
    pair of amplitudes half the state apart, in runs of consecutive
    addresses), as the HBM rate a kernel of this library reaches when it
    only streams."""
    n = q.num_qubits
    c = qs.Circuit(n, [{"op": "gadget", "targs": (n - 1,), "paulis": (1,), "theta": 0.3}]).compile(0, q.precision)
    c.apply(q)
    ms = time_steps(c, q, reps, torch) * 1e3
    ab = 8 if q.precision == "c64" else 16
    return {"kernel": f"k_gadget_pairs<{'float' if ab == 8 else 'double'}> (X gadget on qubit {n - 1})",
            "ms": ms, "GBps": 2 * ab * q.num_amps / (ms * 1e-3) / 1e9}


def pmc_probe(args):
    import torch
    import synth
    import paper_2311_01512_amd as qs
    n = args.qubits
    src = torch.zeros(1 << 28, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)                      # reads 2 GiB, writes 2 GiB
    torch.cuda.synchronize()
    del src, dst
    density = args.workload == "density14"
    if args.workload == "sv34":
        n = 34
        ops = synth.config5_circuit()
    elif density:
        n = 14
        ops, traced = synth.config3_circuit()
    else:
        ops = synth.config2_circuit(num_qubits=n, num_gates=args.gates)
    q = qs.Qureg(n, density=density, precision=args.probe_precision).init_hashed(11)
    circ = qs.Circuit(n, ops, density=density).compile(args.probe_fuse_k, args.probe_precision)
    if args.probe_specialize:
        circ.specialize()
    circ.apply(q)
    q.sync()
    if density:
        # the partial trace over the workload's 7 qubits, into a preallocated output
        red = qs.Qureg(n - len(traced), density=True, precision=args.probe_precision)
        for _ in range(3):
            q.partial_trace(traced, out=red)
        q.sync()
    print(json.dumps({"pmc_probe": "done", "gates": len(ops), "num_qubits": n,
                      "fuse_k": args.probe_fuse_k, "precision": args.probe_precision,
                      "specialized": circ.specialized}), flush=True)


def base_line(metric_value, unit, steps, warmup, ms, dtype, workload, extra):
    d = {"metric": "amplitude-updates/s & %HBM peak; fused FP32 vs plain FP64 at <=1e-5 amp err",
         "value": metric_value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic seeded inputs (PCG64 generators, counter-hashed states)",
         "config": {"workload": workload}}
    d.update(extra)
    return d


def dm_op_kind(op):
    k = len(op["targs"]) + len(op.get("ctrls", ()))
    return ("dm_unitary" if op["op"] == "unitary" else "kraus") + f"_{k}q"


def path_text(k, specialized=False):
    if k == 0:
        return "one pass per operator"
    if k <= 6:
        return f"operators fused into dense blocks of <= {k} qubits (FP32 MFMA for 4-6 qubit blocks)"
    return (f"tile steps of 2^{k} amplitudes: each step applies its operators on chip in one HBM pass"
            + ("; each step compiled into a kernel of its own at run time" if specialized else ""))


def autotune(circ, q, cands, args):
    """The library's autotuner over `cands`, with specialised tile steps as
    further candidates unless --no-specialize; returns (best_k, generic ms by
    k, specialised ms by k or None)."""
    if args.no_specialize:
        best_k, tune_ms = circ.autotune(q, cands)
        return best_k, tune_ms, None
    return circ.autotune(q, cands, specialize=True)


def bench_channels(q, torch, amp_bytes):
    """One application of each bespoke channel on a density qureg: ms and
    GB/s of the amplitudes it must read and write (dephasing touches half of
    the Choi vector, two-qubit dephasing three quarters, the others all)."""
    n = q.num_qubits
    calls = [("dephasing", lambda: q.apply_dephasing(3, 0.1), 0.5),
             ("dephasing_2q", lambda: q.apply_two_qubit_dephasing(2, n - 1, 0.1), 0.75),
             ("depolarising", lambda: q.apply_depolarising(n - 1, 0.1), 1.0),
             ("depolarising_2q", lambda: q.apply_two_qubit_depolarising(0, n - 2, 0.1), 1.0),
             ("damping", lambda: q.apply_damping(5, 0.1), 1.0)]
    res = {}
    for name, fn, frac in calls:
        fn()                                   # untimed first call
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(q.stream)
        fn()
        b.record(q.stream)
        b.synchronize()
        ms = a.elapsed_time(b)
        byts = 2 * amp_bytes * frac * (1 << (2 * n))
        res[name] = {"ms": ms, "GBps": byts / (ms * 1e-3) / 1e9}
    return res


def bench_special(q, torch, amp_bytes, reps=3):
    """The matrix-free special unitaries on a statevector or density qureg:
    average ms of `reps` applications and GB/s of the 128-byte lines each
    must read and write: a SWAP of two high qubits moves half of a
    statevector in whole lines; a SWAP or multi-SWAP with a qubit inside a
    line (qubit 0 here) moves part of every line, so every line is read and
    written; Pauli tensors, phase gadgets and gadgets read and write every
    amplitude."""
    n = q.num_qubits
    if q.density:
        calls = [("swap_low_high", lambda: q.apply_swap(0, n - 1), 1.0),
                 ("pauli_tensor_xyz", lambda: q.apply_pauli_tensor([0, 5, n - 1], [1, 2, 3]), 1.0),
                 ("phase_gadget_3", lambda: q.apply_phase_gadget([1, 6, n - 2], 0.3), 1.0),
                 ("pauli_gadget_xyz", lambda: q.apply_pauli_gadget([0, 5, n - 1], [1, 2, 3], 0.3), 1.0)]
    else:
        calls = [("swap_low_high", lambda: q.apply_swap(0, n - 1), 1.0),
                 ("swap_high_high", lambda: q.apply_swap(n - 2, n - 1), 0.5),
                 ("multi_swap_3", lambda: q.apply_multi_swap([0, 1, 2], [n - 1, n - 2, n - 3]), 1.0),
                 ("pauli_tensor_xyz", lambda: q.apply_pauli_tensor([0, 11, n - 1], [1, 2, 3]), 1.0),
                 ("phase_gadget_3", lambda: q.apply_phase_gadget([1, 12, n - 2], 0.3), 1.0)]
    res = {}
    for name, fn, frac in calls:
        fn()                                   # untimed first call
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(q.stream)
        for _ in range(reps):
            fn()
        b.record(q.stream)
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        byts = 2 * amp_bytes * frac * q.num_amps
        res[name] = {"ms": ms, "GBps": byts / (ms * 1e-3) / 1e9, "hbm_frac": byts / (ms * 1e-3) / 8e12}
    return res


def bench_reductions(q, torch, amp_bytes, reps=3):
    """The read-only calculations on a statevector or density qureg: average
    ms per call (each call ends with the scalar copied to the host) and GB/s
    of the amplitudes the kernel must read.  Statevector: norm (every
    amplitude), P(qubit N-1 = 0) (half), a 20-term Pauli sum (one read of
    the state per tile span of 7 flip masks).  Density matrix: trace and
    P(qubit = 0) (the 2^N diagonal entries), purity (every entry), the
    20-term Pauli sum (2^N entries per term)."""
    import numpy as np
    n = q.num_qubits
    rng = np.random.default_rng(20)
    codes = rng.integers(0, 4, size=(20, n)).astype(np.int32)
    coeffs = rng.standard_normal(20)
    masks = {int(sum(1 << k for k in range(n) if c[k] in (1, 2))) for c in codes}
    # statevectors: a tile of 2^11 amplitudes holds the partners of up to 7
    # independent flip masks, so the sum reads the state once per 7 masks
    spans = max(1, -(-len(masks - {0}) // 7))
    if q.density:
        calls = [("trace", lambda: q.trace(), 1 << n),
                 ("prob_of_outcome", lambda: q.prob_of_outcome(0, 0), 1 << n),
                 ("purity", lambda: q.purity(), q.num_amps),
                 ("expec_pauli_sum_20", lambda: q.expec_pauli_sum(codes, coeffs), 20 << n)]
    else:
        calls = [("total_prob", lambda: q.total_prob(), q.num_amps),
                 ("prob_of_outcome", lambda: q.prob_of_outcome(n - 1, 0), q.num_amps // 2),
                 ("expec_pauli_sum_20", lambda: q.expec_pauli_sum(codes, coeffs), spans * q.num_amps)]
    res = {}
    for name, fn, amps in calls:
        fn()                                   # untimed first call
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(q.stream)
        for _ in range(reps):
            fn()
        b.record(q.stream)
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        byts = amp_bytes * amps
        res[name] = {"ms": ms, "GBps": byts / (ms * 1e-3) / 1e9, "hbm_frac": byts / (ms * 1e-3) / 8e12}
    return res


def bench_density(args, torch, qs, synth):
    """14-qubit density matrix (Choi vector of 2^28 amplitudes): 300 ops of
    Haar unitaries, depolarising, damping and random Kraus maps applied as
    superoperators, then the partial trace over 7 qubits, trace and purity.
    Plain: the per-operator API in complex128 and complex64.  Fused: the same
    ops as a density circuit in complex64, compiled at the autotuned width."""
    n = 14
    ops, traced = synth.config3_circuit()
    logical = synth.count_logical_updates(ops, n, density=True)
    out = {}
    for prec in ("c128", "c64"):
        q = qs.Qureg(n, density=True, precision=prec).init_zero()
        for _ in range(args.warmup):
            q.run_ops(ops)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in ops]
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(q.stream)
        for _ in range(args.steps):
            q.run_ops(ops)
        t1.record(q.stream)
        t1.synchronize()
        step_s = t0.elapsed_time(t1) * 1e-3 / args.steps
        for op, (a, b) in zip(ops, ev):
            a.record(q.stream)
            q.run_ops([op])
            b.record(q.stream)
        torch.cuda.synchronize()
        kinds = {}
        for op, (a, b) in zip(ops, ev):
            c = kinds.setdefault(dm_op_kind(op), [0, 0.0, 0, 0])
            k = len(op["targs"]) + len(op.get("ctrls", ()))
            c[0] += 1
            c[1] += a.elapsed_time(b)
            c[2] += 1 << (2 * n)                          # one pass over the Choi vector
            c[3] += 8 * (1 << (2 * k)) * (1 << (2 * n))   # 4^k x 4^k superoperator
        ab = 16 if prec == "c128" else 8
        out[prec] = {"value": logical / step_s, "ms_per_step": step_s * 1e3,
                     "roofline": roofline(kinds, ab, "density14"),
                     "per_kind": per_kernel_table(kinds, ab),
                     "channels": bench_channels(q, torch, ab),
                     "special_ops": bench_special(q, torch, ab),
                     "reductions": bench_reductions(q, torch, ab)}
        if prec == "c128":
            # reference result of the plain FP64 path, from |0><0|, one application
            q.init_zero().run_ops(ops)
            ref = q.tensor.clone()
        del q

    # fused complex64 density circuit
    q = qs.Qureg(n, density=True, precision="c64")
    circ = qs.Circuit(n, ops, density=True)
    cands = tuple(int(x) for x in args.fuse_candidates.split(","))
    best_k, tune_ms, spec_ms = autotune(circ, q, cands, args)
    q.init_zero()
    for _ in range(args.warmup):
        circ.apply(q)
    step_s = time_steps(circ, q, args.steps, torch)
    kinds = time_passes(circ, q, torch)
    q.init_zero()
    circ.apply(q)
    with torch.no_grad():
        err = ((q.tensor.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()
    # the partial trace into a preallocated output: kernel time only
    red = q.partial_trace(traced)
    q.sync()
    ta = torch.cuda.Event(enable_timing=True)
    tb = torch.cuda.Event(enable_timing=True)
    ta.record(q.stream)
    for _ in range(10):
        q.partial_trace(traced, out=red)
    tb.record(q.stream)
    tb.synchronize()
    tr, pur = q.trace(), q.purity()
    st = circ.stats()
    fused = {"value": logical / step_s, "ms_per_step": step_s * 1e3, "fuse_k": best_k,
             "autotune_ms": {str(k): v for k, v in tune_ms.items()},
             "autotune_specialised_ms": spec_ms and {str(k): v for k, v in spec_ms.items()},
             "specialised_kernels": circ.specialized,
             "passes": st["num_passes"], "max_amp_err_vs_c128": err, "per_kernel": per_kernel_table(kinds, 8),
             "partial_trace_ms": ta.elapsed_time(tb) / 10,
             "trace": [tr.real, tr.imag], "purity": [pur.real, pur.imag],
             "reduced_trace": red.trace().real, "reduced_purity": red.purity().real}
    line = base_line(fused["value"], "amplitude-updates/s", args.steps, args.warmup, fused["ms_per_step"],
                     "c64 (f32)", "14-qubit density matrix (28-qubit Choi vector), 300 seeded ops: Haar 1/2-qubit "
                     "unitaries, depolarising, damping, random 2-qubit Kraus maps as superoperators; "
                     "partial trace over 7 qubits, trace, purity",
                     {"roofline": roofline(kinds, 8, "density14"), "fused_c64": fused,
                      "plain_c128": out["c128"], "plain_c64": out["c64"],
                      "speedup_fused_c64_vs_plain_c128": out["c128"]["ms_per_step"] / fused["ms_per_step"]})
    line["config"]["path"] = "complex64 density circuit, " + path_text(best_k, circ.specialized > 0)
    del q, red
    return line


def bench_batch(args, torch, qs, synth, keep=None):
    """512 hardware-efficient-ansatz circuits, N ~ U{10..22}, 6 layers, 20-term
    Pauli-sum energies and adjoint gradients over all angles, one graph replay."""
    import numpy as np
    probs = synth.config4_batch()
    b = qs.Batch(args.batch_precision)
    for p in probs:
        b.add_circuit(p["num_qubits"], p["ops"], len(p["angles"]), p["codes"], p["coeffs"])
    b.compile()
    st = b.stats()
    params = np.concatenate([p["angles"] for p in probs])

    def timed(grads):
        for _ in range(args.warmup):
            b.run(params, grads=grads)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = b.run(params, grads=grads)
        return (time.perf_counter() - t0) / args.steps, out

    # generic step kernels, then the run-time specialised ones (the faster
    # form is the line's value; both are reported)
    full_generic, _ = timed(True)
    spec = {"generic_ms": full_generic * 1e3}
    try:
        t0 = time.perf_counter()
        spec["programs"] = b.specialize()
        spec["specialize_s"] = time.perf_counter() - t0
        full_spec, _ = timed(True)
        spec["specialized_ms"] = full_spec * 1e3
        spec["used"] = "specialized" if full_spec < full_generic else "generic"
        if full_spec >= full_generic:
            b.compile()
    except Exception as exc:   # no run-time compiler: generic kernels
        spec["error"] = str(exc)[:200]
        spec["used"] = "generic"
    full, (e, g) = timed(True)
    fwd, _ = timed(False)
    if keep is not None:   # for the check against the oracle on the host
        keep.update({"probs": probs, "energies": np.array(e), "grads": np.array(g)})
    fwd_upd = st["logical_updates"]
    total = 3 * fwd_upd      # forward, then U^dagger on phi and on lambda
    # algorithmic flops of one run (FP32 or FP64), each operator at the fewest flops
    # its form needs per amplitude: a rotation c 1 + i s P (P = X, Y, Z) 6
    # (one product and one fused multiply-add per real component), a fixed
    # 2 x 2 gate 14 (two complex products and a sum), CZ none; the adjoint
    # sweep applies each operator to two states and forms Im conj(lambda) P phi
    # for every rotation (4 per amplitude: four products summed, the gradient
    # needing no real part); lambda = H psi costs 8 per amplitude and term
    flops = 0
    for p in probs:
        a = 1 << p["num_qubits"]
        rot = sum(1 for op in p["ops"] if op["op"] == "gadget" and "param" in op)
        fixed = sum(1 for op in p["ops"] if op["op"] == "unitary" and not op.get("ctrls"))
        fixed += sum(1 for op in p["ops"] if op["op"] == "gadget" and "param" not in op)
        flops += a * (3 * (6 * rot + 14 * fixed) + 4 * rot + 8 * len(p["coeffs"]))
    achieved = flops / full / 1e12
    peak = FP32_VECTOR_PEAK_TFLOPS if args.batch_precision == "c64" else FP64_VECTOR_PEAK_TFLOPS
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None,
            "kernel": "batch replay (forward, energies, adjoint sweep; states stay in LDS / L2)",
            "flops_per_run": flops}
    return base_line(total / full, "amplitude-updates/s", args.steps, args.warmup, full * 1e3,
                     "c64 (f32)" if args.batch_precision == "c64" else "c128 (f64)",
                     "512 statevectors, N ~ U{10..22}, 6-layer hardware-efficient ansatz, 20-term Pauli-sum "
                     "energy and adjoint gradient over all angles, one HIP-graph replay",
                     {"roofline": roof, "circuits": st["num_circuits"], "total_amplitudes": st["total_amps"],
                      "launch_steps": st["num_steps"], "forward_only_ms": fwd * 1e3,
                      "forward_updates_per_s": fwd_upd / fwd, "gradients": int(params.size),
                      "circuits_per_s_with_gradient": st["num_circuits"] / full,
                      "step_kernels": spec, "energy_mean": float(np.mean(e))})


def bench_sv34(args, torch, qs, synth):
    """34-qubit complex64 statevector (2^34 amplitudes, 128 GiB): 200 gates of
    5-target Haar unitaries with up to 4 controls and Pauli gadgets of weight
    up to 34, plain per-gate vs dense blocks (k = 6) vs tile steps of 2^12 or
    2^13 amplitudes, specialised (5-target gates stay single passes there), one application
    each (the faster fused path is the headline); <Z_0 Z_33> and norm in FP64."""
    import numpy as np
    n = 34
    ops = synth.config5_circuit()
    logical = synth.count_logical_updates(ops, n)
    q = qs.Qureg(n, precision="c64").init_hashed(5)
    res = {}
    norm0 = q.total_prob()
    # tile steps: widths 12 and 13, specialised, the faster kept (one 5 s
    # application each; the autotuner's full candidate list would cost minutes)
    applications = 0
    for label, widths in (("plain_c64", (0,)), ("fused_c64", (6,)), ("tiled_c64", (12, 13))):
        applications += len(widths) + 1   # timed once per width, then pass by pass
        best = None
        for k in widths:
            circ = qs.Circuit(n, ops).compile(k, "c64")
            if k >= 8 and not args.no_specialize:
                circ.specialize()
            t = time_steps(circ, q, 1, torch)
            if best is None or t < best[0]:
                best = (t, k, circ)
            else:
                del circ
        t, k, circ = best
        kinds = time_passes(circ, q, torch)
        res[label] = {"value": logical / t, "ms_per_step": t * 1e3, "fuse_k": k, "passes": circ.stats()["num_passes"],
                      "specialised_kernels": circ.specialized,
                      "roofline": roofline(kinds, 8, "sv34"), "per_kernel": per_kernel_table(kinds, 8)}
        del circ, best
    zz = np.zeros((1, n), np.int32)
    zz[0, 0] = zz[0, n - 1] = 3
    ezz = q.expec_pauli_sum(zz, [1.0])
    norm1 = q.total_prob()
    best = min(("fused_c64", "tiled_c64"), key=lambda k: res[k]["ms_per_step"])
    head = res[best]
    return base_line(head["value"], "amplitude-updates/s", 1, 0, head["ms_per_step"], "c64 (f32)",
                     "34-qubit complex64 statevector (128 GiB), 200 seeded gates: 5-target Haar unitaries with "
                     "0-4 controls and Pauli gadgets of weight 1-34",
                     {"path": best, "roofline": head["roofline"], "fused_c64": res["fused_c64"],
                      "tiled_c64": res["tiled_c64"], "plain_c64": res["plain_c64"],
                      "zz_0_33": [ezz.real, ezz.imag], "norm_before": norm0,
                      "norm_after": norm1, "circuit_applications": applications, "relative_norm_drift": abs(norm1 - norm0) / norm0})


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe(args)
        return
    import torch
    if args.workload != "circuit28":
        import synth
        import paper_2311_01512_amd as qs
        fn = {"density14": bench_density, "batch512": bench_batch, "sv34": bench_sv34}[args.workload]
        print(json.dumps(fn(args, torch, qs, synth)), flush=True)
        return
    import synth
    import paper_2311_01512_amd as qs

    n, seed = args.qubits, 11
    workload = "circuit28" if (n, args.gates) == (28, 500) else f"circuit{n}_{args.gates}"
    ops = synth.config2_circuit(num_qubits=n, num_gates=args.gates)
    logical = synth.count_logical_updates(ops, n)

    # fused complex64: autotune the fusion width on a scratch run
    q64 = qs.Qureg(n, precision="c64").init_hashed(seed)
    fused = qs.Circuit(n, ops)
    cands = tuple(int(x) for x in args.fuse_candidates.split(","))
    best_k, tune_ms, spec_ms = autotune(fused, q64, cands, args)
    # plain complex128, one pass per gate
    plain = qs.Circuit(n, ops).compile(0, "c128")
    q128 = qs.Qureg(n, precision="c128")

    # one application of each path from the counter-hashed state: kept for
    # the comparison with the oracle's result
    q64.init_hashed(seed)
    q128.init_hashed(seed)
    fused.apply(q64)
    plain.apply(q128)
    torch.cuda.synchronize()
    saved = {"fused_c64": q64.tensor.clone(), "plain_c128": q128.tensor.clone()}
    with torch.no_grad():
        ref = saved["plain_c128"]
        err = ((saved["fused_c64"].to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()

    for _ in range(args.warmup):
        fused.apply(q64)
        plain.apply(q128)
    t64, kinds64 = timed_region(fused, q64, args.steps, torch)
    t128, kinds128 = timed_region(plain, q128, args.steps, torch, lines=line_amps(ops, n, 16))
    t64_plain_launch = time_steps(fused, q64, args.steps, torch)

    st = fused.stats()
    result = {
        "metric": "amplitude-updates/s & %HBM peak; fused FP32 vs plain FP64 at <=1e-5 amp err",
        "value": logical / t64,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (f32)",
        "data": "synthetic seeded random circuit (PCG64), counter-hashed initial state",
        "config": {"workload": f"{n}-qubit statevector, {len(ops)}-gate random circuit (Haar 1q, "
                               "2-target Haar with 0-3 controls, Pauli gadgets of weight 1-N)",
                   "num_qubits": n, "gates": len(ops),
                   "path": f"complex64, {path_text(best_k, fused.specialized > 0)} (fusion width autotuned)"},
        "roofline": roofline(kinds64, 8, workload),
        "fused_c64": {"value": logical / t64, "ms_per_step": t64 * 1e3,
                      "ms_per_step_without_pass_events": t64_plain_launch * 1e3, "fuse_k": best_k,
                      "autotune_ms": {str(k): v for k, v in tune_ms.items()},
                      "autotune_specialised_ms": spec_ms and {str(k): v for k, v in spec_ms.items()},
                      "specialised_kernels": fused.specialized,
                      "passes": st["num_passes"], "passes_by_width": st["passes_by_width"],
                      "max_amp_err_vs_c128": err, "per_kernel": per_kernel_table(kinds64, 8)},
        "plain_c128": {"value": logical / t128, "ms_per_step": t128 * 1e3, "passes": len(ops),
                       "roofline": roofline(kinds128, 16, workload), "per_kernel": per_kernel_table(kinds128, 16)},
        "speedup_fused_c64_vs_plain_c128": t128 / t64,
        "special_ops_c128": bench_special(q128, torch, 16),
        "special_ops_c64": bench_special(q64, torch, 8),
        "reductions_c128": bench_reductions(q128, torch, 16),
        "reductions_c64": bench_reductions(q64, torch, 8),
    }
    # fused complex128: tile steps, width autotuned, specialised
    del q128
    torch.cuda.empty_cache()
    f128 = qs.Circuit(n, ops)
    qf128 = qs.Qureg(n, precision="c128")
    k128, tune128, spec128 = autotune(f128, qf128, (0, 10, 11, 12, 13), args)
    qf128.init_hashed(seed)
    f128.apply(qf128)
    torch.cuda.synchronize()
    saved["fused_c128"] = qf128.tensor.clone()
    for _ in range(args.warmup):
        f128.apply(qf128)
    tf128, kindsf128 = timed_region(f128, qf128, args.steps, torch)
    result["fused_c128"] = {"value": logical / tf128, "ms_per_step": tf128 * 1e3, "fuse_k": k128,
                            "path": "complex128, " + path_text(k128, f128.specialized > 0),
                            "autotune_ms": {str(k): v for k, v in tune128.items()},
                            "autotune_specialised_ms": spec128 and {str(k): v for k, v in spec128.items()},
                            "passes": f128.stats()["num_passes"], "roofline": roofline(kindsf128, 16, workload),
                            "speedup_vs_plain_c128": t128 / tf128}
    del qf128, f128
    torch.cuda.empty_cache()
    # dense blocks of up to 6 qubits on the FP32 matrix cores (the 6-qubit
    # blocks are MFMA-bound: 32 flop/B at complex64)
    if not args.no_workloads:
        d6 = qs.Circuit(n, ops).compile(6, "c64")
        q64.init_hashed(seed)
        d6.apply(q64)
        td6, kindsd6 = timed_region(d6, q64, max(1, args.steps // 4), torch)
        result["dense_k6_c64"] = {"value": logical / td6, "ms_per_step": td6 * 1e3,
                                  "passes": d6.stats()["num_passes"],
                                  "passes_by_width": d6.stats()["passes_by_width"],
                                  "roofline": roofline({k: v for k, v in kindsd6.items()
                                                        if k.startswith("k_dense_mfma<6>")} or kindsd6, 8, workload),
                                  "per_kernel": per_kernel_table(kindsd6, 8)}
        del d6
    # the fastest in-house streaming kernel, for reading the roofline fraction
    stream = streaming_ceiling(qs, q64, torch)
    stream["frac_of_peak"] = stream["GBps"] / HBM_PEAK_GBS
    if result["roofline"]["unit"] == "GB/s":
        stream["roofline_achieved_over_streaming"] = result["roofline"]["achieved"] / stream["GBps"]
    result["streaming_ceiling"] = stream
    del q64
    torch.cuda.empty_cache()
    if not args.no_workloads:
        result["density14"] = bench_density(args, torch, qs, synth)
        batch_keep = {}
        result["batch512"] = bench_batch(args, torch, qs, synth, batch_keep)
    if not args.no_cpu_baseline:
        base, psi = cpu_baseline(ops, n, seed, args.cpu_runs)
        result["cpu_baseline"] = base
        want = torch.from_numpy(psi).to("cuda")
        del psi
        with torch.no_grad():
            scale = want.abs().max()
            errs = {k: ((v.to(torch.complex128) - want).abs().max() / scale).item() for k, v in saved.items()}
        result["max_amp_err_vs_oracle"] = errs
        result["fused_c64"]["max_amp_err_vs_oracle"] = errs["fused_c64"]
        result["plain_c128"]["max_amp_err_vs_oracle"] = errs["plain_c128"]
        result["fused_c128"]["max_amp_err_vs_oracle"] = errs["fused_c128"]
        del want
        if not args.no_workloads:
            result["batch512"]["vs_oracle"] = batch_vs_oracle(batch_keep)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
