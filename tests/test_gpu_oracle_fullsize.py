"""Whole-state parity with the FP64 oracle at the sizes the benchmark
measures: every amplitude of the 28-qubit 500-gate circuit, of the
5-target circuit generator at 28 qubits, and of the 14-qubit density matrix
after its 300 operators (the full 2^28-entry Choi vector, its partial trace
over 7 qubits, trace and purity), and the energies of all 512 batched
circuits with sampled gradients of circuits of 17 or more qubits.

The oracle runs on the host cores (tens of seconds to a few minutes per
workload, once per module); its result is uploaded to the GPU, where the
error of each GPU path is taken as max_i |got_i - want_i| / max_i |want_i|.
Tolerances: complex128 1e-12, complex64 1e-5 (relative to the largest
amplitude); scalars as stated in each test.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, banner, progress, run_oracle_ops

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def _to_gpu(torch, a):
    return torch.from_numpy(a).to("cuda")


def gpu_err(torch, q, ref):
    """Normalised max-abs error of qureg q against the oracle state ref (a
    complex128 tensor on the GPU)."""
    q.sync()
    with torch.no_grad():
        return ((q.tensor.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()


# ---- 28-qubit 500-gate circuit (the headline workload) --------------------------------

HEAD_N, HEAD_SEED = 28, 11


@pytest.fixture(scope="module")
def headline(qs, request):
    import torch
    banner("oracle: 28-qubit 500-gate circuit from the counter-hashed state (seed 11)")
    ops = synth.config2_circuit(num_qubits=HEAD_N, num_gates=500)
    psi = oracle.hashed_state(HEAD_N, HEAD_SEED)
    run_oracle_ops(request, psi, ops, label="28-qubit circuit")
    norm = oracle.sv_total_prob(psi)
    zz = np.zeros((1, HEAD_N), np.int32)
    zz[0, 0] = zz[0, HEAD_N - 1] = 3
    ezz = oracle.sv_expec_pauli_sum(psi, zz, [1.0]).real
    p27 = oracle.sv_prob_of_outcome(psi, HEAD_N - 1, 0)
    ref = _to_gpu(torch, psi)
    del psi
    yield {"ops": ops, "ref": ref, "norm": norm, "zz": (zz, ezz), "p27": p27}
    del ref
    torch.cuda.empty_cache()


def test_headline_plain_c128(qs, headline):
    import torch
    banner("28q circuit: plain per-gate complex128 vs oracle")
    q = qs.Qureg(HEAD_N, precision="c128").init_hashed(HEAD_SEED)
    qs.Circuit(HEAD_N, headline["ops"]).compile(0, "c128").apply(q)
    err = gpu_err(torch, q, headline["ref"])
    print(f"[gpu-test] plain c128 err {err:.3e}", flush=True)
    assert err < TOL["c128"], err
    assert abs(q.total_prob() - headline["norm"]) < 1e-12 * headline["norm"]
    zz, ezz = headline["zz"]
    assert abs(q.expec_pauli_sum(zz, [1.0]) - ezz) < 1e-12
    assert abs(q.prob_of_outcome(HEAD_N - 1, 0) - headline["p27"]) < 1e-12
    del q
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,k,spec", [("c64", 13, True), ("c64", 12, False), ("c64", 12, True),
                                         ("c64", 5, False), ("c64", 0, False), ("c128", 11, True)])
def test_headline_fused(qs, headline, prec, k, spec):
    """Fused paths: tile steps (generic kernel or specialised per step),
    dense blocks on the matrix cores, plain complex64."""
    import torch
    banner(f"28q circuit: {prec} width {k} specialised={spec} vs oracle")
    q = qs.Qureg(HEAD_N, precision=prec).init_hashed(HEAD_SEED)
    c = qs.Circuit(HEAD_N, headline["ops"]).compile(k, prec)
    if spec:
        assert c.specialize() > 0
    c.apply(q)
    err = gpu_err(torch, q, headline["ref"])
    print(f"[gpu-test] {prec} k={k} spec={spec} err {err:.3e}", flush=True)
    assert err < TOL[prec], err
    assert abs(q.total_prob() - headline["norm"]) < TOL[prec] * headline["norm"]
    del q, c
    torch.cuda.empty_cache()


def test_headline_autotuned(qs, headline):
    """The form the benchmark times: the autotuner's choice over plain, dense
    blocks and tile steps (generic and specialised), complex64."""
    import torch
    banner("28q circuit: autotuned complex64 vs oracle")
    q = qs.Qureg(HEAD_N, precision="c64")
    c = qs.Circuit(HEAD_N, headline["ops"])
    best, _, _ = c.autotune(q, (0, 4, 5, 10, 11, 12, 13), specialize=True)
    q.init_hashed(HEAD_SEED)
    c.apply(q)
    err = gpu_err(torch, q, headline["ref"])
    print(f"[gpu-test] autotuned k={best} specialised={c.specialized} err {err:.3e}", flush=True)
    assert err < TOL["c64"], err
    del q, c
    torch.cuda.empty_cache()


# ---- 5-target circuit generator at 28 qubits ---------------------------------------

C5_N, C5_SEED = 28, 12


@pytest.fixture(scope="module")
def config5(qs, request):
    import torch
    banner("oracle: 5-target circuit generator at 28 qubits")
    ops = synth.config5_circuit(num_qubits=C5_N)
    psi = oracle.hashed_state(C5_N, C5_SEED)
    run_oracle_ops(request, psi, ops, label="5-target circuit at 28 qubits")
    zz = np.zeros((1, C5_N), np.int32)
    zz[0, 0] = zz[0, C5_N - 1] = 3
    ezz = oracle.sv_expec_pauli_sum(psi, zz, [1.0]).real
    norm = oracle.sv_total_prob(psi)
    ref = _to_gpu(torch, psi)
    del psi
    yield {"ops": ops, "ref": ref, "zz": (zz, ezz), "norm": norm}
    del ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,k,spec", [("c128", 0, False), ("c64", 0, False), ("c64", 6, False),
                                         ("c64", 12, True), ("c64", 13, True)])
def test_config5_28q(qs, config5, prec, k, spec):
    import torch
    banner(f"config5 28q: {prec} k={k} specialised={spec} vs oracle")
    q = qs.Qureg(C5_N, precision=prec).init_hashed(C5_SEED)
    c = qs.Circuit(C5_N, config5["ops"]).compile(k, prec)
    if spec:
        c.specialize()
    c.apply(q)
    err = gpu_err(torch, q, config5["ref"])
    print(f"[gpu-test] config5 {prec} k={k} err {err:.3e}", flush=True)
    assert err < TOL[prec], err
    zz, ezz = config5["zz"]
    assert abs(q.expec_pauli_sum(zz, [1.0]) - ezz) < TOL[prec]
    assert abs(q.total_prob() - config5["norm"]) < TOL[prec] * config5["norm"]
    del q, c
    torch.cuda.empty_cache()


# ---- 14-qubit density matrix, 300 operators ---------------------------------------

DM_N = 14


@pytest.fixture(scope="module")
def density(qs, request):
    import torch
    banner("oracle: 14-qubit density matrix, 300 operators from |0><0|")
    ops, traced = synth.config3_circuit()
    rho = run_oracle_ops(request, oracle.zero_state(DM_N, density=True), ops, density=True,
                         label="14-qubit density matrix")
    red = oracle.partial_trace(rho, traced)
    out = {"ops": ops, "traced": traced, "trace": oracle.dm_trace(rho), "purity": oracle.dm_purity(rho),
           "red": red, "red_trace": oracle.dm_trace(red), "red_purity": oracle.dm_purity(red)}
    out["ref"] = _to_gpu(torch, rho)
    del rho
    yield out
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,k,spec", [("c128", None, False), ("c64", None, False), ("c64", 12, True),
                                         ("c64", 12, False), ("c64", 5, False), ("c128", 11, True)])
def test_density_14q(qs, density, prec, k, spec):
    """k = None: the per-operator API (the paper's two passes per unitary,
    one superoperator pass per Kraus map); otherwise the density circuit
    compiled at width k."""
    import torch
    banner(f"density 14q: {prec} k={k} specialised={spec} vs oracle")
    q = qs.Qureg(DM_N, density=True, precision=prec).init_zero()
    if k is None:
        q.run_ops(density["ops"])
    else:
        c = qs.Circuit(DM_N, density["ops"], density=True).compile(k, prec)
        if spec:
            c.specialize()
        c.apply(q)
    err = gpu_err(torch, q, density["ref"])
    print(f"[gpu-test] density {prec} k={k} err {err:.3e}", flush=True)
    assert err < TOL[prec], err
    tol = TOL[prec]
    assert abs(q.trace() - density["trace"]) < tol
    assert abs(q.purity() - density["purity"]) < tol
    red = q.partial_trace(density["traced"])
    got = red.get_amps()
    want = density["red"]
    assert np.abs(got - want).max() / np.abs(want).max() < tol
    assert abs(red.trace() - density["red_trace"]) < tol
    assert abs(red.purity() - density["red_purity"]) < tol
    del q, red
    torch.cuda.empty_cache()


def test_density_partial_trace_13_of_14(qs, density):
    """Tracing out 13 of the 14 qubits (26 spliced index bits), every single
    kept qubit, and the traced set of the workload, on the oracle's final
    state uploaded to the GPU."""
    import torch
    banner("density 14q: partial traces of the oracle state")
    q = qs.Qureg(DM_N, density=True, precision="c128")
    q.tensor.copy_(density["ref"])
    torch.cuda.synchronize()
    rho = density["ref"].cpu().numpy()
    for keep in (0, 6, 13):
        traced = [x for x in range(DM_N) if x != keep]
        red = q.partial_trace(traced)
        want = oracle.partial_trace(rho, traced)
        assert np.abs(red.get_amps() - want).max() < 1e-12 * np.abs(want).max(), keep
    del q, rho
    torch.cuda.empty_cache()


# ---- 512 batched circuits ------------------------------------------------------------

@pytest.fixture(scope="module")
def batch_ref(qs, request):
    import time
    banner("oracle: energies of the 512 batched circuits")
    probs = synth.config4_batch()
    energies = np.empty(len(probs))
    t0 = last = time.perf_counter()
    for i, p in enumerate(probs):
        psi = oracle.run_ops(oracle.zero_state(p["num_qubits"]), p["ops"])
        energies[i] = oracle.sv_expec_pauli_sum(psi, p["codes"], p["coeffs"]).real
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            progress(request, f"batch energies: {i + 1}/{len(probs)} circuits, {last - t0:.0f} s")
    progress(request, f"batch energies: {len(probs)} circuits in {time.perf_counter() - t0:.1f} s")
    return probs, energies


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_batch_512_energies_and_gradients(qs, batch_ref, prec):
    """All 512 energies against the oracle; the gradients of two circuits
    of 17 or more qubits on 12 sampled parameters each against the oracle's
    exact two-term shift rule.  Energy tolerance: the precision's bound times
    sum |h_n| (the largest |<psi|H|psi>| a normalised state can give);
    gradients: 1e-10 (complex128), 1e-4 max|g| (complex64)."""
    banner(f"batch 512 {prec} vs oracle")
    probs, want_e = batch_ref
    b = qs.Batch(prec)
    for p in probs:
        b.add_circuit(p["num_qubits"], p["ops"], len(p["angles"]), p["codes"], p["coeffs"])
    b.compile()
    params = np.concatenate([p["angles"] for p in probs])
    e, g = b.run(params)
    hnorm = np.array([np.abs(p["coeffs"]).sum() for p in probs])
    rel = np.abs(e - want_e) / hnorm
    print(f"[gpu-test] batch {prec} worst energy error / sum|h| {rel.max():.3e}", flush=True)
    assert rel.max() < TOL[prec], rel.max()
    offs = np.cumsum([0] + [len(p["angles"]) for p in probs])
    rng = np.random.default_rng(17)
    big = [i for i, p in enumerate(probs) if 17 <= p["num_qubits"] <= 19]
    for ci in rng.choice(big, size=2, replace=False):
        p = probs[int(ci)]
        n = p["num_qubits"]
        pick = np.sort(rng.choice(len(p["angles"]), size=12, replace=False))
        want = sampled_shift_gradient(n, p["ops"], p["codes"], p["coeffs"], pick)
        got = g[offs[ci] + pick]
        bound = 1e-10 if prec == "c128" else 1e-4 * max(1.0, np.abs(want).max())
        assert np.abs(got - want).max() < bound, (int(ci), n, np.abs(got - want).max())


def sampled_shift_gradient(num_qubits, ops, codes, coeffs, params):
    """dE/dparameter for the listed parameters by the oracle's exact
    two-term rule for exp(i theta P) (each parameter drives one gadget)."""
    out = []
    for k in params:
        idx = [i for i, op in enumerate(ops) if op.get("param") == k]
        assert len(idx) == 1
        i = idx[0]
        e = []
        for delta in (np.pi / 4, -np.pi / 4):
            shifted = list(ops)
            shifted[i] = dict(ops[i], theta=ops[i]["theta"] + delta)
            psi = oracle.run_ops(oracle.zero_state(num_qubits), shifted)
            e.append(oracle.sv_expec_pauli_sum(psi, codes, coeffs).real)
        out.append(ops[i].get("scale", 1.0) * (e[0] - e[1]))
    return np.array(out)
