"""Parity at the workloads' full sizes (28 and 34 qubits, the 14-qubit
density matrix, the 512-circuit batch) on sampled outputs the oracle
recomputes independently.

The states start from the counter-hashed state, which the oracle regenerates
entry by entry.  Circuits act only on a chosen set Q of qubits (spread over
low and high positions), so each coset {base | spread(m, Q)} evolves on its
own: the oracle runs the same ops on that 2^|Q|-entry sub-state and the
result must match the GPU's amplitudes of the coset element by element.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def coset_indices(base, Q):
    m = np.arange(1 << len(Q), dtype=np.uint64)
    idx = np.full(m.shape, np.uint64(base), dtype=np.uint64)
    for p, q in enumerate(Q):
        idx |= ((m >> np.uint64(p)) & np.uint64(1)) << np.uint64(q)
    return idx


def remap(ops, Q):
    pos = {q: p for p, q in enumerate(Q)}
    out = []
    for op in ops:
        o = dict(op)
        o["targs"] = tuple(pos[q] for q in op["targs"])
        if "ctrls" in op:
            o["ctrls"] = tuple(pos[q] for q in op["ctrls"])
        out.append(o)
    return out


def ops_on(rng, Q, num, max_targets=2, max_ctrls=3, gadget_weight=None):
    """Random ops whose qubits all lie in Q: Haar 1-qubit, Haar
    max_targets-target with 0..max_ctrls controls, Pauli gadgets."""
    ops = []
    gw = gadget_weight or len(Q)
    for _ in range(num):
        kind = int(rng.integers(0, 3))
        if kind == 0:
            ops.append({"op": "unitary", "ctrls": (), "targs": (int(rng.choice(Q)),),
                        "matrix": synth.haar_unitary(rng, 2)})
        elif kind == 1:
            s = int(rng.integers(0, max_ctrls + 1))
            qs_ = [int(x) for x in rng.choice(Q, size=max_targets + s, replace=False)]
            ops.append({"op": "unitary", "ctrls": tuple(qs_[max_targets:]), "targs": tuple(qs_[:max_targets]),
                        "matrix": synth.haar_unitary(rng, 1 << max_targets)})
        else:
            w = int(rng.integers(1, gw + 1))
            t = [int(x) for x in rng.choice(Q, size=w, replace=False)]
            ops.append({"op": "gadget", "targs": tuple(t), "paulis": tuple(int(x) for x in rng.integers(1, 4, size=w)),
                        "theta": float(rng.uniform(0, 2 * np.pi))})
    return ops


def gpu_gather(torch, q, idx):
    return q.tensor[torch.from_numpy(idx.astype(np.int64)).to(q.tensor.device)].cpu().numpy().astype(np.complex128)


def check_cosets(torch, q, n_bits, seed, Q, ops, rng, num_cosets, tol, density=False):
    others = np.uint64(((1 << n_bits) - 1) & ~sum(1 << x for x in Q))
    mini_ops = remap(ops, Q)
    worst = 0.0
    for _ in range(num_cosets):
        base = np.uint64(int(rng.integers(0, 1 << n_bits, dtype=np.uint64)) & int(others))
        idx = coset_indices(base, Q)
        mini = oracle.hashed_amps_at(n_bits, seed, idx)
        oracle.run_ops(mini, mini_ops, density=density)
        got = gpu_gather(torch, q, idx)
        worst = max(worst, amp_err(got, mini))
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("path", [("c128", 0), ("c64", 4), ("c64", 6), ("c64", 12), ("c128", 11)])
def test_28_qubits_sampled(qs, path):
    import torch
    prec, k = path
    banner(f"28 qubits {prec} fuse_k={k}")
    N, seed = 28, 2801
    rng = np.random.default_rng(28)
    Q = sorted([0, 1, 2, 27, 26] + [int(x) for x in rng.choice(np.arange(3, 26), size=7, replace=False)])
    ops = ops_on(rng, Q, 200)
    q = qs.Qureg(N, precision=prec).init_hashed(seed)
    circ = qs.Circuit(N, ops).compile(k, prec)
    circ.apply(q)
    check_cosets(torch, q, N, seed, Q, ops, rng, 24, TOL[prec])
    del q
    torch.cuda.empty_cache()


def test_28_qubits_single_ops_every_kernel(qs):
    """One op at a time on the full 28-qubit complex128 state, each kind of
    kernel and target position, sampled cosets."""
    import torch
    N, seed = 28, 2802
    rng = np.random.default_rng(29)
    q = qs.Qureg(N, precision="c128")
    cases = [
        [{"op": "unitary", "ctrls": (), "targs": (0,), "matrix": synth.haar_unitary(rng, 2)}],
        [{"op": "unitary", "ctrls": (), "targs": (27,), "matrix": synth.haar_unitary(rng, 2)}],
        [{"op": "unitary", "ctrls": (1, 20), "targs": (26, 0), "matrix": synth.haar_unitary(rng, 4)}],
        [{"op": "unitary", "ctrls": (), "targs": (3, 17, 0), "matrix": synth.random_matrix(rng, 8) / 3}],
        [{"op": "unitary", "ctrls": (5,), "targs": (27, 2, 9, 14, 1, 22), "matrix": synth.haar_unitary(rng, 64)}],
        [{"op": "gadget", "targs": (0, 5, 27, 13), "paulis": (1, 2, 3, 2), "theta": 0.7}],
        [{"op": "gadget", "targs": (4, 19), "paulis": (3, 3), "theta": -1.3}],
        [{"op": "swap", "targs": (27, 0)}],
        [{"op": "swap", "targs": (9, 21)}],
        [{"op": "pauli_tensor", "targs": (0, 26, 11, 3), "paulis": (2, 1, 3, 2)}],
        [{"op": "phase_gadget", "targs": (27, 2, 15), "theta": 0.9}],
    ]
    for ops in cases:
        banner(f"28q single op {ops[0]['op']} targs={ops[0]['targs']}")
        q.init_hashed(seed)
        q.run_ops(ops)
        Q = sorted(set(ops[0]["targs"]) | set(ops[0].get("ctrls", ())))
        check_cosets(torch, q, N, seed, Q, ops, rng, 64, TOL["c128"])
    del q
    torch.cuda.empty_cache()


def test_28_qubit_circuit_width13_plan(qs):
    """The 500-gate 28-qubit circuit that the benchmark times, in 2^13 tiles
    with specialised steps (complex64).  Its plan comes from a two-sweep
    admission rule (57 steps, one fewer than the plain greedy), whose steps
    list members out of circuit order where operators commute.  The result
    is checked against the plain per-gate complex128 path, which has no
    planner: a wrong order of two operators would show as an O(1) error."""
    import torch
    banner("28-qubit circuit, 2^13 tiles, specialised")
    N = 28
    ops = synth.config2_circuit(num_qubits=N, num_gates=500)
    fused = qs.Circuit(N, ops).compile(13, "c64")
    assert fused.stats()["num_passes"] <= 57
    assert fused.specialize() > 0
    q64 = qs.Qureg(N, precision="c64").init_hashed(9)
    q128 = qs.Qureg(N, precision="c128").init_hashed(9)
    fused.apply(q64)
    qs.Circuit(N, ops).compile(0, "c128").apply(q128)
    q64.sync()
    q128.sync()
    err = (q64.tensor.to(torch.complex128) - q128.tensor).abs().max().item()
    scale = q128.tensor.abs().max().item()
    assert err < 1e-5 * scale, (err, scale)
    del q64, q128
    torch.cuda.empty_cache()


def test_28_qubit_pauli_sum_by_term(qs):
    """The 20-term Pauli sum at full size (3 tile spans of flip masks, as
    timed) against a second route: each term applied to a copy by the
    Pauli-tensor kernel, then <psi|P psi> by the inner product, the
    coefficients summed on the host."""
    import torch
    n = 28
    rng = np.random.default_rng(20)
    codes = rng.integers(0, 4, size=(20, n)).astype(np.int32)
    coeffs = rng.standard_normal(20)
    for prec in ("c64", "c128"):
        banner(f"28-qubit Pauli sum by term {prec}")
        q = qs.Qureg(n, precision=prec).init_hashed(5)
        p = qs.Qureg(n, precision=prec)
        got = q.expec_pauli_sum(codes, coeffs)
        q.sync()
        want = 0.0
        for t in range(len(coeffs)):
            targs = [k for k in range(n) if codes[t, k]]
            p.tensor.copy_(q.tensor)
            torch.cuda.synchronize()
            p.apply_pauli_tensor(targs, [int(codes[t, k]) for k in targs])
            want += coeffs[t] * q.inner_product(p)
        # complex128: both routes form exact FP64 products; complex64 tiles
        # form each product in FP32 (relative rounding 2^-24 per product,
        # every sum in FP64), which the complex64 scalar bound covers
        bound = 1e-11 if prec == "c128" else 1e-5
        assert abs(got - want) < bound * np.abs(coeffs).sum(), (prec, got, want)
        del q, p
        torch.cuda.empty_cache()


def test_14_qubit_density_matrix_sampled(qs):
    """Choi vector of 2^28 entries, complex128: Kraus maps, DM unitaries and a
    gadget on qubits Q; cosets over Q and Q + N are mini density matrices."""
    import torch
    banner("14-qubit density matrix c128")
    N, seed = 14, 1401
    rng = np.random.default_rng(14)
    Qd = [0, 6, 13]
    ops = [{"op": "kraus", "targs": (0, 13), "kraus": synth.kraus_random_isometry(rng, 2, 4)},
           {"op": "unitary", "ctrls": (), "targs": (6, 0), "matrix": synth.haar_unitary(rng, 4)},
           {"op": "kraus", "targs": (6,), "kraus": synth.kraus_depolarising_1q(0.04)},
           {"op": "unitary", "ctrls": (13,), "targs": (6,), "matrix": synth.haar_unitary(rng, 2)},
           {"op": "kraus", "targs": (13,), "kraus": synth.kraus_damping_1q(0.08)},
           {"op": "gadget", "targs": (0, 6, 13), "paulis": (2, 1, 3), "theta": 0.4},
           {"op": "swap", "targs": (13, 0)},
           {"op": "pauli_tensor", "targs": (6, 13), "paulis": (2, 1)},
           {"op": "phase_gadget", "targs": (0, 13), "theta": -0.8},
           {"op": "gadget", "targs": (6,), "paulis": (2,), "theta": 1.2}]
    q = qs.Qureg(N, density=True, precision="c128").init_hashed(seed)
    q.run_ops(ops)
    # Choi index bits: Qd on the row half, Qd + N on the column half
    Qc = Qd + [x + N for x in Qd]
    check_cosets(torch, q, 2 * N, seed, Qc, remap_dm(ops, Qd), rng, 32, TOL["c128"], density=True)
    del q
    torch.cuda.empty_cache()


def remap_dm(ops, Qd):
    """Express DM ops on qubits Qd so that remap(ops, Qc) with Qc = Qd + Qd+N
    yields mini-DM ops on qubits 0..len(Qd)-1 (identity: the first half of Qc
    is Qd itself)."""
    return ops


def test_14_qubit_partial_trace_sampled(qs):
    """Partial trace of the 2^28-entry hashed Choi vector over 7 qubits:
    each sampled output is the trace of a 7-qubit sub-matrix the oracle
    builds from the hashed generator."""
    import torch
    banner("14-qubit partial trace c128")
    N, seed = 14, 1402
    rng = np.random.default_rng(15)
    traced = sorted(int(x) for x in rng.choice(N, size=7, replace=False))
    kept = [x for x in range(N) if x not in traced]
    q = qs.Qureg(N, density=True, precision="c128").init_hashed(seed)
    red = q.partial_trace(traced)
    got_all = red.get_amps()
    m = len(kept)
    for _ in range(40):
        i = int(rng.integers(0, 1 << (2 * m)))
        k_red, l_red = i & ((1 << m) - 1), i >> m
        k0 = sum(((k_red >> p) & 1) << q_ for p, q_ in enumerate(kept))
        l0 = sum(((l_red >> p) & 1) << q_ for p, q_ in enumerate(kept))
        # mini 7-qubit matrix over the traced qubits: rows k0 | f(v1), columns l0 | f(v2)
        v = np.arange(1 << 7, dtype=np.uint64)
        f = np.zeros_like(v)
        for p, q_ in enumerate(traced):
            f |= ((v >> np.uint64(p)) & np.uint64(1)) << np.uint64(q_)
        rows = np.uint64(k0) | f
        cols = np.uint64(l0) | f
        choi_idx = (rows[:, None] + (cols[None, :] << np.uint64(N))).flatten(order="F")
        mini = oracle.hashed_amps_at(2 * N, seed, choi_idx)
        want = oracle.dm_trace(np.ascontiguousarray(mini))
        assert abs(got_all[i] - want) < 1e-12 * max(1.0, abs(want)), (i, got_all[i], want)
    del q, red
    torch.cuda.empty_cache()


def test_512_circuit_batch_sampled(qs):
    """The full 512-circuit batch in one replay; the smallest circuits'
    energies and gradients against the oracle."""
    banner("batch 512")
    probs = synth.config4_batch()
    b = qs.Batch("c64")
    for p in probs:
        b.add_circuit(p["num_qubits"], p["ops"], len(p["angles"]), p["codes"], p["coeffs"])
    b.compile()
    params = np.concatenate([p["angles"] for p in probs])
    e, g = b.run(params)
    offs = np.cumsum([0] + [len(p["angles"]) for p in probs])
    order = np.argsort([p["num_qubits"] for p in probs], kind="stable")
    for ci in list(order[:3]) + [int(order[len(order) // 2])]:
        p = probs[ci]
        n, mm = p["num_qubits"], len(p["angles"])
        if n > 16:
            continue
        psi = oracle.run_ops(oracle.zero_state(n), p["ops"])
        assert abs(e[ci] - oracle.sv_expec_pauli_sum(psi, p["codes"], p["coeffs"]).real) < 1e-4
        want = oracle.param_shift_gradient(n, p["ops"], p["codes"], p["coeffs"], mm)
        got = g[offs[ci]:offs[ci] + mm]
        assert np.abs(got - want).max() < 1e-4 * max(1.0, np.abs(want).max())


def test_34_qubits_sampled(qs):
    """2^34 complex64 amplitudes (128 GiB): 5-target Haar gates with up to 4
    controls and gadgets, fused (k = 6) and plain, on 12 qubits spread over
    the register; sampled cosets against the oracle; closed forms of
    <Z_0 Z_33> and the norm at full size."""
    import torch
    N, seed = 34, 3401
    rng = np.random.default_rng(34)
    Q = sorted([0, 1, 2, 3, 33, 32, 31] + [int(x) for x in rng.choice(np.arange(4, 31), size=5, replace=False)])
    ops = ops_on(rng, Q, 12, max_targets=5, max_ctrls=4, gadget_weight=12)
    q = qs.Qureg(N, precision="c64")
    for k in (6, 0, 12):
        banner(f"34 qubits fuse_k={k}")
        q.init_hashed(seed)
        n0 = q.total_prob()
        qs.Circuit(N, ops).compile(k, "c64").apply(q)
        check_cosets(torch, q, N, seed, Q, ops, rng, 8, TOL["c64"])
        assert abs(q.total_prob() - n0) < 1e-5 * n0
    zz = np.zeros((1, N), np.int32)
    zz[0, 0] = zz[0, N - 1] = 3
    q.init_basis((1 << 33) | 6)
    assert abs(q.expec_pauli_sum(zz, [1.0]) - (-1.0)) < 1e-6
    q.init_plus()
    assert abs(q.total_prob() - 1.0) < 1e-5
    assert abs(q.expec_pauli_sum(zz, [1.0])) < 1e-6
    del q
    torch.cuda.empty_cache()
