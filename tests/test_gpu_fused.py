"""Parity of the FP32-MFMA dense kernel and of fused circuits (dense k-qubit
blocks built in FP64) with the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner

pytestmark = pytest.mark.gpu


def trajectory(psi, ops):
    """The oracle's final state and the largest amplitude magnitude of any
    intermediate state.  With operators that are not unitary, each rounding
    error is made relative to the amplitudes present when its operator runs,
    so errors are normalised by this peak rather than by the final state's
    largest amplitude (the reading stated with the tolerances)."""
    state = psi.copy()
    peak = np.abs(state).max()
    for op in ops:
        oracle.run_ops(state, [op])
        peak = max(peak, np.abs(state).max())
    return state, peak


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


DENSE_CASES = [
    # (N, targets, controls): low, high, mixed target sets, with and without controls
    (8, [0, 1, 2, 3], []), (9, [3, 0, 8, 5], []), (12, [11, 10, 9, 8, 7], []), (12, [0, 5, 1, 9, 3], [11]),
    (13, [2, 4, 6, 8, 10, 12], []), (14, [0, 1, 2, 3, 4, 5], [13, 7]), (15, [14, 0, 7, 3, 11, 5], [1, 2, 9]),
    (16, [6, 7, 8, 9], [0, 1, 2, 3]), (5, [0, 1, 2, 3], []), (6, [5, 4, 3, 2, 1], [0]),
]


@pytest.mark.parametrize("case", range(len(DENSE_CASES)))
def test_mfma_dense_gate_parity(qs, case):
    N, t, c = DENSE_CASES[case]
    banner(f"mfma dense N={N} t={t} c={c}")
    rng = np.random.default_rng(7000 + case)
    M = synth.haar_unitary(rng, 1 << len(t))
    psi = synth.random_state(rng, 1 << N)
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    q.apply_unitary(c, t, M)
    want = oracle.apply_gate(psi.copy(), c, t, M)
    assert amp_err(q.get_amps(), want) < TOL["c64"]


def test_mfma_nonunitary_many_tiles(qs):
    """A general matrix on 6 targets of 18 qubits (4096 tiles of 16 groups)."""
    rng = np.random.default_rng(7100)
    N, t = 18, [17, 2, 9, 0, 13, 5]
    M = synth.random_matrix(rng, 64) / 8
    psi = synth.random_state(rng, 1 << N)
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    q.apply_unitary([], t, M)
    assert amp_err(q.get_amps(), oracle.apply_gate(psi.copy(), [], t, M)) < TOL["c64"]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("k", [0, 2, 3, 4, 5, 6, 8, 10, 11, 12])
def test_fused_circuit_parity(qs, prec, k):
    banner(f"fused circuit k={k} {prec}")
    N = 14
    ops = synth.config2_circuit(num_qubits=N, num_gates=300)
    rng = np.random.default_rng(3)
    psi = synth.random_state(rng, 1 << N)
    circ = qs.Circuit(N, ops).compile(k, prec)
    st = circ.stats()
    assert st["num_ops"] == len(ops)
    assert st["logical_updates"] == synth.count_logical_updates(ops, N)
    if k == 0:
        assert st["num_passes"] == len(ops)
    else:
        assert st["num_passes"] < len(ops)
        if k <= 6:
            assert max(i for i, w in enumerate(st["passes_by_width"]) if w) <= k
        else:
            kinds = [circ.pass_info(i)["kernel"] for i in range(st["num_passes"])]
            assert kinds.count("tile") >= 1
            assert all(circ.pass_info(i)["num_targs"] <= k for i in range(st["num_passes"])
                       if kinds[i] == "tile")
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    circ.apply(q)
    want = oracle.run_ops(psi.copy(), ops)
    assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("k", [2, 3, 4, 6, 8, 9])
def test_fusion_respects_order(qs, k, prec):
    """Dense non-commuting gates on overlapping qubits, interleaved with gates
    elsewhere: blocks may only absorb ops that commute with what they skip."""
    rng = np.random.default_rng(11 + k)
    N = 10
    ops = []
    for g in range(120):
        a = int(rng.integers(0, N))
        b = (a + int(rng.integers(1, 3))) % N
        if g % 3 == 0:
            ops.append({"op": "unitary", "ctrls": (), "targs": (a, b), "matrix": synth.random_matrix(rng, 4) / 2})
        elif g % 3 == 1:
            ops.append({"op": "unitary", "ctrls": (b,), "targs": (a,), "matrix": synth.random_matrix(rng, 2)})
        else:
            w = int(rng.integers(1, 4))
            qs_ = rng.permutation(N)[:w]
            ops.append({"op": "gadget", "targs": tuple(int(x) for x in qs_),
                        "paulis": tuple(int(x) for x in rng.integers(0, 4, size=w)), "theta": rng.uniform(-3, 3)})
    psi = synth.random_state(rng, 1 << N)
    want, peak = trajectory(psi, ops)
    circ = qs.Circuit(N, ops).compile(k, prec)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    circ.apply(q)
    err = np.abs(q.get_amps() - want).max() / peak
    print(f"[gpu-test] non-unitary k={k} {prec}: error / trajectory peak {err:.2e}", flush=True)
    assert err < TOL[prec], err


@pytest.mark.parametrize("k", [9, 10, 12])
def test_tile_matrix_core_gates(qs, k):
    """Tile steps in complex64 with 2-, 3- and 4-target gates (the matrix-core
    operators, two targets on lane coordinates), controls, 1-target gates and
    gadgets interleaved."""
    banner(f"tile mfma gates N=13 k={k}")
    N = 13
    rng = np.random.default_rng(300 + k)
    ops = []
    for g in range(160):
        kind = g % 5
        if kind in (0, 1, 2):
            nt = 2 + kind
            q = rng.permutation(N)
            nc = int(rng.integers(0, 3))
            ops.append({"op": "unitary", "ctrls": tuple(int(x) for x in q[nt:nt + nc]),
                        "targs": tuple(int(x) for x in q[:nt]), "matrix": synth.haar_unitary(rng, 1 << nt)})
        elif kind == 3:
            ops.append({"op": "unitary", "ctrls": (), "targs": (int(rng.integers(0, N)),),
                        "matrix": synth.haar_unitary(rng, 2)})
        else:
            w = int(rng.integers(1, N + 1))
            t = rng.permutation(N)[:w]
            ops.append({"op": "gadget", "targs": tuple(int(x) for x in t),
                        "paulis": tuple(int(x) for x in rng.integers(1, 4, size=w)), "theta": rng.uniform(-3, 3)})
    psi = synth.random_state(rng, 1 << N)
    circ = qs.Circuit(N, ops).compile(k, "c64")
    kinds = [circ.pass_info(i)["kernel"] for i in range(circ.stats()["num_passes"])]
    assert kinds.count("tile") >= 1
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    circ.apply(q)
    assert amp_err(q.get_amps(), oracle.run_ops(psi.copy(), ops)) < TOL["c64"]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("k", [10, 12])
def test_tile_sparse_gates(qs, prec, k):
    """Tile steps with the sparse register forms: diagonal 1- and 2-target
    gates and 2-target gates coupling each member with one partner (j and
    j ^ s), among dense gates and gadgets."""
    banner(f"tile sparse gates N=12 k={k} {prec}")
    N = 12
    rng = np.random.default_rng(500 + k)
    ops = []
    for g in range(150):
        kind = g % 5
        q = [int(x) for x in rng.permutation(N)[:2]]
        if kind == 0:
            m = np.diag(np.exp(1j * rng.uniform(0, 6, size=2)))
            ops.append({"op": "unitary", "ctrls": (), "targs": (q[0],), "matrix": m})
        elif kind == 1:
            m = np.diag(rng.normal(size=4) + 1j * rng.normal(size=4)) / 2
            ops.append({"op": "unitary", "ctrls": (), "targs": tuple(q), "matrix": m})
        elif kind == 2:
            s_ = int(rng.integers(1, 4))
            m = synth.random_matrix(rng, 4) / 2
            for r in range(4):
                for c in range(4):
                    if (r ^ c) not in (0, s_):
                        m[r, c] = 0
            ops.append({"op": "unitary", "ctrls": (), "targs": tuple(q), "matrix": m})
        elif kind == 3:
            ops.append({"op": "unitary", "ctrls": (), "targs": (q[0],), "matrix": synth.haar_unitary(rng, 2)})
        else:
            w = int(rng.integers(1, N + 1))
            t = rng.permutation(N)[:w]
            ops.append({"op": "gadget", "targs": tuple(int(x) for x in t),
                        "paulis": tuple(int(x) for x in rng.integers(1, 4, size=w)), "theta": rng.uniform(-3, 3)})
    psi = synth.random_state(rng, 1 << N)
    want, peak = trajectory(psi, ops)
    circ = qs.Circuit(N, ops).compile(k, prec)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    circ.apply(q)
    err = np.abs(q.get_amps() - want).max() / peak
    print(f"[gpu-test] sparse k={k} {prec}: error / trajectory peak {err:.2e}", flush=True)
    assert err < TOL[prec], err


def test_config5_fused_reduced(qs):
    """The 34-qubit generator at 14 qubits: 5-target gates with up to 4
    controls and heavy gadgets, fused with k = 6 in complex64."""
    banner("config5 fused N=14")
    N = 14
    ops = synth.config5_circuit(num_qubits=N)
    rng = np.random.default_rng(5)
    psi = synth.random_state(rng, 1 << N)
    circ = qs.Circuit(N, ops).compile(6, "c64")
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    circ.apply(q)
    want = oracle.run_ops(psi.copy(), ops)
    assert amp_err(q.get_amps(), want) < TOL["c64"]


def test_circuit_errors(qs):
    c = qs.Circuit(4)
    with pytest.raises(ValueError):
        c.add({"op": "unitary", "ctrls": (0,), "targs": (0,), "matrix": np.eye(2)})
    with pytest.raises(ValueError):
        c.add({"op": "kraus", "targs": (0,), "kraus": np.eye(2)[None]})
    c.add({"op": "unitary", "ctrls": (), "targs": (1,), "matrix": np.eye(2)})
    q = qs.Qureg(4, precision="c64").init_zero()
    with pytest.raises(ValueError):
        c.apply(q)                                   # not compiled
    c.compile(0, "c128")
    with pytest.raises(TypeError):
        c.apply(q)                                   # compiled for the other precision
    with pytest.raises(ValueError):
        c.compile(7, "c64")


def _random_mixed_ops(rng, N, count):
    """Every operator shape the compilers handle: 1-4 target gates (dense,
    diagonal, paired-sparse) with 0-4 controls, gadgets of any weight
    including all-Z ones."""
    ops = []
    for _ in range(count):
        kind = int(rng.integers(0, 6))
        q = [int(x) for x in rng.permutation(N)]
        if kind <= 2:
            nt = int(rng.integers(1, 5))
            nc = int(rng.integers(0, min(5, N - nt) + 1))
            m = synth.haar_unitary(rng, 1 << nt)
            if kind == 2 and nt <= 2:
                s_ = int(rng.integers(0, 1 << nt))
                m = m * np.array([[1 if (r ^ c) in (0, s_) else 0 for c in range(1 << nt)] for r in range(1 << nt)])
            ops.append({"op": "unitary", "ctrls": tuple(q[nt:nt + nc]), "targs": tuple(q[:nt]), "matrix": m})
        else:
            w = int(rng.integers(1, N + 1))
            codes = rng.integers(1, 4, size=w) if kind != 5 else np.full(w, 3)
            ops.append({"op": "gadget", "targs": tuple(q[:w]), "paulis": tuple(int(c) for c in codes),
                        "theta": rng.uniform(-3, 3)})
    return ops


@pytest.mark.parametrize("seed", range(6))
def test_random_circuits_every_compile(qs, seed):
    """Random circuits compiled plain, as dense blocks and as tile steps of
    several widths, in both precisions, against the oracle."""
    rng = np.random.default_rng(4000 + seed)
    N = int(rng.integers(9, 13))
    ops = _random_mixed_ops(rng, N, 120)
    psi = synth.random_state(rng, 1 << N)
    want = oracle.run_ops(psi.copy(), ops)
    for prec in ("c128", "c64"):
        for k in (0, 4, 8, 9, 10, 11, 12):
            banner(f"random circuit seed={seed} N={N} k={k} {prec}")
            circ = qs.Circuit(N, ops).compile(k, prec)
            q = qs.Qureg(N, precision=prec).set_amps(psi)
            circ.apply(q)
            assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("k", [8, 9, 10])
def test_tiles_move_commuting_operators(qs, k, prec):
    """Tile steps move an operator ahead of skipped ones it commutes with:
    gadgets whose Pauli strings commute though they overlap (XX and ZZ on the
    same pair, Z strings), gadgets that are Z on a gate's controls, gates that
    share only controls; mixed with pairs that do not commute."""
    banner(f"commuting operators k={k} {prec}")
    rng = np.random.default_rng(31 + k)
    N = 12
    ops = []
    for g in range(160):
        a, b, c, d = (int(x) for x in rng.permutation(N)[:4])
        kind = g % 6
        if kind == 0:
            ops.append({"op": "gadget", "targs": (a, b), "paulis": (1, 1), "theta": rng.uniform(-3, 3)})
            ops.append({"op": "gadget", "targs": (a, b), "paulis": (3, 3), "theta": rng.uniform(-3, 3)})
        elif kind == 1:
            ops.append({"op": "unitary", "ctrls": (c,), "targs": (a, b), "matrix": synth.haar_unitary(rng, 4)})
            ops.append({"op": "gadget", "targs": (c, d), "paulis": (3, 3),
                        "theta": rng.uniform(-3, 3)})
        elif kind == 2:
            ops.append({"op": "unitary", "ctrls": (c,), "targs": (a,), "matrix": synth.haar_unitary(rng, 2)})
            ops.append({"op": "unitary", "ctrls": (c,), "targs": (b,), "matrix": synth.haar_unitary(rng, 2)})
        elif kind == 3:
            w = int(rng.integers(2, 7))
            t = tuple(int(x) for x in rng.permutation(N)[:w])
            ops.append({"op": "gadget", "targs": t, "paulis": tuple(int(x) for x in rng.integers(1, 4, size=w)),
                        "theta": rng.uniform(-3, 3)})
        elif kind == 4:
            ops.append({"op": "gadget", "targs": (a,), "paulis": (1,), "theta": rng.uniform(-3, 3)})
            ops.append({"op": "gadget", "targs": (a,), "paulis": (3,), "theta": rng.uniform(-3, 3)})
        else:
            ops.append({"op": "unitary", "ctrls": (), "targs": (a, b), "matrix": synth.haar_unitary(rng, 4)})
    psi = synth.random_state(rng, 1 << N)
    want = oracle.run_ops(psi.copy(), ops)
    circ = qs.Circuit(N, ops).compile(k, prec)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    circ.apply(q)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    if circ.specialize():
        q.set_amps(psi)
        circ.apply(q)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("k", [8, 10])
def test_tile_member_fusion(qs, prec, k):
    """Operators that tile steps fuse into one matrix (uncontrolled gates whose
    targets nest inside another's, with commuting operators between them)
    next to ones they must not fuse with (a controlled gate or a gadget on
    the same qubit in between), against the oracle, generic and specialised."""
    banner(f"tile member fusion {prec} k={k}")
    N = 11
    rng = np.random.default_rng(910 + k)

    def u(targs, ctrls=()):
        return {"op": "unitary", "ctrls": tuple(ctrls), "targs": tuple(targs),
                "matrix": synth.haar_unitary(rng, 1 << len(targs))}

    ops = []
    for rep in range(12):
        a, b, c, d, e = (int(x) for x in rng.permutation(N)[:5])
        # u(a) joins u(a, b) across the commuting u(d); u(b) joins it too
        ops += [u([a]), u([d]), u([a, b]), u([b]), u([e, d])]
        # the controlled gate on a is not fused, and nothing on a fuses across it
        ops += [u([b, a]), u([a], [c]), u([a])]
        # nor across the gadget on c and e
        ops += [u([c]), {"op": "gadget", "targs": (c, e), "paulis": (1, 3), "theta": 0.3 + rep}, u([c, e])]
        # nested target sets of 1 to 4 qubits (4: the matrix cores in complex64)
        ops += [u([a, b, c]), u([c]), u([b, a]), u([a, b, c, d]), u([d]), u([b, d])]
    psi = synth.random_state(rng, 1 << N)
    want = oracle.run_ops(psi.copy(), ops)
    circ = qs.Circuit(N, ops).compile(k, prec)
    kinds = [circ.pass_info(i)["kernel"] for i in range(circ.stats()["num_passes"])]
    assert kinds.count("tile") >= 1
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    circ.apply(q)
    generic = q.get_amps()
    assert amp_err(generic, want) < TOL[prec]
    circ.specialize()
    q.set_amps(psi)
    circ.apply(q)
    assert np.array_equal(q.get_amps(), generic)
