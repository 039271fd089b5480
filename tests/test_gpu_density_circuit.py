"""Density circuits (operators recorded on the Choi vector and compiled like
statevector circuits: plain, dense blocks, tile steps) against the FP64
oracle's density-matrix routines."""
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


def _mixed_ops(rng, N, count):
    """Controlled unitaries, gadgets with X/Y/Z, explicit superoperators and
    1- and 2-qubit Kraus maps on an N-qubit density matrix."""
    ops = []
    for g in range(count):
        kind = g % 6
        if kind == 0:
            q = rng.permutation(N)[:3]
            ops.append({"op": "unitary", "ctrls": (int(q[2]),), "targs": (int(q[0]), int(q[1])),
                        "matrix": synth.haar_unitary(rng, 4)})
        elif kind == 1:
            ops.append({"op": "unitary", "ctrls": (), "targs": (int(rng.integers(0, N)),),
                        "matrix": synth.haar_unitary(rng, 2)})
        elif kind == 2:
            w = int(rng.integers(1, N + 1))
            t = rng.permutation(N)[:w]
            ops.append({"op": "gadget", "targs": tuple(int(x) for x in t),
                        "paulis": tuple(int(x) for x in rng.integers(1, 4, size=w)), "theta": rng.uniform(-3, 3)})
        elif kind == 3:
            t = int(rng.integers(0, N))
            ks = synth.kraus_damping_1q(rng.uniform(0, 0.2))
            ops.append({"op": "superop", "targs": (t,), "matrix": oracle.build_superop(ks)})
        elif kind == 4:
            ops.append({"op": "kraus", "targs": (int(rng.integers(0, N)),),
                        "kraus": synth.kraus_depolarising_1q(rng.uniform(0, 0.1))})
        else:
            q = rng.permutation(N)[:2]
            ops.append({"op": "kraus", "targs": (int(q[0]), int(q[1])),
                        "kraus": synth.kraus_random_isometry(rng, 2, 4)})
    return ops


def _oracle_run(rho, ops):
    for op in ops:
        if op["op"] == "superop":
            oracle.dm_apply_superop(rho, op["targs"], op["matrix"])
        else:
            oracle.run_ops(rho, [op], density=True)
    return rho


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("k", [0, 2, 4, 6, 8, 10, 11, 13])
def test_density_circuit_config3_ops(qs, prec, k):
    """The 14-qubit density-matrix generator at 7 qubits (a 14-bit Choi
    vector), compiled at every kind of pass, from a random mixed state."""
    banner(f"density circuit config3 N=7 k={k} {prec}")
    N = 7
    ops, _ = synth.config3_circuit(num_qubits=N, num_ops=120)
    rng = np.random.default_rng(40 + k)
    psi = synth.random_state(rng, 1 << N)
    rho0 = np.outer(psi, psi.conj()).reshape(-1, order="F")   # Choi vector: k + l 2^N
    circ = qs.Circuit(N, ops, density=True).compile(k, prec)
    st = circ.stats()
    assert st["logical_updates"] == synth.count_logical_updates(ops, N, density=True)
    q = qs.Qureg(N, density=True, precision=prec).set_amps(rho0)
    circ.apply(q)
    want = oracle.run_ops(rho0.copy(), ops, density=True)
    assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("k", [0, 3, 8, 12])
def test_density_circuit_mixed_ops(qs, k):
    banner(f"density circuit mixed N=6 k={k}")
    N = 6
    rng = np.random.default_rng(900 + k)
    ops = _mixed_ops(rng, N, 90)
    psi = synth.random_state(rng, 1 << N)
    rho0 = np.outer(psi, psi.conj()).reshape(-1, order="F")
    circ = qs.Circuit(N, ops, density=True).compile(k, "c128")
    q = qs.Qureg(N, density=True, precision="c128").set_amps(rho0)
    circ.apply(q)
    want = _oracle_run(rho0.copy(), ops)
    assert amp_err(q.get_amps(), want) < TOL["c128"]
    assert abs(q.trace() - oracle.dm_trace(want)) < 1e-12


def test_density_circuit_errors(qs):
    c = qs.Circuit(3)
    with pytest.raises(ValueError):
        c.add({"op": "kraus", "targs": (0,), "kraus": np.eye(2)[None]})
    d = qs.Circuit(3, density=True)
    d.add({"op": "unitary", "ctrls": (), "targs": (0,), "matrix": np.eye(2)}).compile(0, "c128")
    with pytest.raises(ValueError):
        d.apply(qs.Qureg(3, precision="c128").init_zero())        # statevector
    with pytest.raises(ValueError):
        d.apply(qs.Qureg(4, density=True, precision="c128").init_zero())   # other size
