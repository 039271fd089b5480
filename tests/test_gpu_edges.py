"""Degenerate and extreme cases against the FP64 oracle: one-qubit
registers, the widest gates, a target with every other qubit as control,
empty Pauli sums and circuits, identity-only Pauli strings, a partial trace
that keeps one qubit."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner, scalar_tol

pytestmark = pytest.mark.gpu

PRECS = ["c128", "c64"]


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


@pytest.mark.parametrize("prec", PRECS)
def test_one_qubit_statevector(qs, prec):
    banner(f"one-qubit statevector {prec}")
    rng = np.random.default_rng(61)
    psi = synth.random_state(rng, 2)
    u = synth.haar_unitary(rng, 2)
    q = qs.Qureg(1, precision=prec).set_amps(psi)
    q.apply_unitary([], [0], u)
    q.apply_pauli_gadget([0], [2], 0.7)
    q.apply_pauli_tensor([0], [1])
    q.apply_phase_gadget([0], -0.3)
    want = oracle.apply_gate(psi.copy(), [], [0], u)
    want = oracle.apply_pauli_gadget(want, [0], [2], 0.7)
    want = oracle.apply_pauli_tensor(want, [0], [1])
    want = oracle.apply_phase_gadget(want, [0], -0.3)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    assert abs(q.prob_of_outcome(0, 1) - oracle.sv_prob_of_outcome(want, 0, 1)) < scalar_tol(prec)
    codes = np.array([[1], [2], [3], [0]], np.int32)
    coeffs = np.array([0.3, -1.1, 0.7, 0.25])
    e = q.expec_pauli_sum(codes, coeffs)
    assert abs(e.real - oracle.sv_expec_pauli_sum(want, codes, coeffs).real) < scalar_tol(prec, 2.4)


@pytest.mark.parametrize("prec", PRECS)
def test_one_qubit_density_matrix(qs, prec):
    banner(f"one-qubit density matrix {prec}")
    rng = np.random.default_rng(62)
    a = synth.random_matrix(rng, 2)
    rho = a @ a.conj().T
    rho = (rho / np.trace(rho)).reshape(-1, order="F")
    u = synth.haar_unitary(rng, 2)
    q = qs.Qureg(1, density=True, precision=prec).set_amps(rho)
    q.apply_unitary([], [0], u)
    q.apply_kraus_map([0], synth.kraus_damping_1q(0.3))
    q.apply_depolarising(0, 0.2)
    q.apply_pauli_gadget([0], [1], 0.4)
    want = oracle.dm_apply_gate(rho.copy(), [], [0], u)
    want = oracle.dm_apply_kraus(want, [0], synth.kraus_damping_1q(0.3))
    want = oracle.dm_apply_kraus(want, [0], synth.kraus_depolarising_1q(0.2))
    want = oracle.dm_apply_pauli_gadget(want, [0], [1], 0.4)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    assert abs(q.trace() - oracle.dm_trace(want)) < scalar_tol(prec)
    assert abs(q.purity() - oracle.dm_purity(want)) < scalar_tol(prec)


@pytest.mark.parametrize("prec", PRECS)
def test_widest_gate_with_four_controls(qs, prec):
    """Six targets and four controls on 11 qubits: one group per 2^10
    amplitudes, the vector kernel (complex128) and the matrix cores
    (complex64)."""
    banner(f"6 targets + 4 controls {prec}")
    rng = np.random.default_rng(63)
    N = 11
    psi = synth.random_state(rng, 1 << N)
    perm = [int(x) for x in rng.permutation(N)]
    t, c = perm[:6], perm[6:10]
    m = synth.haar_unitary(rng, 64)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    q.apply_unitary(c, t, m)
    assert amp_err(q.get_amps(), oracle.apply_gate(psi.copy(), c, t, m)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_every_other_qubit_a_control(qs, prec):
    banner(f"one target, N-1 controls {prec}")
    rng = np.random.default_rng(64)
    N = 10
    psi = synth.random_state(rng, 1 << N)
    u = synth.haar_unitary(rng, 2)
    for t in (0, 5, 9):
        c = [x for x in range(N) if x != t]
        q = qs.Qureg(N, precision=prec).set_amps(psi)
        q.apply_unitary(c, [t], u)
        assert amp_err(q.get_amps(), oracle.apply_gate(psi.copy(), c, [t], u)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_identity_strings_and_empty_sums(qs, prec):
    banner(f"identity strings, empty sums {prec}")
    rng = np.random.default_rng(65)
    N = 6
    psi = synth.random_state(rng, 1 << N)
    q = qs.Qureg(N, precision=prec).set_amps(psi)
    q.apply_pauli_gadget([1, 4], [0, 0], 0.9)          # e^{i 0.9} times the state
    assert amp_err(q.get_amps(), np.exp(0.9j) * psi) < TOL[prec]
    q.apply_pauli_tensor([2, 3], [0, 0])               # identity
    assert amp_err(q.get_amps(), np.exp(0.9j) * psi) < TOL[prec]
    e = q.expec_pauli_sum(np.zeros((0, N), np.int32), np.zeros(0))
    assert e == 0
    e = q.expec_pauli_sum(np.zeros((1, N), np.int32), np.array([2.5]))   # 2.5 * identity
    assert abs(e.real - 2.5 * np.vdot(psi, psi).real) < scalar_tol(prec, 2.5)
    rho = np.outer(psi, psi.conj()).reshape(-1, order="F")
    d = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
    d.apply_pauli_gadget([0, 5], [0, 0], 1.3)           # G rho G^dagger = rho
    assert amp_err(d.get_amps(), rho) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_partial_trace_keeping_one_qubit(qs, prec):
    banner(f"partial trace to one qubit {prec}")
    rng = np.random.default_rng(66)
    N = 6
    a = synth.random_matrix(rng, 1 << N)
    rho = a @ a.conj().T
    rho = (rho / np.trace(rho)).reshape(-1, order="F")
    for keep in (0, 3, 5):
        traced = [x for x in range(N) if x != keep]
        q = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
        red = q.partial_trace(traced)
        want = oracle.partial_trace(rho.copy(), traced)
        assert red.num_qubits == 1
        assert amp_err(red.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("k", [0, 4, 12])
def test_empty_circuit(qs, k):
    banner(f"empty circuit k={k}")
    rng = np.random.default_rng(67)
    N = 12
    psi = synth.random_state(rng, 1 << N)
    c = qs.Circuit(N, []).compile(k, "c64")
    assert c.stats()["num_passes"] == 0
    q = qs.Qureg(N, precision="c64").set_amps(psi)
    c.apply(q)
    assert amp_err(q.get_amps(), psi) < 1e-7
