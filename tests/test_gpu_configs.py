"""Whole-workload parity with the oracle: the 12-qubit circuit at full size,
and the 28-qubit, 14-qubit density-matrix and 34-qubit workloads on the same
generators at sizes the oracle finishes in seconds."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner, scalar_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def test_config1_full(qs):
    """12-qubit complex128 circuit of 200 gates from |0..0>: amplitudes,
    norm, all 2^12 Z-basis outcome probabilities and per-qubit P(0)."""
    banner("config1 N=12 c128")
    N = 12
    ops = synth.config1_circuit()
    q = qs.Qureg(N, precision="c128").init_zero().run_ops(ops)
    want = oracle.run_ops(oracle.zero_state(N), ops)
    got = q.get_amps()
    assert amp_err(got, want) < TOL["c128"]
    assert abs(q.total_prob() - oracle.sv_total_prob(want)) < 1e-12
    assert np.abs(np.abs(got) ** 2 - np.abs(want) ** 2).max() < 1e-12
    for k in range(N):
        assert abs(q.prob_of_outcome(k, 0) - oracle.sv_prob_of_outcome(want, k, 0)) < 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_config2_reduced(qs, prec):
    """The 28-qubit generator (Haar 1q, controlled Haar 2q, Pauli gadgets) at
    16 qubits, 500 gates, plain per-gate path."""
    banner(f"config2 N=16 {prec}")
    N = 16
    ops = synth.config2_circuit(num_qubits=N)
    rng = np.random.default_rng(2)
    psi = synth.random_state(rng, 1 << N)
    q = qs.Qureg(N, precision=prec).set_amps(psi).run_ops(ops)
    want = oracle.run_ops(psi.copy(), ops)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    assert abs(q.total_prob() - 1) < scalar_tol(prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_config3_reduced(qs, prec):
    """The 14-qubit density-matrix generator at 6 qubits: 300 ops of Haar
    unitaries, depolarising, damping and random Kraus maps from |0><0|, then
    the partial trace over 3 qubits, trace and purity."""
    banner(f"config3 N=6 {prec}")
    N = 6
    ops, traced = synth.config3_circuit(num_qubits=N, num_traced=3)
    q = qs.Qureg(N, density=True, precision=prec).init_zero().run_ops(ops)
    want = oracle.run_ops(oracle.zero_state(N, density=True), ops, density=True)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    red = q.partial_trace(traced)
    want_red = oracle.partial_trace(want, traced)
    assert amp_err(red.get_amps(), want_red) < TOL[prec]
    for st, ref in ((q, want), (red, want_red)):
        assert abs(st.trace() - oracle.dm_trace(ref)) < scalar_tol(prec)
        assert abs(st.purity() - oracle.dm_purity(ref)) < scalar_tol(prec)


def test_config5_reduced(qs):
    """The 34-qubit generator (5-target Haar with up to 4 controls, Pauli
    gadgets) at 14 qubits in complex64: amplitudes, <Z_0 Z_13> and norm."""
    banner("config5 N=14 c64")
    N = 14
    ops = synth.config5_circuit(num_qubits=N)
    rng = np.random.default_rng(5)
    psi = synth.random_state(rng, 1 << N)
    q = qs.Qureg(N, precision="c64").set_amps(psi).run_ops(ops)
    want = oracle.run_ops(psi.copy(), ops)
    assert amp_err(q.get_amps(), want) < TOL["c64"]
    zz = np.zeros((1, N), np.int32)
    zz[0, 0] = zz[0, N - 1] = 3
    assert abs(q.expec_pauli_sum(zz, [1.0]) - oracle.sv_expec_pauli_sum(want, zz, [1.0])) < 1e-5
    assert abs(q.total_prob() - oracle.sv_total_prob(want)) < 1e-5
