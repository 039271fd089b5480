"""Run by tests/test_oracle_checks.py in a subprocess with the write-counting
oracle build (ORACLE_VARIANT=count): each routine's amplitude writes against
the counts the paper states for its algorithm.  Prints one line per check
and exits non-zero on the first mismatch."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
import synth  # noqa: E402


def check(label, fn, want):
    oracle.reset_writes()
    fn()
    got = oracle.writes()
    print(f"{label}: {got} writes, expected {want}", flush=True)
    if got != want:
        sys.exit(f"write count mismatch for {label}: {got} != {want}")


def main():
    assert oracle.counts_writes(), "the write-counting build was not loaded"
    rng = np.random.default_rng(3)
    for N in (5, 7):
        psi = synth.random_state(rng, 1 << N)
        u2, u4, u8 = synth.haar_unitary(rng, 2), synth.haar_unitary(rng, 4), synth.haar_unitary(rng, 8)
        # one-target gate: 2^N writes (Sec. one-target gate)
        check(f"N={N} one-target gate", lambda: oracle.apply_gate(psi, (), (2,), u2), 1 << N)
        # s controls: 2^(N-s) writes (Sec. many-control gate; the loop range reading)
        for s in (1, 2, 3):
            check(f"N={N} {s}-control one-target gate",
                  lambda: oracle.apply_gate(psi, tuple(range(1, 1 + s)), (0,), u2), 1 << (N - s))
        # n-target gate: every amplitude once (Sec. many-target gate)
        check(f"N={N} two-target gate", lambda: oracle.apply_gate(psi, (), (3, 0), u4), 1 << N)
        check(f"N={N} three-target gate, one control",
              lambda: oracle.apply_gate(psi, (4,), (0, 2, 1), u8), 1 << (N - 1))
        # SWAP: half the amplitudes (Table alg_summary_table: Lambda / 2)
        check(f"N={N} SWAP", lambda: oracle.apply_swap(psi, 1, 4), 1 << (N - 1))
        # Pauli tensor, phase gadget, Pauli gadget: Lambda writes
        check(f"N={N} Pauli tensor", lambda: oracle.apply_pauli_tensor(psi, (0, 2, 3), (1, 2, 3)), 1 << N)
        check(f"N={N} phase gadget", lambda: oracle.apply_phase_gadget(psi, (1, 3), 0.4), 1 << N)
        check(f"N={N} Pauli gadget", lambda: oracle.apply_pauli_gadget(psi, (0, 4), (2, 1), 0.7), 1 << N)
        check(f"N={N} Z-only Pauli gadget", lambda: oracle.apply_pauli_gadget(psi, (0, 4), (3, 3), 0.7), 1 << N)
        # expectation values, probabilities: no writes
        codes, coeffs = synth.random_pauli_sum(rng, N, 4)
        check(f"N={N} Pauli-sum expectation", lambda: oracle.sv_expec_pauli_sum(psi, codes, coeffs), 0)
        check(f"N={N} outcome probability", lambda: oracle.sv_prob_of_outcome(psi, 2, 1), 0)
    for N in (3, 4):
        rho = synth.random_state(rng, 1 << (2 * N))
        lam = 1 << (2 * N)
        u2, u4 = synth.haar_unitary(rng, 2), synth.haar_unitary(rng, 4)
        # density-matrix unitary: the statevector algorithm twice on 2N qubits
        check(f"N={N} DM unitary", lambda: oracle.dm_apply_gate(rho, (), (1, 0), u4), 2 * lam)
        check(f"N={N} DM controlled unitary", lambda: oracle.dm_apply_gate(rho, (2,), (0,), u2), 2 * (lam >> 1))
        # specific unitaries (Table alg_summary_table): SWAP Lambda, Pauli
        # tensor, phase and Pauli gadgets 2 Lambda
        check(f"N={N} DM SWAP", lambda: oracle.dm_apply_swap(rho, 0, 2), lam)
        check(f"N={N} DM Pauli tensor", lambda: oracle.dm_apply_pauli_tensor(rho, (0, 1), (2, 3)), 2 * lam)
        check(f"N={N} DM phase gadget", lambda: oracle.dm_apply_phase_gadget(rho, (0, 2), 0.3), 2 * lam)
        check(f"N={N} DM Pauli gadget", lambda: oracle.dm_apply_pauli_gadget(rho, (1, 2), (1, 2), 0.3), 2 * lam)
        # Kraus map: the superoperator as a 2n-target gate, every entry once
        check(f"N={N} Kraus map", lambda: oracle.dm_apply_kraus(rho, (0, 2), synth.kraus_random_isometry(rng, 2, 4)),
              lam)
        # expectation: no writes (Sec. Pauli string expectation value)
        codes, coeffs = synth.random_pauli_sum(rng, N, 3)
        check(f"N={N} DM Pauli-sum expectation", lambda: oracle.dm_expec_pauli_sum(rho, codes, coeffs), 0)
        # partial trace: one write per entry of the reduced matrix
        check(f"N={N} partial trace of 2", lambda: oracle.partial_trace(rho, (0, 2)), 1 << (2 * (N - 2)))
    print("write counts ok", flush=True)


if __name__ == "__main__":
    main()
