"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only draws random inputs (circuits, matrices, Pauli sums) and
holds none of the simulation arithmetic: no gate application, superoperator
construction, reduction or trace lives here.
"""
from .circuits import (  # noqa: F401
    PAULI_I, PAULI_X, PAULI_Y, PAULI_Z,
    haar_unitary, haar_isometry, random_matrix, random_state,
    pauli_matrix_2x2, rotation_y, rotation_z,
    kraus_depolarising_1q, kraus_damping_1q, kraus_dephasing_1q,
    kraus_depolarising_2q, kraus_dephasing_2q, kraus_random_isometry,
    random_pauli_sum,
    config1_circuit, config2_circuit, config3_circuit, config4_batch,
    config5_circuit, op_qubits, count_logical_updates,
    CONFIG_SEEDS,
)
