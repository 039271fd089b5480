"""Host logic of libqsim exercised without a GPU, run by
tests/test_host_sanitizers.py in a subprocess against the sanitizer build of
the host code: argument validation, recording, fusion and tile planning
(qs_circuit_compile plans and packs every pass before it allocates device
memory, which fails without a GPU), batch recording with gadget
decompositions, parameter updates."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import synth  # noqa: E402
from paper_2311_01512_amd import native as N  # noqa: E402


def compile_or_alloc_error(c, k, prec):
    try:
        N.qs_circuit_compile(c, k, prec)
    except MemoryError:
        pass      # planned and packed; the device upload needs a GPU


def record(ops, n, density=False):
    c = (N.qs_circuit_create_density if density else N.qs_circuit_create)(n)
    for op in ops:
        if op["op"] == "unitary":
            N.qs_circuit_add_unitary(c, op["ctrls"], op["targs"], op["matrix"])
        elif op["op"] == "gadget":
            N.qs_circuit_add_pauli_gadget(c, op["targs"], op["paulis"], op["theta"])
        elif op["op"] == "kraus":
            N.qs_circuit_add_kraus_map(c, op["targs"], op["kraus"])
    return c


def main():
    ops = synth.config2_circuit(num_qubits=20, num_gates=200)
    c = record(ops, 20)
    for prec in (N.QS_C64, N.QS_C128):
        for k in (0, 2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13):
            if prec == N.QS_C128 and k > 12:
                continue
            compile_or_alloc_error(c, k, prec)
    N.qs_circuit_destroy(c)
    c5 = record(synth.config5_circuit(num_qubits=16, num_gates=60), 16)
    for k in (0, 6, 12):
        compile_or_alloc_error(c5, k, N.QS_C64)
    N.qs_circuit_destroy(c5)
    dops, _ = synth.config3_circuit(num_qubits=6, num_ops=80, num_traced=3)
    d = record(dops, 6, density=True)
    for k in (0, 4, 10, 12):
        compile_or_alloc_error(d, k, N.QS_C64)
    N.qs_circuit_destroy(d)
    # parametrised gadgets and their angles
    p = N.qs_circuit_create(8)
    for w in range(1, 9):
        N.qs_circuit_add_param_gadget(p, list(range(w)), [1 + (i % 3) for i in range(w)], w - 1, 0.5)
    N.qs_circuit_set_params(p, np.linspace(0, 1, 8))
    compile_or_alloc_error(p, 10, N.QS_C64)
    N.qs_circuit_destroy(p)
    # batch recording, gadgets of every weight decomposed
    b = N.qs_batch_create(N.QS_C64)
    for n in (3, 9, 14):
        ci = N.qs_batch_add_circuit(b, n, 2 * n)
        for w in range(1, n + 1):
            N.qs_batch_add_gadget(b, ci, list(range(n - w, n)), [1 + (i % 3) for i in range(w)], w % (2 * n), 0.7)
        N.qs_batch_add_gadget(b, ci, [0, n - 1], [2, 3], -1, 0.3)
        codes, coeffs = synth.random_pauli_sum(np.random.default_rng(n), n, 5)
        N.qs_batch_set_observable(b, ci, codes, coeffs, n)
    N.qs_batch_destroy(b)
    print("host logic ok", flush=True)


if __name__ == "__main__":
    main()
