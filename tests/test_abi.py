"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects malformed arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(qs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2311_01512_amd import native
    return native.lib


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qs_create_qureg", "qs_apply_multi_ctrl_multi_targ_unitary", "qs_apply_pauli_gadget",
                     "qs_apply_superop", "qs_apply_kraus_map", "qs_calc_partial_trace",
                     "qs_calc_expec_pauli_sum", "qs_calc_prob_of_outcome"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_argument_checks(lib):
    """Validation that happens before any HIP call."""
    out = C.c_void_p()
    lib.qs_create_qureg.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
    assert lib.qs_create_qureg(4, 0, 7, None, None, C.byref(out)) == -1        # bad precision
    assert b"precision" in lib.qs_last_error()
    assert lib.qs_create_qureg(0, 0, 1, None, None, C.byref(out)) == -1        # no qubits
    assert lib.qs_create_qureg(4, 0, 1, None, None, None) == -1                # null output
    assert lib.qs_create_qureg(21, 1, 1, None, None, C.byref(out)) == -3       # 2^42 amplitudes
    lib.qs_apply_pauli_gadget.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double]
    assert lib.qs_apply_pauli_gadget(None, None, None, 1, 0.1) == -1           # null qureg
    lib.qs_apply_swap.argtypes = [C.c_void_p, C.c_int, C.c_int]
    assert lib.qs_apply_swap(None, 0, 1) == -1                                 # null qureg
    lib.qs_apply_pauli_tensor.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
    assert lib.qs_apply_pauli_tensor(None, None, None, 1) == -1
    lib.qs_apply_phase_gadget.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double]
    assert lib.qs_apply_phase_gadget(None, None, 1, 0.1) == -1
    assert lib.qs_destroy_qureg(None) == 0


def test_binding_rejects_bad_shapes():
    from paper_2311_01512_amd import native as N
    import numpy as np
    with pytest.raises(ValueError):
        N.qs_apply_multi_ctrl_multi_targ_unitary(None, [], [0, 1], np.eye(2))
    with pytest.raises(ValueError):
        N.qs_apply_kraus_map(None, [0], np.eye(4)[None])
    with pytest.raises(ValueError):
        N.qs_apply_superop(None, [0], np.eye(2))
    with pytest.raises(ValueError):
        N.qs_apply_pauli_gadget(None, [0, 1], [1], 0.2)
    with pytest.raises(ValueError):
        N.qs_apply_pauli_tensor(None, [0, 1], [1])
    with pytest.raises(ValueError):
        N.qs_apply_multi_swap(None, [0, 1], [2])


def test_circuit_recording_checks(lib):
    """Circuit creation and recording are host-only: kinds, sizes, qubits."""
    from paper_2311_01512_amd import native as N
    import numpy as np
    with pytest.raises(ValueError):
        N.qs_circuit_create_density(21)                      # 2^42 Choi amplitudes
    c = N.qs_circuit_create(3)
    try:
        with pytest.raises(ValueError, match="density"):
            N.qs_circuit_add_kraus_map(c, [0], np.eye(2)[None])
        with pytest.raises(ValueError, match="density"):
            N.qs_circuit_add_superop(c, [0], np.eye(4))
    finally:
        N.qs_circuit_destroy(c)
    d = N.qs_circuit_create_density(3)
    try:
        N.qs_circuit_add_unitary(d, [1], [0], np.eye(2))
        N.qs_circuit_add_pauli_gadget(d, [0, 2], [2, 3], 0.3)
        N.qs_circuit_add_kraus_map(d, [2], np.eye(2)[None])
        with pytest.raises(ValueError):
            N.qs_circuit_add_superop(d, [3], np.eye(4))      # qubit 3 of 3
        n_ops = C.c_int()
        lib.qs_circuit_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p, C.c_void_p]
        assert lib.qs_circuit_stats(d, C.byref(n_ops), None, None, None) == 0
        assert n_ops.value == 5        # unitary and gadget twice (rows, columns), the map once
    finally:
        N.qs_circuit_destroy(d)
