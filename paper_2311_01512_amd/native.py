"""ctypes binding of libqsim.so: the C entry points under the same names,
argument marshalling only.  Importing this module raises if the HIP library
has not been built; there is no fallback implementation.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QS_LIB may name another build of the same library (the CPU tests load the
# sanitizer build of the host code this way)
LIB_PATH = os.environ.get("QS_LIB") or os.path.join(HERE, "libqsim.so")
HEADER = os.path.join(HERE, "..", "include", "qsim.h")

QS_C64, QS_C128 = 0, 1
QS_OK, QS_E_ARG, QS_E_PRECOND, QS_E_ALLOC, QS_E_HIP, QS_E_TYPE = 0, -1, -2, -3, -4, -5

_ERRS = {QS_E_ARG: ValueError, QS_E_PRECOND: ValueError, QS_E_ALLOC: MemoryError, QS_E_TYPE: TypeError}


class QsError(RuntimeError):
    pass


def _load():
    # PyTorch ships its own HIP runtime.  Loading torch first makes
    # libqsim.so bind to that same runtime (same soname), so device pointers
    # and streams from torch are valid here; otherwise two runtimes would
    # coexist in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2311_01512_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback path")
    return C.CDLL(LIB_PATH)


lib = _load()

_P, _I, _D, _U64 = C.c_void_p, C.c_int, C.c_double, C.c_uint64
_PP = C.POINTER(C.c_void_p)
_PD = C.POINTER(C.c_double)

_SIGS = {
    "qs_create_qureg": [_I, _I, _I, _P, _P, _PP],
    "qs_destroy_qureg": [_P],
    "qs_get_info": [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_uint64), _PP],
    "qs_set_stream": [_P, _P],
    "qs_sync": [_P],
    "qs_init_zero_state": [_P],
    "qs_init_basis_state": [_P, _U64],
    "qs_init_plus_state": [_P],
    "qs_init_pure_density": [_P, _P],
    "qs_init_hashed_state": [_P, _U64],
    "qs_set_amps": [_P, _U64, _P, _U64],
    "qs_get_amps": [_P, _U64, _P, _U64],
    "qs_apply_multi_ctrl_multi_targ_unitary": [_P, _P, _I, _P, _I, _P],
    "qs_apply_pauli_gadget": [_P, _P, _P, _I, _D],
    "qs_apply_swap": [_P, _I, _I],
    "qs_apply_multi_swap": [_P, _P, _P, _I],
    "qs_apply_pauli_tensor": [_P, _P, _P, _I],
    "qs_apply_phase_gadget": [_P, _P, _I, _D],
    "qs_apply_superop": [_P, _P, _I, _P],
    "qs_apply_kraus_map": [_P, _P, _I, _P, _I],
    "qs_calc_partial_trace": [_P, _P, _I, _P],
    "qs_calc_expec_pauli_sum": [_P, _P, _P, _I, _PD, _PD],
    "qs_calc_expec_pauli_sum_noalloc": [_P, _I, _I, _I, _P, _P, _P, _I, _PD, _PD],
    "qs_calc_prob_of_outcome": [_P, _I, _I, _PD],
    "qs_calc_total_prob": [_P, _PD],
    "qs_calc_trace": [_P, _PD, _PD],
    "qs_calc_purity": [_P, _PD, _PD],
    "qs_calc_inner_product": [_P, _P, _PD, _PD],
    "qs_apply_dephasing": [_P, _I, _D],
    "qs_apply_two_qubit_dephasing": [_P, _I, _I, _D],
    "qs_apply_depolarising": [_P, _I, _D],
    "qs_apply_two_qubit_depolarising": [_P, _I, _I, _D],
    "qs_apply_damping": [_P, _I, _D],
    "qs_circuit_create": [_I, _PP],
    "qs_circuit_create_density": [_I, _PP],
    "qs_circuit_add_superop": [_P, _P, _I, _P],
    "qs_circuit_add_kraus_map": [_P, _P, _I, _P, _I],
    "qs_circuit_destroy": [_P],
    "qs_circuit_add_unitary": [_P, _P, _I, _P, _I, _P],
    "qs_circuit_add_pauli_gadget": [_P, _P, _P, _I, _D],
    "qs_circuit_compile": [_P, _I, _I],
    "qs_circuit_specialize": [_P, C.POINTER(C.c_int)],
    "qs_circuit_stats": [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_uint64), C.POINTER(C.c_int)],
    "qs_apply_circuit": [_P, _P],
    "qs_apply_circuit_passes": [_P, _P, _I, _I],
    "qs_circuit_pass_info": [_P, _I, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "qs_circuit_autotune": [_P, _P, _P, _I, C.POINTER(C.c_int), _PD],
    "qs_circuit_autotune_ex": [_P, _P, _P, _I, _I, C.POINTER(C.c_int), C.POINTER(C.c_int), _PD, _PD],
    "qs_batch_create": [_I, _PP],
    "qs_batch_destroy": [_P],
    "qs_batch_add_circuit": [_P, _I, _I, C.POINTER(C.c_int)],
    "qs_batch_add_rotation": [_P, _I, _I, _I, _I, _D],
    "qs_batch_add_gate1": [_P, _I, _I, _P],
    "qs_batch_add_cz": [_P, _I, _I, _I],
    "qs_circuit_add_param_gadget": [_P, _P, _P, _I, _I, _D],
    "qs_circuit_set_params": [_P, _P, _I],
    "qs_circuit_adjoint_gradient": [_P, _P, _P, _P, _P, _I, _I, _PD, _P],
    "qs_batch_add_gadget": [_P, _I, _P, _P, _I, _I, _D],
    "qs_batch_set_observable": [_P, _I, _P, _P, _I],
    "qs_batch_compile": [_P, _P, _I],
    "qs_batch_run": [_P, _P, _P, _P],
    "qs_batch_get_state": [_P, _I, _P],
    "qs_batch_stats": [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
    "qs_batch_specialize": [_P, C.POINTER(C.c_int)],
}

for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
lib.qs_last_error.argtypes = []
lib.qs_last_error.restype = C.c_char_p


def check(rc, what=""):
    if rc != QS_OK:
        msg = lib.qs_last_error().decode(errors="replace")
        raise _ERRS.get(rc, QsError)(f"{what}: {msg} (status {rc})")
    return rc


def ints(xs):
    return np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))


def ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def cmatrix(m):
    """Complex matrix -> contiguous interleaved (re, im) float64 array."""
    m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    return m.view(np.float64)


# ---- thin wrappers with the C names ----------------------------------------

def qs_create_qureg(num_qubits, is_density, precision, device_ptr=None, hip_stream=None):
    out = C.c_void_p()
    check(lib.qs_create_qureg(num_qubits, int(bool(is_density)), precision, device_ptr, hip_stream,
                              C.byref(out)), "qs_create_qureg")
    return out


def qs_destroy_qureg(q):
    check(lib.qs_destroy_qureg(q), "qs_destroy_qureg")


def qs_set_stream(q, hip_stream):
    check(lib.qs_set_stream(q, hip_stream), "qs_set_stream")


def qs_sync(q):
    check(lib.qs_sync(q), "qs_sync")


def qs_init_zero_state(q):
    check(lib.qs_init_zero_state(q), "qs_init_zero_state")


def qs_init_basis_state(q, index):
    check(lib.qs_init_basis_state(q, index), "qs_init_basis_state")


def qs_init_plus_state(q):
    check(lib.qs_init_plus_state(q), "qs_init_plus_state")


def qs_init_pure_density(rho, psi):
    check(lib.qs_init_pure_density(rho, psi), "qs_init_pure_density")


def qs_init_hashed_state(q, seed):
    check(lib.qs_init_hashed_state(q, seed), "qs_init_hashed_state")


def qs_set_amps(q, start, amps):
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128))
    check(lib.qs_set_amps(q, start, ptr(a), a.size), "qs_set_amps")


def qs_get_amps(q, start, count):
    a = np.empty(count, dtype=np.complex128)
    check(lib.qs_get_amps(q, start, ptr(a), count), "qs_get_amps")
    return a


def _square(m, dim, what):
    if np.shape(m) != (dim, dim):
        raise ValueError(f"{what} must be {dim} x {dim}, got shape {np.shape(m)}")


def qs_apply_multi_ctrl_multi_targ_unitary(q, ctrls, targs, matrix):
    c, t = ints(ctrls), ints(targs)
    _square(matrix, 1 << t.size, "matrix")
    m = cmatrix(matrix)
    check(lib.qs_apply_multi_ctrl_multi_targ_unitary(q, ptr(c), c.size, ptr(t), t.size, ptr(m)),
          "qs_apply_multi_ctrl_multi_targ_unitary")


def qs_apply_pauli_gadget(q, targs, paulis, theta):
    t, p = ints(targs), ints(paulis)
    if t.size != p.size:
        raise ValueError("targs and paulis differ in length")
    check(lib.qs_apply_pauli_gadget(q, ptr(t), ptr(p), t.size, float(theta)), "qs_apply_pauli_gadget")


def qs_apply_swap(q, qubit1, qubit2):
    check(lib.qs_apply_swap(q, int(qubit1), int(qubit2)), "qs_apply_swap")


def qs_apply_multi_swap(q, qubits1, qubits2):
    a, b = ints(qubits1), ints(qubits2)
    if a.size != b.size:
        raise ValueError("qubits1 and qubits2 differ in length")
    check(lib.qs_apply_multi_swap(q, ptr(a), ptr(b), a.size), "qs_apply_multi_swap")


def qs_apply_pauli_tensor(q, targs, paulis):
    t, p = ints(targs), ints(paulis)
    if t.size != p.size:
        raise ValueError("targs and paulis differ in length")
    check(lib.qs_apply_pauli_tensor(q, ptr(t), ptr(p), t.size), "qs_apply_pauli_tensor")


def qs_apply_phase_gadget(q, targs, theta):
    t = ints(targs)
    check(lib.qs_apply_phase_gadget(q, ptr(t), t.size, float(theta)), "qs_apply_phase_gadget")


def qs_apply_superop(q, targs, superop):
    t = ints(targs)
    _square(superop, 1 << (2 * t.size), "superoperator")
    s = cmatrix(superop)
    check(lib.qs_apply_superop(q, ptr(t), t.size, ptr(s)), "qs_apply_superop")


def qs_apply_kraus_map(q, targs, kraus):
    t = ints(targs)
    k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128))
    if k.ndim != 3 or k.shape[1:] != (1 << t.size, 1 << t.size):
        raise ValueError(f"Kraus operators must have shape (M, {1 << t.size}, {1 << t.size})")
    check(lib.qs_apply_kraus_map(q, ptr(t), t.size, ptr(k.view(np.float64)), k.shape[0]), "qs_apply_kraus_map")


def qs_apply_dephasing(q, target, p):
    check(lib.qs_apply_dephasing(q, int(target), float(p)), "qs_apply_dephasing")


def qs_apply_two_qubit_dephasing(q, target1, target2, p):
    check(lib.qs_apply_two_qubit_dephasing(q, int(target1), int(target2), float(p)), "qs_apply_two_qubit_dephasing")


def qs_apply_depolarising(q, target, p):
    check(lib.qs_apply_depolarising(q, int(target), float(p)), "qs_apply_depolarising")


def qs_apply_two_qubit_depolarising(q, target1, target2, p):
    check(lib.qs_apply_two_qubit_depolarising(q, int(target1), int(target2), float(p)),
          "qs_apply_two_qubit_depolarising")


def qs_apply_damping(q, target, p):
    check(lib.qs_apply_damping(q, int(target), float(p)), "qs_apply_damping")


def qs_calc_partial_trace(q_in, targs, q_out):
    t = ints(targs)
    check(lib.qs_calc_partial_trace(q_in, ptr(t), t.size, q_out), "qs_calc_partial_trace")


def qs_get_info(q):
    n, d, p, na, ptr_ = C.c_int(), C.c_int(), C.c_int(), C.c_uint64(), C.c_void_p()
    check(lib.qs_get_info(q, C.byref(n), C.byref(d), C.byref(p), C.byref(na), C.byref(ptr_)), "qs_get_info")
    return {"num_qubits": n.value, "is_density": d.value, "precision": p.value, "num_amps": na.value,
            "device_ptr": ptr_.value}


def qs_calc_expec_pauli_sum(q, paulis, coeffs):
    p = np.ascontiguousarray(np.asarray(paulis, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    if p.size != c.size * qs_get_info(q)["num_qubits"]:
        raise ValueError("need num_terms * num_qubits Pauli codes")
    re, im = C.c_double(), C.c_double()
    check(lib.qs_calc_expec_pauli_sum(q, ptr(p), ptr(c), c.size, C.byref(re), C.byref(im)),
          "qs_calc_expec_pauli_sum")
    return complex(re.value, im.value)


def qs_calc_expec_pauli_sum_noalloc(amps_ptr, num_qubits, is_density, precision, stream, paulis, coeffs):
    p = np.ascontiguousarray(np.asarray(paulis, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    if p.size != c.size * num_qubits:
        raise ValueError("need num_terms * num_qubits Pauli codes")
    re, im = C.c_double(), C.c_double()
    check(lib.qs_calc_expec_pauli_sum_noalloc(amps_ptr, num_qubits, int(is_density), precision, stream, ptr(p),
                                              ptr(c), c.size, C.byref(re), C.byref(im)),
          "qs_calc_expec_pauli_sum_noalloc")
    return complex(re.value, im.value)


def qs_calc_prob_of_outcome(q, qubit, outcome):
    out = C.c_double()
    check(lib.qs_calc_prob_of_outcome(q, qubit, outcome, C.byref(out)), "qs_calc_prob_of_outcome")
    return out.value


def qs_calc_total_prob(q):
    out = C.c_double()
    check(lib.qs_calc_total_prob(q, C.byref(out)), "qs_calc_total_prob")
    return out.value


def qs_calc_trace(q):
    re, im = C.c_double(), C.c_double()
    check(lib.qs_calc_trace(q, C.byref(re), C.byref(im)), "qs_calc_trace")
    return complex(re.value, im.value)


def qs_calc_purity(q):
    re, im = C.c_double(), C.c_double()
    check(lib.qs_calc_purity(q, C.byref(re), C.byref(im)), "qs_calc_purity")
    return complex(re.value, im.value)


def qs_calc_inner_product(a, b):
    re, im = C.c_double(), C.c_double()
    check(lib.qs_calc_inner_product(a, b, C.byref(re), C.byref(im)), "qs_calc_inner_product")
    return complex(re.value, im.value)


# ---- circuits ------------------------------------------------------------------

def qs_circuit_create(num_qubits):
    out = C.c_void_p()
    check(lib.qs_circuit_create(num_qubits, C.byref(out)), "qs_circuit_create")
    return out


def qs_circuit_create_density(num_qubits):
    out = C.c_void_p()
    check(lib.qs_circuit_create_density(num_qubits, C.byref(out)), "qs_circuit_create_density")
    return out


def qs_circuit_add_superop(c, targs, superop):
    t = ints(targs)
    _square(superop, 1 << (2 * t.size), "superoperator")
    s = cmatrix(superop)
    check(lib.qs_circuit_add_superop(c, ptr(t), t.size, ptr(s)), "qs_circuit_add_superop")


def qs_circuit_add_kraus_map(c, targs, kraus):
    t = ints(targs)
    k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128))
    if k.ndim != 3 or k.shape[1:] != (1 << t.size, 1 << t.size):
        raise ValueError(f"Kraus operators must have shape (M, {1 << t.size}, {1 << t.size})")
    check(lib.qs_circuit_add_kraus_map(c, ptr(t), t.size, ptr(k.view(np.float64)), k.shape[0]),
          "qs_circuit_add_kraus_map")


def qs_circuit_destroy(c):
    check(lib.qs_circuit_destroy(c), "qs_circuit_destroy")


def qs_circuit_add_unitary(c, ctrls, targs, matrix):
    cc, t = ints(ctrls), ints(targs)
    _square(matrix, 1 << t.size, "matrix")
    m = cmatrix(matrix)
    check(lib.qs_circuit_add_unitary(c, ptr(cc), cc.size, ptr(t), t.size, ptr(m)), "qs_circuit_add_unitary")


def qs_circuit_add_pauli_gadget(c, targs, paulis, theta):
    t, p = ints(targs), ints(paulis)
    if t.size != p.size:
        raise ValueError("targs and paulis differ in length")
    check(lib.qs_circuit_add_pauli_gadget(c, ptr(t), ptr(p), t.size, float(theta)), "qs_circuit_add_pauli_gadget")


def qs_circuit_compile(c, fuse_k, precision):
    check(lib.qs_circuit_compile(c, fuse_k, precision), "qs_circuit_compile")


def qs_circuit_specialize(c):
    n = C.c_int()
    check(lib.qs_circuit_specialize(c, C.byref(n)), "qs_circuit_specialize")
    return n.value


def qs_circuit_stats(c):
    no, npass, lu = C.c_int(), C.c_int(), C.c_uint64()
    widths = (C.c_int * 7)()
    check(lib.qs_circuit_stats(c, C.byref(no), C.byref(npass), C.byref(lu), widths), "qs_circuit_stats")
    return {"num_ops": no.value, "num_passes": npass.value, "logical_updates": lu.value,
            "passes_by_width": list(widths)}


def qs_apply_circuit(q, c):
    check(lib.qs_apply_circuit(q, c), "qs_apply_circuit")


def qs_apply_circuit_passes(q, c, first, count):
    check(lib.qs_apply_circuit_passes(q, c, first, count), "qs_apply_circuit_passes")


PASS_KERNELS = {0: "gadget_pairs", 1: "gadget_diag", 2: "dense_vector", 3: "dense_mfma", 4: "tile"}


def qs_circuit_pass_info(c, index):
    k, nt, nc, m, ph = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
    check(lib.qs_circuit_pass_info(c, index, C.byref(k), C.byref(nt), C.byref(nc), C.byref(m), C.byref(ph)),
          "qs_circuit_pass_info")
    return {"kernel": PASS_KERNELS[k.value], "num_targs": nt.value, "num_ctrls": nc.value, "members": m.value,
            "phases": ph.value}


def qs_circuit_autotune(q, c, candidates):
    cand = ints(candidates)
    best = C.c_int()
    ms = np.zeros(cand.size, dtype=np.float64)
    check(lib.qs_circuit_autotune(q, c, ptr(cand), cand.size, C.byref(best),
                                  ms.ctypes.data_as(_PD)), "qs_circuit_autotune")
    return best.value, ms


def qs_circuit_autotune_ex(q, c, candidates, try_specialized):
    cand = ints(candidates)
    best, spec = C.c_int(), C.c_int()
    ms = np.zeros(cand.size, dtype=np.float64)
    ms_spec = np.zeros(cand.size, dtype=np.float64)
    check(lib.qs_circuit_autotune_ex(q, c, ptr(cand), cand.size, int(bool(try_specialized)), C.byref(best),
                                     C.byref(spec), ms.ctypes.data_as(_PD), ms_spec.ctypes.data_as(_PD)),
          "qs_circuit_autotune_ex")
    return best.value, bool(spec.value), ms, ms_spec


# ---- batches -------------------------------------------------------------------

def qs_batch_create(precision):
    out = C.c_void_p()
    check(lib.qs_batch_create(precision, C.byref(out)), "qs_batch_create")
    return out


def qs_batch_destroy(b):
    check(lib.qs_batch_destroy(b), "qs_batch_destroy")


def qs_batch_add_circuit(b, num_qubits, num_params):
    idx = C.c_int()
    check(lib.qs_batch_add_circuit(b, num_qubits, num_params, C.byref(idx)), "qs_batch_add_circuit")
    return idx.value


def qs_batch_add_rotation(b, circuit, qubit, pauli, param, scale):
    check(lib.qs_batch_add_rotation(b, circuit, qubit, pauli, param, float(scale)), "qs_batch_add_rotation")


def qs_batch_add_gate1(b, circuit, qubit, matrix):
    _square(matrix, 2, "matrix")
    m = cmatrix(matrix)
    check(lib.qs_batch_add_gate1(b, circuit, qubit, ptr(m)), "qs_batch_add_gate1")


def qs_batch_add_gadget(b, circuit, targs, paulis, param, scale):
    t, p = ints(targs), ints(paulis)
    if t.size != p.size:
        raise ValueError("one Pauli code per target")
    check(lib.qs_batch_add_gadget(b, circuit, ptr(t), ptr(p), t.size, param, scale), "qs_batch_add_gadget")


def qs_circuit_add_param_gadget(c, targs, paulis, param, scale):
    t, p = ints(targs), ints(paulis)
    if t.size != p.size:
        raise ValueError("one Pauli code per target")
    check(lib.qs_circuit_add_param_gadget(c, ptr(t), ptr(p), t.size, param, scale), "qs_circuit_add_param_gadget")


def qs_circuit_set_params(c, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    check(lib.qs_circuit_set_params(c, ptr(p), p.size), "qs_circuit_set_params")


def qs_circuit_adjoint_gradient(c, psi, lam, paulis, coeffs, num_qubits, num_params):
    p = np.ascontiguousarray(np.asarray(paulis, dtype=np.int32))
    h = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    if p.size != h.size * num_qubits:
        raise ValueError("need num_terms * num_qubits Pauli codes")
    e = C.c_double()
    g = np.zeros(num_params, dtype=np.float64)
    check(lib.qs_circuit_adjoint_gradient(c, psi, lam, ptr(p), ptr(h), h.size, num_params, C.byref(e), ptr(g)),
          "qs_circuit_adjoint_gradient")
    return e.value, g


def qs_batch_add_cz(b, circuit, q1, q2):
    check(lib.qs_batch_add_cz(b, circuit, q1, q2), "qs_batch_add_cz")


def qs_batch_set_observable(b, circuit, paulis, coeffs, num_qubits):
    p = np.ascontiguousarray(np.asarray(paulis, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    if p.size != c.size * num_qubits:
        raise ValueError("need num_terms * num_qubits Pauli codes")
    check(lib.qs_batch_set_observable(b, circuit, ptr(p), ptr(c), c.size), "qs_batch_set_observable")


def qs_batch_compile(b, hip_stream=None, use_graph=True):
    check(lib.qs_batch_compile(b, hip_stream, int(bool(use_graph))), "qs_batch_compile")


def qs_batch_run(b, params, num_circuits, num_params, grads=True):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if p.size != num_params:
        raise ValueError(f"expected {num_params} parameters, got {p.size}")
    e = np.zeros(num_circuits, dtype=np.float64)
    g = np.zeros(max(1, num_params), dtype=np.float64) if grads else None
    check(lib.qs_batch_run(b, ptr(p), ptr(e), ptr(g)), "qs_batch_run")
    return (e, g[:num_params]) if grads else (e, None)


def qs_batch_get_state(b, circuit, num_qubits):
    a = np.empty(1 << num_qubits, dtype=np.complex128)
    check(lib.qs_batch_get_state(b, circuit, ptr(a)), "qs_batch_get_state")
    return a


def qs_batch_specialize(b):
    n = C.c_int(0)
    check(lib.qs_batch_specialize(b, C.byref(n)), "qs_batch_specialize")
    return n.value


def qs_batch_stats(b):
    nc, ns, ta, lu = C.c_int(), C.c_int(), C.c_uint64(), C.c_uint64()
    check(lib.qs_batch_stats(b, C.byref(nc), C.byref(ns), C.byref(ta), C.byref(lu)), "qs_batch_stats")
    return {"num_circuits": nc.value, "num_steps": ns.value, "total_amps": ta.value, "logical_updates": lu.value}
