"""ctypes front end of the C oracle (test infrastructure only).

All arrays are NumPy complex128 (statevector: 2^N entries; density matrix:
Choi vector of 2^(2N) entries, entry k + l*2^N = rho[k][l]).  Functions that
update a state do so in place and also return it.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """The compiled oracle; the environment variable ORACLE_VARIANT selects
    the write-counting ("count") or sanitizer ("asan") build for the CPU
    tests that run it in a subprocess."""
    global _lib
    if _lib is None:
        variant = os.environ.get("ORACLE_VARIANT", "plain")
        path = _build.lib_path(variant)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(variant=variant)
        L = C.CDLL(path)
        P = C.c_void_p
        i = C.c_int
        d = C.c_double
        u64 = C.c_uint64
        pd = C.POINTER(C.c_double)
        sig = {
            "oracle_apply_gate": [P, i, P, i, P, i, P],
            "oracle_apply_pauli_gadget": [P, i, P, P, i, d],
            "oracle_dm_apply_gate": [P, i, P, i, P, i, P],
            "oracle_dm_apply_pauli_gadget": [P, i, P, P, i, d],
            "oracle_apply_swap": [P, i, i, i],
            "oracle_dm_apply_swap": [P, i, i, i],
            "oracle_apply_pauli_tensor": [P, i, P, P, i],
            "oracle_dm_apply_pauli_tensor": [P, i, P, P, i],
            "oracle_apply_phase_gadget": [P, i, P, i, d],
            "oracle_dm_apply_phase_gadget": [P, i, P, i, d],
            "oracle_build_superop": [P, i, i, P],
            "oracle_dm_apply_superop": [P, i, P, i, P],
            "oracle_dm_apply_kraus": [P, i, P, i, P, i],
            "oracle_partial_trace": [P, i, P, i, P],
            "oracle_dm_expec_pauli_sum": [P, i, P, P, i, pd, pd],
            "oracle_sv_expec_pauli_sum": [P, i, P, P, i, pd, pd],
            "oracle_sv_prob_of_outcome": [P, i, i, i, pd],
            "oracle_dm_prob_of_outcome": [P, i, i, i, pd],
            "oracle_sv_total_prob": [P, i, pd],
            "oracle_dm_trace": [P, i, pd, pd],
            "oracle_dm_purity": [P, i, pd, pd],
            "oracle_init_basis": [P, i, u64],
            "oracle_init_plus": [P, i, i],
            "oracle_init_pure_dm": [P, P, i],
            "oracle_hashed_amps": [i, u64, u64, u64, P],
            "oracle_hashed_amps_at": [i, u64, P, u64, P],
            "oracle_splitmix64_at": [u64, u64],
            "oracle_num_threads": [],
            "oracle_counts_writes": [],
            "oracle_reset_writes": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.oracle_splitmix64_at.restype = u64
        L.oracle_writes.argtypes = []
        L.oracle_writes.restype = u64
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _ints(xs):
    return np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))


def _cplx(a):
    a = np.asarray(a)
    if a.dtype != np.complex128 or not a.flags.c_contiguous:
        raise TypeError("oracle expects a C-contiguous complex128 array")
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments")


def _num_qubits(a, density):
    n = int(a.size).bit_length() - 1
    if (1 << n) != a.size:
        raise ValueError("state length is not a power of two")
    if density:
        if n % 2:
            raise ValueError("Choi vector length must be 4^N")
        return n // 2
    return n


# ---- statevector ----------------------------------------------------------

def apply_gate(psi, ctrls, targs, matrix):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128))
    c, t = _ints(ctrls), _ints(targs)
    if m.shape != (1 << len(t), 1 << len(t)):
        raise ValueError("matrix shape does not match targets")
    _check(lib().oracle_apply_gate(_ptr(psi), N, _ptr(c), len(c), _ptr(t), len(t), _ptr(m)), "apply_gate")
    return psi


def apply_pauli_gadget(psi, targs, paulis, theta):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    t, p = _ints(targs), _ints(paulis)
    _check(lib().oracle_apply_pauli_gadget(_ptr(psi), N, _ptr(t), _ptr(p), len(t), float(theta)),
           "apply_pauli_gadget")
    return psi


def apply_swap(psi, t1, t2):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    _check(lib().oracle_apply_swap(_ptr(psi), N, int(t1), int(t2)), "apply_swap")
    return psi


def apply_pauli_tensor(psi, targs, paulis):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    t, p = _ints(targs), _ints(paulis)
    if len(t) != len(p):
        raise ValueError("one Pauli code per target")
    _check(lib().oracle_apply_pauli_tensor(_ptr(psi), N, _ptr(t), _ptr(p), len(t)), "apply_pauli_tensor")
    return psi


def apply_phase_gadget(psi, targs, theta):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    t = _ints(targs)
    _check(lib().oracle_apply_phase_gadget(_ptr(psi), N, _ptr(t), len(t), float(theta)), "apply_phase_gadget")
    return psi


def sv_expec_pauli_sum(psi, codes, coeffs):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    codes = np.ascontiguousarray(np.asarray(codes, dtype=np.int32).reshape(-1, N))
    coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    re, im = C.c_double(), C.c_double()
    _check(lib().oracle_sv_expec_pauli_sum(_ptr(psi), N, _ptr(codes), _ptr(coeffs), len(coeffs),
                                           C.byref(re), C.byref(im)), "sv_expec_pauli_sum")
    return complex(re.value, im.value)


def sv_prob_of_outcome(psi, qubit, outcome):
    psi = _cplx(psi)
    out = C.c_double()
    _check(lib().oracle_sv_prob_of_outcome(_ptr(psi), _num_qubits(psi, False), qubit, outcome,
                                           C.byref(out)), "sv_prob_of_outcome")
    return out.value


def sv_total_prob(psi):
    psi = _cplx(psi)
    out = C.c_double()
    _check(lib().oracle_sv_total_prob(_ptr(psi), _num_qubits(psi, False), C.byref(out)), "sv_total_prob")
    return out.value


# ---- density matrix --------------------------------------------------------

def dm_apply_gate(rho, ctrls, targs, matrix):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128))
    c, t = _ints(ctrls), _ints(targs)
    _check(lib().oracle_dm_apply_gate(_ptr(rho), N, _ptr(c), len(c), _ptr(t), len(t), _ptr(m)),
           "dm_apply_gate")
    return rho


def dm_apply_pauli_gadget(rho, targs, paulis, theta):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t, p = _ints(targs), _ints(paulis)
    _check(lib().oracle_dm_apply_pauli_gadget(_ptr(rho), N, _ptr(t), _ptr(p), len(t), float(theta)),
           "dm_apply_pauli_gadget")
    return rho


def dm_apply_swap(rho, t1, t2):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    _check(lib().oracle_dm_apply_swap(_ptr(rho), N, int(t1), int(t2)), "dm_apply_swap")
    return rho


def dm_apply_pauli_tensor(rho, targs, paulis):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t, p = _ints(targs), _ints(paulis)
    if len(t) != len(p):
        raise ValueError("one Pauli code per target")
    _check(lib().oracle_dm_apply_pauli_tensor(_ptr(rho), N, _ptr(t), _ptr(p), len(t)), "dm_apply_pauli_tensor")
    return rho


def dm_apply_phase_gadget(rho, targs, theta):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t = _ints(targs)
    _check(lib().oracle_dm_apply_phase_gadget(_ptr(rho), N, _ptr(t), len(t), float(theta)),
           "dm_apply_phase_gadget")
    return rho


def build_superop(kraus):
    k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128))
    M, d, _ = k.shape
    n = d.bit_length() - 1
    S = np.zeros((d * d, d * d), dtype=np.complex128)
    _check(lib().oracle_build_superop(_ptr(k), M, n, _ptr(S)), "build_superop")
    return S


def dm_apply_superop(rho, targs, superop):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t = _ints(targs)
    S = np.ascontiguousarray(np.asarray(superop, dtype=np.complex128))
    if S.shape != (1 << (2 * len(t)), 1 << (2 * len(t))):
        raise ValueError("superoperator shape does not match targets")
    _check(lib().oracle_dm_apply_superop(_ptr(rho), N, _ptr(t), len(t), _ptr(S)), "dm_apply_superop")
    return rho


def dm_apply_kraus(rho, targs, kraus):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t = _ints(targs)
    k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128))
    _check(lib().oracle_dm_apply_kraus(_ptr(rho), N, _ptr(t), len(t), _ptr(k), k.shape[0]), "dm_apply_kraus")
    return rho


def partial_trace(rho, targs):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    t = _ints(targs)
    out = np.zeros(1 << (2 * (N - len(t))), dtype=np.complex128)
    _check(lib().oracle_partial_trace(_ptr(rho), N, _ptr(t), len(t), _ptr(out)), "partial_trace")
    return out


def dm_expec_pauli_sum(rho, codes, coeffs):
    rho = _cplx(rho)
    N = _num_qubits(rho, True)
    codes = np.ascontiguousarray(np.asarray(codes, dtype=np.int32).reshape(-1, N))
    coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    re, im = C.c_double(), C.c_double()
    _check(lib().oracle_dm_expec_pauli_sum(_ptr(rho), N, _ptr(codes), _ptr(coeffs), len(coeffs),
                                           C.byref(re), C.byref(im)), "dm_expec_pauli_sum")
    return complex(re.value, im.value)


def dm_prob_of_outcome(rho, qubit, outcome):
    rho = _cplx(rho)
    out = C.c_double()
    _check(lib().oracle_dm_prob_of_outcome(_ptr(rho), _num_qubits(rho, True), qubit, outcome,
                                           C.byref(out)), "dm_prob_of_outcome")
    return out.value


def dm_trace(rho):
    rho = _cplx(rho)
    re, im = C.c_double(), C.c_double()
    _check(lib().oracle_dm_trace(_ptr(rho), _num_qubits(rho, True), C.byref(re), C.byref(im)), "dm_trace")
    return complex(re.value, im.value)


def dm_purity(rho):
    rho = _cplx(rho)
    re, im = C.c_double(), C.c_double()
    _check(lib().oracle_dm_purity(_ptr(rho), _num_qubits(rho, True), C.byref(re), C.byref(im)), "dm_purity")
    return complex(re.value, im.value)


# ---- states ----------------------------------------------------------------

def zero_state(N, density=False):
    a = np.empty(1 << (2 * N if density else N), dtype=np.complex128)
    _check(lib().oracle_init_basis(_ptr(a), 2 * N if density else N, 0), "init_basis")
    return a


def basis_state(N, index, density=False):
    """SV: |index>; DM: |index><index|, Choi entry index*(2^N+1)."""
    a = np.empty(1 << (2 * N if density else N), dtype=np.complex128)
    i = index * ((1 << N) + 1) if density else index
    _check(lib().oracle_init_basis(_ptr(a), 2 * N if density else N, i), "init_basis")
    return a


def plus_state(N, density=False):
    a = np.empty(1 << (2 * N if density else N), dtype=np.complex128)
    _check(lib().oracle_init_plus(_ptr(a), N, int(density)), "init_plus")
    return a


def pure_dm(psi):
    psi = _cplx(psi)
    N = _num_qubits(psi, False)
    rho = np.empty(1 << (2 * N), dtype=np.complex128)
    _check(lib().oracle_init_pure_dm(_ptr(rho), _ptr(psi), N), "init_pure_dm")
    return rho


def hashed_state(num_index_bits, seed, start=0, count=None):
    if count is None:
        count = (1 << num_index_bits) - start
    out = np.empty(count, dtype=np.complex128)
    _check(lib().oracle_hashed_amps(num_index_bits, seed, start, count, _ptr(out)), "hashed_amps")
    return out


def hashed_amps_at(num_index_bits, seed, indices):
    idx = np.ascontiguousarray(np.asarray(indices, dtype=np.uint64))
    out = np.empty(idx.size, dtype=np.complex128)
    _check(lib().oracle_hashed_amps_at(num_index_bits, seed, _ptr(idx), idx.size, _ptr(out)), "hashed_amps_at")
    return out


def splitmix64_at(seed, counter):
    return int(lib().oracle_splitmix64_at(seed, counter))


def num_threads():
    return int(lib().oracle_num_threads())


def counts_writes():
    return bool(lib().oracle_counts_writes())


def writes():
    """Amplitude writes since reset_writes() (write-counting build only)."""
    return int(lib().oracle_writes())


def reset_writes():
    lib().oracle_reset_writes()


# ---- circuits (drive the routines above op by op) ---------------------------

def run_ops(state, ops, density=False):
    """Apply a list of synth-style op dicts in order."""
    for op in ops:
        kind = op["op"]
        if kind == "unitary":
            (dm_apply_gate if density else apply_gate)(state, op["ctrls"], op["targs"], op["matrix"])
        elif kind == "gadget":
            (dm_apply_pauli_gadget if density else apply_pauli_gadget)(state, op["targs"], op["paulis"],
                                                                       op["theta"])
        elif kind == "swap":
            (dm_apply_swap if density else apply_swap)(state, op["targs"][0], op["targs"][1])
        elif kind == "pauli_tensor":
            (dm_apply_pauli_tensor if density else apply_pauli_tensor)(state, op["targs"], op["paulis"])
        elif kind == "phase_gadget":
            (dm_apply_phase_gadget if density else apply_phase_gadget)(state, op["targs"], op["theta"])
        elif kind == "kraus":
            if not density:
                raise ValueError("Kraus map needs a density matrix")
            dm_apply_kraus(state, op["targs"], op["kraus"])
        else:
            raise ValueError(kind)
    return state


def param_shift_gradient(num_qubits, ops, codes, coeffs, num_params):
    """dE/dparameter for every parameter of a circuit whose parametrised ops
    are single-Pauli gadgets exp(i*theta*P) with theta = scale * parameter.
    Uses the exact two-term rule for exp(i*theta*P): dE/dtheta =
    E(theta + pi/4) - E(theta - pi/4), times scale.  Each evaluation is a
    fresh oracle run from |0..0>."""
    def energy(shift_op, delta):
        psi = zero_state(num_qubits)
        for k, op in enumerate(ops):
            if k == shift_op:
                op = dict(op)
                op["theta"] = op["theta"] + delta
            run_ops(psi, [op])
        return sv_expec_pauli_sum(psi, codes, coeffs).real

    grad = np.zeros(num_params)
    for k, op in enumerate(ops):
        if op["op"] == "gadget" and "param" in op:
            g = energy(k, np.pi / 4) - energy(k, -np.pi / 4)
            grad[op["param"]] += op.get("scale", 1.0) * g
    return grad
