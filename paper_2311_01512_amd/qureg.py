"""Qureg: a statevector or density matrix in HBM, owned by a torch tensor and
ordered on a torch stream, driven through the C ABI of libqsim.so."""
import numpy as np
import torch

from . import native as N


class Qureg:
    """N-qubit statevector (2^N amplitudes) or density matrix (Choi vector of
    2^(2N) amplitudes) in complex64 ("c64") or complex128 ("c128")."""

    def __init__(self, num_qubits, density=False, precision="c128", device="cuda", stream=None):
        if precision not in ("c64", "c128"):
            raise ValueError("precision is 'c64' or 'c128'")
        self.num_qubits = int(num_qubits)
        self.density = bool(density)
        self.precision = precision
        bits = 2 * self.num_qubits if self.density else self.num_qubits
        self.num_amps = 1 << bits
        dtype = torch.complex64 if precision == "c64" else torch.complex128
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.tensor = torch.empty(self.num_amps, dtype=dtype, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._q = N.qs_create_qureg(self.num_qubits, self.density,
                                        N.QS_C64 if precision == "c64" else N.QS_C128,
                                        self.tensor.data_ptr(), self.stream.cuda_stream)

    # ---- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_q", None) is not None:
            N.qs_destroy_qureg(self._q)
            self._q = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._q

    def sync(self):
        N.qs_sync(self._q)

    # ---- states -----------------------------------------------------------------
    def init_zero(self):
        N.qs_init_zero_state(self._q)
        return self

    def init_basis(self, index):
        N.qs_init_basis_state(self._q, index)
        return self

    def init_plus(self):
        N.qs_init_plus_state(self._q)
        return self

    def init_hashed(self, seed):
        N.qs_init_hashed_state(self._q, seed)
        return self

    def init_pure(self, psi):
        N.qs_init_pure_density(self._q, psi.handle)
        return self

    def set_amps(self, amps, start=0):
        N.qs_set_amps(self._q, start, amps)
        return self

    def get_amps(self, start=0, count=None):
        if count is None:
            count = self.num_amps - start
        return N.qs_get_amps(self._q, start, count)

    # ---- operators ----------------------------------------------------------------
    def apply_unitary(self, ctrls, targs, matrix):
        N.qs_apply_multi_ctrl_multi_targ_unitary(self._q, ctrls, targs, matrix)
        return self

    def apply_pauli_gadget(self, targs, paulis, theta):
        N.qs_apply_pauli_gadget(self._q, targs, paulis, theta)
        return self

    def apply_swap(self, qubit1, qubit2):
        N.qs_apply_swap(self._q, qubit1, qubit2)
        return self

    def apply_multi_swap(self, qubits1, qubits2):
        N.qs_apply_multi_swap(self._q, qubits1, qubits2)
        return self

    def apply_pauli_tensor(self, targs, paulis):
        N.qs_apply_pauli_tensor(self._q, targs, paulis)
        return self

    def apply_phase_gadget(self, targs, theta):
        N.qs_apply_phase_gadget(self._q, targs, theta)
        return self

    def apply_superop(self, targs, superop):
        N.qs_apply_superop(self._q, targs, superop)
        return self

    def apply_kraus_map(self, targs, kraus):
        N.qs_apply_kraus_map(self._q, targs, kraus)
        return self

    def run_ops(self, ops):
        """Apply op dicts ({"op": "unitary"|"gadget"|"kraus"|"swap"|"pauli_tensor"|
        "phase_gadget", ...}) in order."""
        for op in ops:
            kind = op["op"]
            if kind == "unitary":
                N.qs_apply_multi_ctrl_multi_targ_unitary(self._q, op["ctrls"], op["targs"], op["matrix"])
            elif kind == "gadget":
                N.qs_apply_pauli_gadget(self._q, op["targs"], op["paulis"], op["theta"])
            elif kind == "kraus":
                N.qs_apply_kraus_map(self._q, op["targs"], op["kraus"])
            elif kind == "swap":
                N.qs_apply_swap(self._q, op["targs"][0], op["targs"][1])
            elif kind == "pauli_tensor":
                N.qs_apply_pauli_tensor(self._q, op["targs"], op["paulis"])
            elif kind == "phase_gadget":
                N.qs_apply_phase_gadget(self._q, op["targs"], op["theta"])
            else:
                raise ValueError(f"unknown op {kind}")
        return self

    def apply_dephasing(self, target, p):
        N.qs_apply_dephasing(self._q, target, p)
        return self

    def apply_two_qubit_dephasing(self, target1, target2, p):
        N.qs_apply_two_qubit_dephasing(self._q, target1, target2, p)
        return self

    def apply_depolarising(self, target, p):
        N.qs_apply_depolarising(self._q, target, p)
        return self

    def apply_two_qubit_depolarising(self, target1, target2, p):
        N.qs_apply_two_qubit_depolarising(self._q, target1, target2, p)
        return self

    def apply_damping(self, target, p):
        N.qs_apply_damping(self._q, target, p)
        return self

    # ---- calculations -----------------------------------------------------------------
    def partial_trace(self, targs, out=None):
        targs = list(targs)
        if out is None:
            out = Qureg(self.num_qubits - len(targs), density=True, precision=self.precision,
                        device=self.device, stream=self.stream)
        N.qs_calc_partial_trace(self._q, targs, out.handle)
        return out

    def expec_pauli_sum(self, codes, coeffs):
        codes = np.asarray(codes, dtype=np.int32).reshape(-1, self.num_qubits)
        return N.qs_calc_expec_pauli_sum(self._q, codes, coeffs)

    def prob_of_outcome(self, qubit, outcome):
        return N.qs_calc_prob_of_outcome(self._q, qubit, outcome)

    def total_prob(self):
        return N.qs_calc_total_prob(self._q)

    def trace(self):
        return N.qs_calc_trace(self._q)

    def purity(self):
        return N.qs_calc_purity(self._q)

    def inner_product(self, other):
        return N.qs_calc_inner_product(self._q, other.handle)
