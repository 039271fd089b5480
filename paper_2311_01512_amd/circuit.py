"""Circuit: a recorded list of statevector operators, compiled once (plain
per-gate passes, or dense k-qubit blocks) and applied through the C ABI."""
from . import native as N


class Circuit:
    def __init__(self, num_qubits, ops=()):
        self.num_qubits = int(num_qubits)
        self._c = N.qs_circuit_create(self.num_qubits)
        self.compiled_for = None
        for op in ops:
            self.add(op)

    def add(self, op):
        """Append an op dict ({"op": "unitary"|"gadget", ...})."""
        if op["op"] == "unitary":
            N.qs_circuit_add_unitary(self._c, op["ctrls"], op["targs"], op["matrix"])
        elif op["op"] == "gadget":
            N.qs_circuit_add_pauli_gadget(self._c, op["targs"], op["paulis"], op["theta"])
        else:
            raise ValueError(f"circuits hold statevector operators, not {op['op']}")
        self.compiled_for = None
        return self

    def compile(self, fuse_k=0, precision="c64"):
        N.qs_circuit_compile(self._c, int(fuse_k), N.QS_C64 if precision == "c64" else N.QS_C128)
        self.compiled_for = (int(fuse_k), precision)
        return self

    def stats(self):
        return N.qs_circuit_stats(self._c)

    def apply(self, qureg):
        N.qs_apply_circuit(qureg.handle, self._c)
        return qureg

    def apply_passes(self, qureg, first, count):
        N.qs_apply_circuit_passes(qureg.handle, self._c, first, count)
        return qureg

    def pass_info(self, index):
        return N.qs_circuit_pass_info(self._c, index)

    def autotune(self, qureg, candidates=(0, 3, 4, 5, 6)):
        """Times one application per fusion width on `qureg` (overwriting its
        state) and leaves the circuit compiled with the fastest; returns
        (best_k, {k: ms})."""
        best, ms = N.qs_circuit_autotune(qureg.handle, self._c, candidates)
        self.compiled_for = (best, qureg.precision)
        return best, dict(zip(candidates, ms.tolist()))

    def close(self):
        if getattr(self, "_c", None) is not None:
            N.qs_circuit_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
