"""Circuit: a recorded list of operators on a statevector or a density
matrix, compiled once (plain per-gate passes, dense k-qubit blocks, or tile
steps) and applied through the C ABI."""
from . import native as N


class Circuit:
    def __init__(self, num_qubits, ops=(), density=False):
        self.num_qubits = int(num_qubits)
        self.density = bool(density)
        self._c = (N.qs_circuit_create_density if self.density else N.qs_circuit_create)(self.num_qubits)
        self.compiled_for = None
        self.specialized = 0
        for op in ops:
            self.add(op)

    def add(self, op):
        """Append an op dict ({"op": "unitary"|"gadget", ...}; density
        circuits also take "kraus" and "superop")."""
        kind = op["op"]
        if kind == "unitary":
            N.qs_circuit_add_unitary(self._c, op.get("ctrls", ()), op["targs"], op["matrix"])
        elif kind == "gadget":
            N.qs_circuit_add_pauli_gadget(self._c, op["targs"], op["paulis"], op["theta"])
        elif kind in ("kraus", "superop") and not self.density:
            raise ValueError(f"{kind} operators belong to density circuits")
        elif kind == "kraus":
            N.qs_circuit_add_kraus_map(self._c, op["targs"], op["kraus"])
        elif kind == "superop":
            N.qs_circuit_add_superop(self._c, op["targs"], op["matrix"])
        else:
            raise ValueError(f"unknown op {kind}")
        self.compiled_for = None
        self.specialized = 0
        return self

    def compile(self, fuse_k=0, precision="c64"):
        N.qs_circuit_compile(self._c, int(fuse_k), N.QS_C64 if precision == "c64" else N.QS_C128)
        self.compiled_for = (int(fuse_k), precision)
        self.specialized = 0
        return self

    def specialize(self):
        """Compiles every tile step of the compiled circuit into a kernel of
        its own at run time (the ROCm clang, run as child processes); returns
        the number of such kernels.
        Recompiling the circuit drops them."""
        self.specialized = N.qs_circuit_specialize(self._c)
        return self.specialized

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

    def autotune(self, qureg, candidates=(0, 3, 4, 5, 6), specialize=False):
        """Times one application per fusion width on `qureg` (overwriting its
        state) and leaves the circuit compiled with the fastest; returns
        (best_k, {k: ms}).  With specialize=True, widths that give tile steps
        are also timed with the steps specialised, the circuit is left in the
        fastest form (`self.specialized` > 0 when that is specialised) and
        the return value is (best_k, {k: ms}, {k: specialised ms})."""
        if not specialize:
            best, ms = N.qs_circuit_autotune(qureg.handle, self._c, candidates)
            self.compiled_for = (best, qureg.precision)
            self.specialized = 0
            return best, dict(zip(candidates, ms.tolist()))
        best, spec, ms, ms_spec = N.qs_circuit_autotune_ex(qureg.handle, self._c, candidates, True)
        self.compiled_for = (best, qureg.precision)
        self.specialized = 0
        if spec:
            self.specialized = sum(1 for i in range(self.stats()["num_passes"])
                                   if self.pass_info(i)["kernel"] == "tile")
        return best, dict(zip(candidates, ms.tolist())), {k: v for k, v in zip(candidates, ms_spec.tolist()) if v >= 0}

    def close(self):
        if getattr(self, "_c", None) is not None:
            N.qs_circuit_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
