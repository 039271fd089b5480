"""Batch: many parametrised circuits of uneven size evaluated together on
the GPU (energies <psi(theta)|H|psi(theta)> and adjoint gradients), driven
through the qs_batch_* C entry points."""
import numpy as np

from . import native as N


class Batch:
    def __init__(self, precision="c64"):
        self.precision = precision
        self._b = N.qs_batch_create(N.QS_C64 if precision == "c64" else N.QS_C128)
        self.num_qubits = []
        self.num_params = []
        self.compiled = False

    def add_circuit(self, num_qubits, ops, num_params, codes=None, coeffs=None):
        """ops: op dicts; supported are single-qubit gadgets carrying a
        parameter ({"op": "gadget", "targs": (q,), "paulis": (p,), "param": k,
        "scale": s}: exp(i s theta_k P)), fixed single-qubit unitaries, and
        CZ (a Z unitary with one control)."""
        c = N.qs_batch_add_circuit(self._b, num_qubits, num_params)
        for op in ops:
            if op["op"] == "gadget" and "param" in op and len(op["targs"]) == 1:
                N.qs_batch_add_rotation(self._b, c, op["targs"][0], op["paulis"][0], op["param"],
                                        op.get("scale", 1.0))
            elif op["op"] == "unitary" and not op["ctrls"] and len(op["targs"]) == 1:
                N.qs_batch_add_gate1(self._b, c, op["targs"][0], op["matrix"])
            elif (op["op"] == "unitary" and len(op["ctrls"]) == 1 and len(op["targs"]) == 1
                  and np.allclose(op["matrix"], np.diag([1, -1]))):
                N.qs_batch_add_cz(self._b, c, op["ctrls"][0], op["targs"][0])
            else:
                raise ValueError("batches hold parametrised single-qubit rotations, single-qubit gates and CZ")
        if codes is not None:
            N.qs_batch_set_observable(self._b, c, codes, coeffs, num_qubits)
        self.num_qubits.append(num_qubits)
        self.num_params.append(num_params)
        self.compiled = False
        return c

    def compile(self, stream=None, use_graph=True):
        N.qs_batch_compile(self._b, None if stream is None else stream.cuda_stream, use_graph)
        self.compiled = True
        return self

    def run(self, params, grads=True):
        """params: concatenated parameter vectors.  Returns (energies, grads)."""
        return N.qs_batch_run(self._b, params, len(self.num_qubits), sum(self.num_params), grads)

    def state(self, circuit):
        return N.qs_batch_get_state(self._b, circuit, self.num_qubits[circuit])

    def stats(self):
        return N.qs_batch_stats(self._b)

    def close(self):
        if getattr(self, "_b", None) is not None:
            N.qs_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
