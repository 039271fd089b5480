"""Batch: many parametrised circuits of uneven size evaluated together on
the GPU (energies <psi(theta)|H|psi(theta)> and adjoint gradients), driven
through the qs_batch_* C entry points, and `energies`, the same as a
differentiable torch function of the parameters."""
import numpy as np
import torch

from . import native as N


class Batch:
    def __init__(self, precision="c64"):
        self.precision = precision
        self._b = N.qs_batch_create(N.QS_C64 if precision == "c64" else N.QS_C128)
        self.num_qubits = []
        self.num_params = []
        self.compiled = False

    def add_circuit(self, num_qubits, ops, num_params, codes=None, coeffs=None):
        """ops: op dicts; supported are Pauli gadgets carrying a parameter
        ({"op": "gadget", "targs": (...), "paulis": (...), "param": k,
        "scale": s}: exp(i s theta_k P), any weight), fixed Pauli gadgets
        ({"op": "gadget", ..., "theta": t} without "param"), fixed
        single-qubit unitaries, and CZ (a Z unitary with one control)."""
        c = N.qs_batch_add_circuit(self._b, num_qubits, num_params)
        for op in ops:
            if op["op"] == "gadget" and "param" in op and len(op["targs"]) == 1 and op["paulis"][0] != 0:
                N.qs_batch_add_rotation(self._b, c, op["targs"][0], op["paulis"][0], op["param"],
                                        op.get("scale", 1.0))
            elif op["op"] == "gadget" and "param" in op:
                N.qs_batch_add_gadget(self._b, c, op["targs"], op["paulis"], op["param"], op.get("scale", 1.0))
            elif op["op"] == "gadget":
                N.qs_batch_add_gadget(self._b, c, op["targs"], op["paulis"], -1, op["theta"])
            elif op["op"] == "unitary" and not op["ctrls"] and len(op["targs"]) == 1:
                N.qs_batch_add_gate1(self._b, c, op["targs"][0], op["matrix"])
            elif (op["op"] == "unitary" and len(op["ctrls"]) == 1 and len(op["targs"]) == 1
                  and np.allclose(op["matrix"], np.diag([1, -1]))):
                N.qs_batch_add_cz(self._b, c, op["ctrls"][0], op["targs"][0])
            else:
                raise ValueError("batches hold Pauli gadgets (parametrised or fixed), single-qubit gates and CZ")
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

    def specialize(self):
        """Run-time specialised step kernels (qs_batch_specialize); returns
        the number of distinct step programs."""
        if not self.compiled:
            raise RuntimeError("compile the batch first")
        return N.qs_batch_specialize(self._b)

    def run(self, params, grads=True):
        """params: concatenated parameter vectors.  Returns (energies, grads)."""
        return N.qs_batch_run(self._b, params, len(self.num_qubits), sum(self.num_params), grads)

    def param_owner(self):
        """Circuit index of every parameter of the concatenated vector."""
        return np.repeat(np.arange(len(self.num_params)), self.num_params)

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


class BatchEnergy(torch.autograd.Function):
    """Energies E_c(theta) of every circuit of a compiled Batch as a function
    of the concatenated parameter vector.  The forward pass runs the batch
    with the adjoint sweep (one GPU run gives the energies and every dE_c /
    dtheta_p) and keeps the gradients; the backward pass returns
    grad_E[c(p)] * dE_c(p) / dtheta_p, c(p) being the circuit that owns
    parameter p (each parameter belongs to exactly one circuit)."""

    @staticmethod
    def forward(ctx, params, batch):
        if not batch.compiled:
            raise RuntimeError("compile the batch first")
        p = params.detach().to(device="cpu", dtype=torch.float64).contiguous().numpy()
        e, g = batch.run(p, grads=True)
        ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(g)))
        ctx.owner = torch.from_numpy(batch.param_owner())
        ctx.device, ctx.dtype = params.device, params.dtype
        return torch.from_numpy(np.ascontiguousarray(e)).to(device=params.device)

    @staticmethod
    def backward(ctx, grad_e):
        (g,) = ctx.saved_tensors
        w = grad_e.detach().to(device="cpu", dtype=torch.float64)[ctx.owner]
        return (w * g).to(device=ctx.device, dtype=ctx.dtype), None


def energies(batch, params):
    """Differentiable energies of a compiled Batch (see BatchEnergy)."""
    return BatchEnergy.apply(params, batch)
