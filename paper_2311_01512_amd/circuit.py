"""Circuit: a recorded list of operators on a statevector or a density
matrix, compiled once (plain per-gate passes, dense k-qubit blocks, or tile
steps) and applied through the C ABI."""
import numpy as np

from . import native as N


class Circuit:
    def __init__(self, num_qubits, ops=(), density=False):
        self.num_qubits = int(num_qubits)
        self.density = bool(density)
        self._c = (N.qs_circuit_create_density if self.density else N.qs_circuit_create)(self.num_qubits)
        self.compiled_for = None
        self.specialized = 0
        self.num_params = 0
        for op in ops:
            self.add(op)
        # parametrised gadgets that also carry their angle start at it
        start = {}
        for op in ops:
            if op.get("op") == "gadget" and "param" in op and "theta" in op and op.get("scale", 1.0) != 0:
                start.setdefault(op["param"], op["theta"] / op.get("scale", 1.0))
        if self.num_params and len(start) == self.num_params:
            self.set_params([start[k] for k in range(self.num_params)])

    def add(self, op):
        """Append an op dict ({"op": "unitary"|"gadget", ...}; density
        circuits also take "kraus" and "superop")."""
        kind = op["op"]
        if kind == "unitary":
            N.qs_circuit_add_unitary(self._c, op.get("ctrls", ()), op["targs"], op["matrix"])
        elif kind == "gadget" and "param" in op:
            # exp(i scale params[param] P); its angle comes from set_params
            N.qs_circuit_add_param_gadget(self._c, op["targs"], op["paulis"], op["param"], op.get("scale", 1.0))
            self.num_params = max(self.num_params, op["param"] + 1)
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

    def set_params(self, params):
        """Angles of the parametrised gadgets: scale * params[param].  The
        circuit must be compiled again before apply()."""
        N.qs_circuit_set_params(self._c, params)
        self.compiled_for = None
        self.specialized = 0
        return self

    def adjoint_gradient(self, psi, lam, codes, coeffs, num_params=None):
        """(E, dE/dparams) for E = <psi|H|psi> after the circuit, H the Pauli
        sum (codes, coeffs); psi holds the initial state (and holds it again
        on return), lam is a statevector qureg of the same shape overwritten
        as workspace.  The adjoint sweep runs in the library's kernels."""
        n = self.num_params if num_params is None else num_params
        codes = np.asarray(codes, dtype=np.int32).reshape(-1, self.num_qubits)
        return N.qs_circuit_adjoint_gradient(self._c, psi.handle, lam.handle, codes, coeffs, self.num_qubits, n)

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


class CircuitEnergy:
    """E(params) = <psi(params)|H|psi(params)> of a statevector Circuit with
    parametrised Pauli gadgets, as a torch.autograd.Function: the forward
    pass runs the library's adjoint sweep (energy and every dE/dparams in one
    call) and keeps the gradient; the backward pass scales it by the incoming
    gradient."""

    @staticmethod
    def _fn():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, params, circuit, initial, codes, coeffs):
                from .qureg import Qureg
                p = params.detach().to(device="cpu", dtype=torch.float64).contiguous().numpy()
                circuit.set_params(p)
                psi = Qureg(circuit.num_qubits, precision=initial.precision, device=initial.device,
                            stream=initial.stream)
                lam = Qureg(circuit.num_qubits, precision=initial.precision, device=initial.device,
                            stream=initial.stream)
                with torch.cuda.stream(initial.stream):
                    psi.tensor.copy_(initial.tensor)
                e, g = circuit.adjoint_gradient(psi, lam, codes, coeffs, num_params=p.size)
                ctx.save_for_backward(torch.from_numpy(g))
                ctx.device, ctx.dtype = params.device, params.dtype
                return torch.tensor(e, dtype=params.dtype, device=params.device)

            @staticmethod
            def backward(ctx, grad_e):
                (g,) = ctx.saved_tensors
                scale = grad_e.detach().to(device="cpu", dtype=torch.float64)
                return (scale * g).to(device=ctx.device, dtype=ctx.dtype), None, None, None, None

        return _F

    @classmethod
    def apply(cls, params, circuit, initial, codes, coeffs):
        return cls._fn().apply(params, circuit, initial, codes, coeffs)


def circuit_energy(circuit, params, initial, codes, coeffs):
    """Differentiable energy of a statevector Circuit (see CircuitEnergy):
    params a torch tensor, initial a Qureg with the initial state, (codes,
    coeffs) the Pauli sum."""
    return CircuitEnergy.apply(params, circuit, initial, codes, coeffs)
