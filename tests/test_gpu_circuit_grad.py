"""Adjoint gradients of single-state circuits (qs_circuit_adjoint_gradient)
with parametrised Pauli gadgets of weight 1..N (Sec. "Pauli gadget") among
fixed many-target gates with controls and fixed gadgets: the energy against
the oracle, the gradient against the oracle's exact two-term shift rule and
central finite differences, and the torch.autograd wrapper."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def problem(rng, n, layers=2, terms=10):
    ops, k = [], 0
    for _ in range(layers):
        for w in range(1, n + 1):
            t = [int(x) for x in rng.permutation(n)[:w]]
            p = [int(x) for x in rng.integers(1, 4, size=w)]
            ops.append({"op": "gadget", "targs": tuple(t), "paulis": tuple(p), "param": k,
                        "scale": float(rng.choice([1.0, -0.5, 0.3]))})
            k += 1
            if w % 3 == 0:
                q = [int(x) for x in rng.permutation(n)[:4]]
                ops.append({"op": "unitary", "ctrls": (q[2],), "targs": (q[0], q[1]),
                            "matrix": synth.haar_unitary(rng, 4)})
                ops.append({"op": "gadget", "targs": (q[3], q[0]), "paulis": (2, 1), "theta": 0.4})
    params = rng.uniform(0, 2 * np.pi, size=k)
    for op in ops:
        if "param" in op:
            op["theta"] = op["scale"] * params[op["param"]]
    codes, coeffs = synth.random_pauli_sum(rng, n, terms)
    return ops, params, codes, coeffs


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 4, 9, 16])
def test_circuit_adjoint_gradient(qs, prec, n):
    banner(f"circuit adjoint gradient n={n} {prec}")
    rng = np.random.default_rng(500 + n)
    ops, params, codes, coeffs = problem(rng, n)
    c = qs.Circuit(n, ops)
    c.set_params(params)
    psi = qs.Qureg(n, precision=prec).init_zero()
    lam = qs.Qureg(n, precision=prec)
    e, g = c.adjoint_gradient(psi, lam, codes, coeffs)
    hnorm = np.abs(coeffs).sum()
    want_psi = oracle.run_ops(oracle.zero_state(n), ops)
    we = oracle.sv_expec_pauli_sum(want_psi, codes, coeffs).real
    assert abs(e - we) < TOL[prec] * max(1.0, hnorm), (e, we)
    want = oracle.param_shift_gradient(n, ops, codes, coeffs, len(params))
    bound = 1e-10 * max(1.0, hnorm) if prec == "c128" else 1e-4 * max(1.0, np.abs(want).max())
    assert np.abs(g - want).max() < bound, np.abs(g - want).max()
    # psi is back at the initial state
    z = oracle.zero_state(n)
    assert np.abs(psi.get_amps() - z).max() < (1e-12 if prec == "c128" else 1e-5)


def test_circuit_gradient_finite_differences(qs):
    banner("circuit gradient finite differences")
    rng = np.random.default_rng(77)
    n = 8
    ops, params, codes, coeffs = problem(rng, n)
    c = qs.Circuit(n, ops)
    psi = qs.Qureg(n, precision="c128").init_zero()
    lam = qs.Qureg(n, precision="c128")
    c.set_params(params)
    _, g = c.adjoint_gradient(psi, lam, codes, coeffs)
    h = 1e-5
    for j in rng.choice(params.size, size=10, replace=False):
        es = []
        for d in (h, -h):
            p = params.copy()
            p[j] += d
            c.set_params(p)
            psi.init_zero()
            es.append(c.adjoint_gradient(psi, lam, codes, coeffs)[0])
        fd = (es[0] - es[1]) / (2 * h)
        assert abs(fd - g[j]) < 1e-6 * max(1.0, abs(g[j])), (int(j), fd, g[j])


def test_circuit_energy_autograd(qs):
    import torch
    banner("circuit energy autograd")
    rng = np.random.default_rng(78)
    n = 7
    ops, params, codes, coeffs = problem(rng, n)
    c = qs.Circuit(n, ops)
    init = qs.Qureg(n, precision="c128").init_zero()
    x = torch.tensor(params, requires_grad=True)
    e = qs.circuit_energy(c, x, init, codes, coeffs)
    (3.0 * e).backward()
    want = oracle.param_shift_gradient(n, ops, codes, coeffs, len(params))
    assert np.abs(x.grad.numpy() - 3.0 * want).max() < 1e-10 * max(1.0, np.abs(want).max())
    we = oracle.sv_expec_pauli_sum(oracle.run_ops(oracle.zero_state(n), ops), codes, coeffs).real
    assert abs(e.item() - we) < 1e-12 * max(1.0, np.abs(coeffs).sum())


def test_circuit_gradient_errors(qs):
    from paper_2311_01512_amd import native as N
    c = qs.Circuit(3, density=True)
    with pytest.raises(ValueError):
        N.qs_circuit_add_param_gadget(c._c, [0], [1], 0, 1.0)       # density circuit
    c2 = qs.Circuit(3, [{"op": "gadget", "targs": (0, 1), "paulis": (1, 3), "param": 2, "scale": 1.0}])
    psi = qs.Qureg(3, precision="c128").init_zero()
    lam = qs.Qureg(3, precision="c128")
    with pytest.raises(ValueError):
        c2.adjoint_gradient(psi, lam, np.zeros((1, 3), np.int32), [1.0], num_params=2)   # param 2 of 2
    with pytest.raises(ValueError):
        c2.adjoint_gradient(psi, psi, np.zeros((1, 3), np.int32), [1.0], num_params=3)   # aliasing
