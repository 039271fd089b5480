"""Parametrised multi-qubit Pauli gadgets in batches: energies and adjoint
gradients for gadgets of weight 2..N (every mix of X, Y and Z, parametrised
and fixed), against the oracle's states, its exact two-term shift rule for
exp(i theta P) (Sec. "Pauli gadget"), and central finite differences of the
batch's own energies; and the differentiable energies() wrapper."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def gadget_problem(rng, n, num_params, terms=8):
    """Layers of single-qubit rotations, a CZ ladder, and Pauli gadgets of
    weight 2..n on random qubits with random X/Y/Z (some with identities
    mixed in), parametrised or fixed."""
    ops = []
    k = 0
    for layer in range(2):
        for q in range(n):
            ops.append({"op": "gadget", "targs": (q,), "paulis": (2,), "theta": 0.0, "param": k, "scale": -0.5})
            k += 1
        for q in range(n - 1):
            ops.append({"op": "unitary", "ctrls": (q,), "targs": (q + 1,), "matrix": np.diag([1.0, -1.0])})
        for w in range(2, n + 1):
            t = [int(x) for x in rng.permutation(n)[:w]]
            p = [int(x) for x in rng.integers(1, 4, size=w)]
            if w >= 3:
                p[int(rng.integers(0, w))] = 0   # an identity inside the string
            if (w + layer) % 3 == 0:
                ops.append({"op": "gadget", "targs": tuple(t), "paulis": tuple(p), "theta": float(rng.uniform(-3, 3))})
            else:
                ops.append({"op": "gadget", "targs": tuple(t), "paulis": tuple(p), "theta": 0.0, "param": k,
                            "scale": float(rng.choice([1.0, -0.5, 0.75]))})
                k += 1
    assert k <= num_params
    params = rng.uniform(0, 2 * np.pi, size=k)
    for op in ops:
        if "param" in op:
            op["theta"] = op["scale"] * params[op["param"]]
    codes, coeffs = synth.random_pauli_sum(rng, n, terms)
    return {"n": n, "ops": ops, "params": params, "codes": codes, "coeffs": coeffs}


def build(qs, probs, prec):
    b = qs.Batch(prec)
    for p in probs:
        b.add_circuit(p["n"], p["ops"], len(p["params"]), p["codes"], p["coeffs"])
    return b.compile()


SIZES = [2, 3, 5, 8, 12, 13, 15]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_gadget_batch_energies_and_gradients(qs, prec):
    banner(f"batch gadgets {prec}")
    rng = np.random.default_rng(91)
    probs = [gadget_problem(rng, n, 10 * n) for n in SIZES]
    b = build(qs, probs, prec)
    params = np.concatenate([p["params"] for p in probs])
    e, g = b.run(params)
    offs = np.cumsum([0] + [len(p["params"]) for p in probs])
    for i, p in enumerate(probs):
        n = p["n"]
        hnorm = np.abs(p["coeffs"]).sum()
        want_psi = oracle.run_ops(oracle.zero_state(n), p["ops"])
        we = oracle.sv_expec_pauli_sum(want_psi, p["codes"], p["coeffs"]).real
        assert abs(e[i] - we) < TOL[prec] * hnorm, (n, e[i], we)
        want = oracle.param_shift_gradient(n, p["ops"], p["codes"], p["coeffs"], len(p["params"]))
        got = g[offs[i]:offs[i + 1]]
        bound = 1e-10 * max(1.0, hnorm) if prec == "c128" else 1e-4 * max(1.0, np.abs(want).max())
        assert np.abs(got - want).max() < bound, (n, np.abs(got - want).max())
    # the state left by a run without gradients
    e2, _ = b.run(params, grads=False)
    for i, p in enumerate(probs):
        want_psi = oracle.run_ops(oracle.zero_state(p["n"]), p["ops"])
        assert amp_err(b.state(i), want_psi) < TOL[prec], p["n"]


def test_gadget_batch_finite_differences(qs):
    """complex128: adjoint gradients of gadget circuits against central
    differences of the batch's own energies (h = 1e-5)."""
    banner("batch gadgets finite differences")
    rng = np.random.default_rng(92)
    probs = [gadget_problem(rng, n, 10 * n) for n in (4, 13)]
    b = build(qs, probs, "c128")
    params = np.concatenate([p["params"] for p in probs])
    _, g = b.run(params)
    h = 1e-5
    pick = rng.choice(params.size, size=16, replace=False)
    for j in pick:
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        ep, _ = b.run(pp, grads=False)
        em, _ = b.run(pm, grads=False)
        fd = (ep - em).sum() / (2 * h)   # parameter j belongs to one circuit
        assert abs(fd - g[j]) < 1e-6 * max(1.0, abs(g[j])), (int(j), fd, g[j])


def test_gadget_energies_autograd(qs):
    """energies() (torch.autograd.Function) on gadget circuits: the gradient
    of a weighted sum of energies against the oracle's shift rule."""
    import torch
    banner("batch gadgets autograd")
    rng = np.random.default_rng(93)
    probs = [gadget_problem(rng, n, 10 * n) for n in (3, 6, 10)]
    b = build(qs, probs, "c128")
    params = torch.tensor(np.concatenate([p["params"] for p in probs]), requires_grad=True)
    w = torch.tensor([0.5, -1.0, 2.0], dtype=torch.float64)
    loss = (qs.energies(b, params) * w).sum()
    loss.backward()
    offs = np.cumsum([0] + [len(p["params"]) for p in probs])
    for i, p in enumerate(probs):
        want = oracle.param_shift_gradient(p["n"], p["ops"], p["codes"], p["coeffs"], len(p["params"]))
        got = params.grad[offs[i]:offs[i + 1]].numpy()
        assert np.abs(got - w[i].item() * want).max() < 1e-10 * max(1.0, np.abs(want).max())


def test_gadget_argument_errors(qs):
    from paper_2311_01512_amd import native as N
    b = qs.Batch("c64")
    c = N.qs_batch_add_circuit(b._b, 4, 2)
    with pytest.raises(ValueError):
        N.qs_batch_add_gadget(b._b, c, [0, 1], [0, 0], 0, 1.0)      # identity string
    with pytest.raises(ValueError):
        N.qs_batch_add_gadget(b._b, c, [0, 0], [1, 2], 0, 1.0)      # duplicate qubit
    with pytest.raises(ValueError):
        N.qs_batch_add_gadget(b._b, c, [0, 4], [1, 2], 0, 1.0)      # qubit out of range
    with pytest.raises(ValueError):
        N.qs_batch_add_gadget(b._b, c, [0, 1], [1, 2], 2, 1.0)      # parameter out of range
