"""Run-time specialised batch steps (qs_batch_specialize): energies,
gradients and states equal those of the generic kernels bit for bit, with
graph replays and eager launches, after specialising twice and after
recompiling; and agree with the oracle."""
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


def hea_problem(rng, n, layers, terms=6, extra=False):
    angles = rng.uniform(0, 2 * np.pi, size=2 * n * layers)
    ops = synth.circuits.hea_circuit(n, angles, layers)
    if extra:   # fixed gates, a long-range CZ and a parametrised gadget as well
        ops = ops[:3] + [{"op": "unitary", "ctrls": (), "targs": (n - 1,), "matrix": synth.haar_unitary(rng, 2)},
                         {"op": "unitary", "ctrls": (0,), "targs": (n - 1,), "matrix": np.diag([1.0, -1.0])},
                         {"op": "gadget", "targs": (1, n - 2, n - 1), "paulis": (1, 2, 3),
                          "theta": 0.75 * angles[0], "param": 0, "scale": 0.75}] + ops[3:]
    codes, coeffs = synth.random_pauli_sum(rng, n, terms)
    return {"n": n, "angles": angles, "ops": ops, "codes": codes, "coeffs": coeffs}


def build(qs, probs, prec, use_graph=True):
    b = qs.Batch(prec)
    for p in probs:
        b.add_circuit(p["n"], p["ops"], len(p["angles"]), p["codes"], p["coeffs"])
    return b.compile(use_graph=use_graph)


# register-path steps (9 and more qubits), several steps per circuit from 13
# qubits on, repeated sizes sharing programs, and a small LDS-path circuit
SIZES = [5, 9, 10, 10, 12, 13, 14, 14, 16]


def params_of(probs, rng):
    return rng.uniform(0, 2 * np.pi, size=sum(len(p["angles"]) for p in probs))


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_specialized_batch_equals_generic(qs, prec):
    banner(f"specialised batch {prec}")
    rng = np.random.default_rng(71)
    probs = [hea_problem(rng, n, 2 + (n % 2), extra=(n in (10, 13))) for n in SIZES]
    gen = build(qs, probs, prec)
    spec = build(qs, probs, prec)
    progs = spec.specialize()
    assert progs >= 1
    for r in range(3):
        params = params_of(probs, rng)
        eg, gg = gen.run(params, grads=(r != 1))
        es, gs = spec.run(params, grads=(r != 1))
        assert np.array_equal(eg, es)
        if r != 1:
            assert np.array_equal(gg, gs)
    # final states (the last run skipped gradients only at r = 1: run forward)
    params = params_of(probs, rng)
    gen.run(params, grads=False)
    spec.run(params, grads=False)
    for i, p in enumerate(probs):
        assert np.array_equal(gen.state(i), spec.state(i)), p["n"]


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_specialized_batch_against_oracle(qs, prec):
    banner(f"specialised batch vs oracle {prec}")
    rng = np.random.default_rng(73)
    probs = [hea_problem(rng, n, 2, extra=(n == 13)) for n in (9, 13, 14)]
    b = build(qs, probs, prec)
    b.specialize()
    params = np.concatenate([p["angles"] for p in probs])
    e, g = b.run(params, grads=True)
    k = 0
    for i, p in enumerate(probs):
        m = len(p["angles"])
        psi = oracle.run_ops(oracle.zero_state(p["n"]), p["ops"])
        we = oracle.sv_expec_pauli_sum(psi, p["codes"], p["coeffs"]).real
        assert abs(e[i] - we) < TOL[prec] * max(1.0, np.abs(p["coeffs"]).sum()), p["n"]
        want = oracle.param_shift_gradient(p["n"], p["ops"], p["codes"], p["coeffs"], m)
        tol = 1e-10 if prec == "c128" else 1e-4
        assert np.abs(g[k:k + m] - want).max() < tol * max(1.0, np.abs(want).max()), p["n"]
        k += m
    b.run(params, grads=False)
    for i, p in enumerate(probs):
        psi = oracle.run_ops(oracle.zero_state(p["n"]), p["ops"])
        assert amp_err(b.state(i), psi) < TOL[prec], p["n"]


def test_specialized_batch_eager_twice_and_recompiled(qs):
    """Eager launches of the specialised kernels equal graph replays;
    specialising a second time and recompiling (which drops the
    specialisation) leave the results unchanged."""
    rng = np.random.default_rng(79)
    probs = [hea_problem(rng, n, 2, extra=(n == 12)) for n in (9, 12, 14)]
    ref = build(qs, probs, "c64")
    eager = build(qs, probs, "c64", use_graph=False)
    eager.specialize()
    twice = build(qs, probs, "c64")
    twice.specialize()
    twice.specialize()
    params = params_of(probs, rng)
    e0, g0 = ref.run(params)
    for b in (eager, twice):
        e, g = b.run(params)
        assert np.array_equal(e, e0) and np.array_equal(g, g0)
    twice.compile()
    e, g = twice.run(params)
    assert np.array_equal(e, e0) and np.array_equal(g, g0)


def test_specialize_requires_compiled(qs):
    b = qs.Batch("c64")
    b.add_circuit(10, [], 0)
    with pytest.raises(RuntimeError):
        b.specialize()
    with pytest.raises(ValueError):
        qs.native.qs_batch_specialize(b._b)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_batch_circuits_without_operators(qs, prec):
    """Circuits with no operators keep |0..0> (the only ones the initial-state
    kernel writes; a circuit's first step reads |0..0> itself), also on a
    second run after an adjoint sweep and with specialised steps."""
    rng = np.random.default_rng(83)
    probs = [hea_problem(rng, n, 1) for n in (4, 10, 11)]
    for p in probs[:2]:
        p["ops"], p["angles"] = [], np.zeros(0)
    b = build(qs, probs, prec)
    b.specialize()
    params = np.concatenate([p["angles"] for p in probs])
    for grads in (True, False):
        e, _ = b.run(params, grads=grads)
        for i, p in enumerate(probs):
            psi = oracle.run_ops(oracle.zero_state(p["n"]), p["ops"])
            we = oracle.sv_expec_pauli_sum(psi, p["codes"], p["coeffs"]).real
            assert abs(e[i] - we) < TOL[prec] * max(1.0, np.abs(p["coeffs"]).sum()), (p["n"], grads)
    for i, p in enumerate(probs):
        psi = oracle.run_ops(oracle.zero_state(p["n"]), p["ops"])
        assert amp_err(b.state(i), psi) < TOL[prec], p["n"]
