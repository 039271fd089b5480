"""Pauli sums on statevectors of 8 or more qubits, evaluated by tiles that
hold the partners of several flip masks at once: parity with the FP64 oracle
for many masks (several tile spans), many terms per mask (several launches
per span), masks inside the contiguous low qubits, diagonal and identity
terms, and more terms than one read-back holds."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import banner, scalar_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def state(qs, rng, n, prec):
    psi = synth.random_state(rng, 1 << n)
    return psi, qs.Qureg(n, precision=prec).set_amps(psi)


def check(qs, n, prec, codes, coeffs, seed):
    rng = np.random.default_rng(seed)
    psi, q = state(qs, rng, n, prec)
    got = q.expec_pauli_sum(codes, coeffs)
    want = oracle.sv_expec_pauli_sum(psi, codes, coeffs)
    assert abs(got - want) < scalar_tol(prec, np.abs(coeffs).sum()), (got, want)
    assert got == q.expec_pauli_sum(codes, coeffs)      # fixed summation order
    return got


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n,T", [(8, 12), (9, 40), (11, 25), (12, 40), (13, 30), (16, 40), (18, 20)])
def test_random_sums(qs, prec, n, T):
    banner(f"tiled Pauli sum N={n} T={T} {prec}")
    rng = np.random.default_rng(8100 + n)
    codes, coeffs = synth.random_pauli_sum(rng, n, T)
    codes[0, :] = 0                                   # identity
    codes[1, :] = rng.choice([0, 3], size=n)          # diagonal
    check(qs, n, prec, codes, coeffs, 8200 + n)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_many_terms_per_mask(qs, prec):
    """40 terms on two flip masks (one span, three launches of at most 16)
    and 70 terms in all (more results than one read-back)."""
    banner(f"tiled Pauli sum, shared masks {prec}")
    n = 14
    rng = np.random.default_rng(8300)
    codes = np.where(rng.random((70, n)) < 0.5, 3, 0).astype(np.int32)
    codes[:35, 2] = 1
    codes[:35, 11] = 2
    codes[35:, 13] = 1
    coeffs = rng.standard_normal(70)
    check(qs, n, prec, codes, coeffs, 8301)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_low_qubit_and_single_masks(qs, prec):
    """Flips confined to the contiguous low qubits, single-qubit X and Y on
    the highest qubit, Y-parity odd and even terms."""
    banner(f"tiled Pauli sum, low masks {prec}")
    n = 15
    rows = []
    for spec in ({0: 1}, {1: 2, 3: 1}, {0: 2, 1: 2}, {n - 1: 1}, {n - 1: 2}, {0: 2, n - 1: 2, 7: 3},
                 {2: 1, 9: 2, 14: 3}, {}):
        r = np.zeros(n, np.int32)
        for k, v in spec.items():
            r[k] = v
        rows.append(r)
    codes = np.array(rows)
    coeffs = np.linspace(-1.0, 1.5, len(rows))
    check(qs, n, prec, codes, coeffs, 8400)


def test_closed_forms(qs):
    """|+>^N: <X_k> = 1, <Z_k> = 0, <Y_k> = 0; a GHZ-like state
    (|0..0> + |1..1>)/sqrt2: <X^N> = 1, <Z_0 Z_k> = 1, <Y_0 Y_1 X^(N-2)> = -1."""
    banner("tiled Pauli sum, closed forms")
    n = 12
    q = qs.Qureg(n, precision="c128").init_plus()
    codes = np.zeros((3, n), np.int32)
    codes[0, 5] = 1
    codes[1, 7] = 3
    codes[2, 11] = 2
    for i in range(3):
        want = 1.0 if i == 0 else 0.0
        assert abs(q.expec_pauli_sum(codes[i:i + 1], [1.0]) - want) < 1e-12
    ghz = np.zeros(1 << n, complex)
    ghz[0] = ghz[-1] = 2 ** -0.5
    q.set_amps(ghz)
    xall = np.ones((1, n), np.int32)
    zz = np.zeros((1, n), np.int32)
    zz[0, 0] = zz[0, 9] = 3
    yyx = np.ones((1, n), np.int32)
    yyx[0, 0] = yyx[0, 1] = 2
    assert abs(q.expec_pauli_sum(xall, [1.0]) - 1.0) < 1e-12
    assert abs(q.expec_pauli_sum(zz, [1.0]) - 1.0) < 1e-12
    assert abs(q.expec_pauli_sum(yyx, [1.0]) + 1.0) < 1e-12
