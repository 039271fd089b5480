"""SWAP gates, multi-swaps, Pauli tensors, phase gadgets and the one-pass
density-matrix Pauli gadget against the FP64 oracle, on statevectors and
density matrices of both precisions."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner

pytestmark = pytest.mark.gpu

PRECS = ["c128", "c64"]


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def _mixed_state(rng, N):
    """A random full-rank density matrix as a Choi vector (k + l 2^N)."""
    a = synth.random_matrix(rng, 1 << N)
    rho = a @ a.conj().T
    rho /= np.trace(rho)
    return rho.reshape(-1, order="F")


def _random_paulis(rng, N, w, codes=(0, 1, 2, 3)):
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.choice(codes, size=w)]
    return t, p


@pytest.mark.parametrize("prec", PRECS)
def test_swap_every_pair(qs, prec):
    N = 7
    rng = np.random.default_rng(11)
    psi = synth.random_state(rng, 1 << N)
    banner(f"swap every pair N={N} {prec}")
    for t1 in range(N):
        for t2 in range(N):
            if t1 == t2:
                continue
            q = qs.Qureg(N, precision=prec).set_amps(psi)
            q.apply_swap(t1, t2)
            want = oracle.apply_swap(psi.copy(), t1, t2)
            assert amp_err(q.get_amps(), want) < TOL[prec], (t1, t2)


@pytest.mark.parametrize("prec", PRECS)
def test_density_swap(qs, prec):
    N = 5
    rng = np.random.default_rng(12)
    rho = _mixed_state(rng, N)
    for t1, t2 in ((0, 1), (4, 0), (2, 3), (1, 4)):
        banner(f"density swap ({t1},{t2}) {prec}")
        q = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
        q.apply_swap(t1, t2)
        want = oracle.dm_apply_swap(rho.copy(), t1, t2)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("density", [False, True])
def test_multi_swap(qs, prec, density):
    """1 to 4 disjoint pairs: one launch of up to three index-bit pairs, two
    launches beyond (a density matrix doubles the pairs)."""
    N = 9 if not density else 5
    rng = np.random.default_rng(13 + density)
    state = _mixed_state(rng, N) if density else synth.random_state(rng, 1 << N)
    for npairs in range(1, N // 2 + 1):
        perm = [int(x) for x in rng.permutation(N)[:2 * npairs]]
        a, b = perm[0::2], perm[1::2]
        banner(f"multi-swap {npairs} pairs density={density} {prec}")
        q = qs.Qureg(N, density=density, precision=prec).set_amps(state)
        q.apply_multi_swap(a, b)
        want = state.copy()
        for x, y in zip(a, b):
            want = (oracle.dm_apply_swap if density else oracle.apply_swap)(want, x, y)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_swaps_staged_through_lds(qs, prec):
    """Pairs that involve a bit inside a 128-byte line go through the
    LDS-staged tile kernel once the register holds a whole tile: single and
    multiple pairs, low-low, low-high, and a density matrix whose pairs are
    doubled onto the column bits."""
    rng = np.random.default_rng(19)
    N = 14
    psi = synth.random_state(rng, 1 << N)
    cases = [([0], [13]), ([0], [1]), ([3], [13]), ([2], [9]), ([0, 1, 2], [13, 12, 11]),
             ([0, 5, 9], [3, 12, 1]), ([1, 8], [11, 2]), ([0, 1, 2, 3], [10, 11, 12, 13])]
    for a, b in cases:
        banner(f"staged swaps {a}<->{b} N={N} {prec}")
        q = qs.Qureg(N, precision=prec).set_amps(psi)
        q.apply_multi_swap(a, b)
        want = psi.copy()
        for x, y in zip(a, b):
            want = oracle.apply_swap(want, x, y)
        assert amp_err(q.get_amps(), want) < TOL[prec]
    Nd = 7
    rho = _mixed_state(rng, Nd)
    for a, b in (([0], [6]), ([1, 0], [5, 3]), ([2], [3])):
        banner(f"staged density swaps {a}<->{b} N={Nd} {prec}")
        q = qs.Qureg(Nd, density=True, precision=prec).set_amps(rho)
        q.apply_multi_swap(a, b)
        want = rho.copy()
        for x, y in zip(a, b):
            want = oracle.dm_apply_swap(want, x, y)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_pauli_tensor(qs, prec):
    N = 8
    rng = np.random.default_rng(14)
    psi = synth.random_state(rng, 1 << N)
    cases = [([0], [1]), ([7], [2]), ([3], [3]), ([0, 7, 3, 5], [3, 3, 0, 3]), ([2, 4], [0, 0])]
    for _ in range(8):
        cases.append(_random_paulis(rng, N, int(rng.integers(1, N + 1))))
    for t, p in cases:
        banner(f"pauli tensor t={t} p={p} {prec}")
        q = qs.Qureg(N, precision=prec).set_amps(psi)
        q.apply_pauli_tensor(t, p)
        want = oracle.apply_pauli_tensor(psi.copy(), t, p)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_density_pauli_tensor(qs, prec):
    N = 5
    rng = np.random.default_rng(15)
    rho = _mixed_state(rng, N)
    cases = [([1], [2]), ([0, 4], [2, 2]), ([3, 1], [3, 0]), ([2], [0])]
    for _ in range(5):
        cases.append(_random_paulis(rng, N, int(rng.integers(1, N + 1))))
    for t, p in cases:
        banner(f"density pauli tensor t={t} p={p} {prec}")
        q = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
        q.apply_pauli_tensor(t, p)
        want = oracle.dm_apply_pauli_tensor(rho.copy(), t, p)
        assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("density", [False, True])
def test_phase_gadget(qs, prec, density):
    N = 8 if not density else 5
    rng = np.random.default_rng(16 + density)
    state = _mixed_state(rng, N) if density else synth.random_state(rng, 1 << N)
    for w in range(1, N + 1):
        t = [int(x) for x in rng.permutation(N)[:w]]
        theta = float(rng.uniform(-7, 7))
        banner(f"phase gadget t={t} density={density} {prec}")
        q = qs.Qureg(N, density=density, precision=prec).set_amps(state)
        q.apply_phase_gadget(t, theta)
        f = oracle.dm_apply_phase_gadget if density else oracle.apply_phase_gadget
        assert amp_err(q.get_amps(), f(state.copy(), t, theta)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_density_pauli_gadget_one_pass(qs, prec):
    """The fused density-matrix gadget (both halves of the Choi vector in one
    pass): X/Y/Z strings of every weight, Z-only, identity-only."""
    N = 5
    rng = np.random.default_rng(17)
    rho = _mixed_state(rng, N)
    cases = [([2], [2]), ([0, 4], [1, 2]), ([1, 3], [3, 3]), ([0], [0]), ([4, 0, 2], [2, 2, 2])]
    for _ in range(8):
        cases.append(_random_paulis(rng, N, int(rng.integers(1, N + 1))))
    for t, p in cases:
        theta = float(rng.uniform(-4, 4))
        banner(f"density gadget t={t} p={p} {prec}")
        q = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
        q.apply_pauli_gadget(t, p, theta)
        want = oracle.dm_apply_pauli_gadget(rho.copy(), t, p, theta)
        assert amp_err(q.get_amps(), want) < TOL[prec]


def test_special_ops_many_groups(qs):
    """11-qubit density matrix (2^22 Choi amplitudes, many blocks per launch)
    and a 20-qubit statevector, every special operator in turn."""
    rng = np.random.default_rng(18)
    N = 11
    psi = synth.random_state(rng, 1 << N)
    rho = np.outer(psi, psi.conj()).reshape(-1, order="F")
    ops = [{"op": "swap", "targs": (0, 10)},
           {"op": "pauli_tensor", "targs": (10, 3, 0), "paulis": (2, 1, 3)},
           {"op": "phase_gadget", "targs": (9, 1, 5, 0), "theta": 0.37},
           {"op": "gadget", "targs": (7, 2), "paulis": (1, 2), "theta": -1.1},
           {"op": "swap", "targs": (4, 6)}]
    want = oracle.run_ops(rho.copy(), ops, density=True)
    for prec in PRECS:
        banner(f"special ops DM N=11 {prec}")
        q = qs.Qureg(N, density=True, precision=prec).set_amps(rho)
        q.run_ops(ops)
        assert amp_err(q.get_amps(), want) < TOL[prec]
    Ns = 20
    psi = synth.random_state(rng, 1 << Ns)
    ops = [{"op": "swap", "targs": (19, 0)},
           {"op": "pauli_tensor", "targs": (19, 3, 0, 11), "paulis": (2, 1, 3, 2)},
           {"op": "phase_gadget", "targs": (18, 1, 5), "theta": 2.2},
           {"op": "swap", "targs": (12, 2)}]
    want = oracle.run_ops(psi.copy(), ops)
    for prec in PRECS:
        banner(f"special ops SV N=20 {prec}")
        q = qs.Qureg(Ns, precision=prec).set_amps(psi)
        q.run_ops(ops)
        assert amp_err(q.get_amps(), want) < TOL[prec]


def test_special_ops_errors(qs):
    q = qs.Qureg(3, precision="c128").init_zero()
    with pytest.raises(ValueError):
        q.apply_swap(1, 1)                          # same qubit
    with pytest.raises(ValueError):
        q.apply_swap(0, 3)                          # qubit 3 of 3
    with pytest.raises(ValueError):
        q.apply_multi_swap([0, 1], [1, 2])          # pairs overlap
    with pytest.raises(ValueError):
        q.apply_pauli_tensor([0, 1], [1, 4])        # bad code
    with pytest.raises(ValueError):
        q.apply_pauli_tensor([0, 0], [1, 1])        # repeated target
    with pytest.raises(ValueError):
        q.apply_phase_gadget([], 0.3)               # no targets
    d = qs.Qureg(2, density=True, precision="c128").init_zero()
    with pytest.raises(ValueError):
        d.apply_swap(0, 2)                          # qubit 2 of a 2-qubit matrix
    with pytest.raises(ValueError):
        d.apply_pauli_gadget([2], [1], 0.1)         # column bit is not a qubit
