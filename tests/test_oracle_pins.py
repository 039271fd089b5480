"""Pins of the FP64 oracle against things other than itself: dense
Kronecker-product operators (oracle/dense.py), the paper's worked examples
(tests/golden), closed forms, the channels' amplitude rules as printed in the
paper, and invariants.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.dense as D
import synth

TOL = 1e-12


def rng_for(seed):
    return np.random.default_rng(seed)


def rand_state(rng, n):
    return synth.random_state(rng, 1 << n)


def rand_dm(rng, n, rank=3):
    """Random positive, unit-trace density matrix (as a dense matrix)."""
    A = rng.standard_normal((1 << n, rank)) + 1j * rng.standard_normal((1 << n, rank))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


# ---- worked examples ---------------------------------------------------------

def test_bit_convention_golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "bit_convention.json")))
    N, idx = g["num_qubits"], g["index"]
    for q, b in g["bits"].items():
        assert (idx >> int(q)) & 1 == b
    assert idx == sum(b << (N - 1 - a) for a, b in enumerate(g["kets_msb_first"]))
    # an X on qubit q flips exactly bit q of the basis index
    for q in range(N):
        psi = oracle.basis_state(N, idx)
        oracle.apply_gate(psi, [], [q], synth.pauli_matrix_2x2(1))
        assert abs(psi[idx ^ (1 << q)] - 1) < TOL and np.count_nonzero(psi) == 1


def test_target_order_golden(golden_dir):
    """The matrix index bit q belongs to targets[q]: a permutation gate that
    maps local state j=0 to j=2 moves |k=1, j=0> to |k=1, j=2> = |3>."""
    g = json.load(open(os.path.join(golden_dir, "target_order.json")))
    N, t = g["num_qubits"], g["targets"]
    P = np.eye(4, dtype=complex)[[2, 1, 0, 3]]      # swaps local states 0 and 2
    # |k=1, j=0>: target qubits zero, k's bit 0 on the lowest free qubit
    free = [q for q in range(N) if q not in t]
    start = sum(((g["k"] >> b) & 1) << q for b, q in enumerate(free))
    psi = oracle.basis_state(N, start)
    oracle.apply_gate(psi, [], t, P)
    assert np.argmax(np.abs(psi)) == g["index"]
    assert abs(psi[g["index"]] - 1) < TOL


def test_splitmix64_golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    for c, want in enumerate(g["outputs"]):
        assert oracle.splitmix64_at(g["seed"], c) == int(want)


# ---- statevector gates -----------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_gate_matches_dense_kronecker(seed):
    rng = rng_for(seed)
    N = int(rng.integers(2, 9))
    nt = int(rng.integers(1, min(4, N) + 1))
    ns = int(rng.integers(0, min(3, N - nt) + 1))
    qs = rng.permutation(N)[:nt + ns]
    t, c = [int(x) for x in qs[:nt]], [int(x) for x in qs[nt:]]
    M = synth.random_matrix(rng, 1 << nt)            # not unitary on purpose
    psi = rand_state(rng, N)
    want = D.gate_operator(N, c, t, M) @ psi
    got = oracle.apply_gate(psi.copy(), c, t, M)
    assert np.abs(got - want).max() < TOL


def test_ghz_closed_form():
    for N in (1, 2, 5, 9):
        psi = oracle.zero_state(N)
        h = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
        oracle.apply_gate(psi, [], [0], h)
        for q in range(N - 1):
            oracle.apply_gate(psi, [q], [q + 1], synth.pauli_matrix_2x2(1))
        want = np.zeros(1 << N, complex)
        want[0] = want[-1] = 1 / np.sqrt(2)
        assert np.abs(psi - want).max() < TOL


def test_qft_of_basis_state_closed_form():
    """QFT|x> = sum_y e^{2 pi i x y / 2^N} |y> / sqrt(2^N), built from H,
    controlled phases and a final qubit reversal by 2-target SWAP gates."""
    h = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    swap = np.eye(4, dtype=complex)[[0, 2, 1, 3]]
    for N, x in ((3, 5), (6, 19), (8, 200)):
        psi = oracle.basis_state(N, x)
        for j in range(N - 1, -1, -1):
            oracle.apply_gate(psi, [], [j], h)
            for k in range(j - 1, -1, -1):
                ph = np.diag([1, np.exp(1j * np.pi / (1 << (j - k)))])
                oracle.apply_gate(psi, [k], [j], ph)
        for q in range(N // 2):
            oracle.apply_gate(psi, [], [q, N - 1 - q], swap)
        y = np.arange(1 << N)
        want = np.exp(2j * np.pi * x * y / (1 << N)) / np.sqrt(1 << N)
        assert np.abs(psi - want).max() < 1e-12


def test_haar_gates_preserve_norm():
    rng = rng_for(7)
    psi = rand_state(rng, 10)
    for _ in range(40):
        n = int(rng.integers(1, 4))
        qs = rng.permutation(10)[:n + 1]
        oracle.apply_gate(psi, [int(qs[-1])], [int(q) for q in qs[:n]], synth.haar_unitary(rng, 1 << n))
    assert abs(oracle.sv_total_prob(psi) - 1) < 1e-12


@pytest.mark.parametrize("seed", range(10))
def test_pauli_gadget_equals_expm(seed):
    rng = rng_for(100 + seed)
    N = int(rng.integers(1, 9))
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(1, 4, size=w)]
    theta = rng.uniform(-7, 7)
    psi = rand_state(rng, N)
    want = D.gadget_operator(N, t, p, theta) @ psi
    # Euler form cos(theta) 1 + i sin(theta) P agrees with the exponential
    P = D.pauli_operator(N, t, p)
    assert np.abs((np.cos(theta) * np.eye(1 << N) + 1j * np.sin(theta) * P) @ psi - want).max() < 1e-12
    got = oracle.apply_pauli_gadget(psi.copy(), t, p, theta)
    assert np.abs(got - want).max() < 1e-12


def test_phase_gadget_is_diagonal():
    rng = rng_for(5)
    N, t, theta = 7, [0, 3, 6], 0.731
    psi = rand_state(rng, N)
    got = oracle.apply_pauli_gadget(psi.copy(), t, [3, 3, 3], theta)
    mask = sum(1 << q for q in t)
    s = np.array([(-1) ** bin(i & mask).count("1") for i in range(1 << N)])
    assert np.abs(got - np.exp(1j * theta * s) * psi).max() < TOL


def test_identity_paulis_are_ignored():
    rng = rng_for(6)
    psi = rand_state(rng, 5)
    a = oracle.apply_pauli_gadget(psi.copy(), [0, 2, 4], [0, 1, 0], 0.3)
    b = oracle.apply_pauli_gadget(psi.copy(), [2], [1], 0.3)
    assert np.abs(a - b).max() < TOL


# ---- density matrices ----------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_dm_gate_matches_dense(seed):
    rng = rng_for(200 + seed)
    N = int(rng.integers(2, 6))
    nt = int(rng.integers(1, min(3, N) + 1))
    ns = int(rng.integers(0, min(2, N - nt) + 1))
    qs = rng.permutation(N)[:nt + ns]
    t, c = [int(x) for x in qs[:nt]], [int(x) for x in qs[nt:]]
    M = synth.random_matrix(rng, 1 << nt)
    rho = rand_dm(rng, N)
    F = D.gate_operator(N, c, t, M)
    want = D.choi(F @ rho @ F.conj().T)
    got = oracle.dm_apply_gate(D.choi(rho), c, t, M)
    assert np.abs(got - want).max() < TOL


@pytest.mark.parametrize("seed", range(8))
def test_dm_gadget_matches_dense(seed):
    """Pins the reading conj(exp(i theta P)) = exp(i (-1)^{m+1} theta P)."""
    rng = rng_for(300 + seed)
    N = int(rng.integers(1, 6))
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(1, 4, size=w)]
    theta = rng.uniform(-4, 4)
    rho = rand_dm(rng, N)
    G = D.gadget_operator(N, t, p, theta)
    want = D.choi(G @ rho @ G.conj().T)
    got = oracle.dm_apply_pauli_gadget(D.choi(rho), t, p, theta)
    assert np.abs(got - want).max() < TOL


@pytest.mark.parametrize("seed", range(8))
def test_kraus_map_matches_operator_sum(seed):
    rng = rng_for(400 + seed)
    N = int(rng.integers(2, 6))
    n = int(rng.integers(1, 3))
    t = [int(x) for x in rng.permutation(N)[:n]]
    M = int(rng.integers(1, 5))
    ks = np.stack([synth.random_matrix(rng, 1 << n) for _ in range(M)])   # not CPTP
    rho = rand_dm(rng, N)
    want = D.choi(D.kraus_apply(N, rho, t, ks))
    got = oracle.dm_apply_kraus(D.choi(rho), t, ks)
    assert np.abs(got - want).max() < 1e-11
    got2 = oracle.dm_apply_superop(D.choi(rho), t, oracle.build_superop(ks))
    assert np.abs(got2 - want).max() < 1e-11


def _choi_bit(i, q):
    return (i >> q) & 1


def test_dephasing_rule():
    """Sec. Dephasing channel: entries whose principal bits differ scale by 1-2p."""
    rng = rng_for(11)
    N, t, p = 3, 1, 0.23
    beta = D.choi(rand_dm(rng, N))
    got = oracle.dm_apply_kraus(beta.copy(), [t], synth.kraus_dephasing_1q(p))
    want = np.array([b if _choi_bit(i, t) == _choi_bit(i, t + N) else (1 - 2 * p) * b
                     for i, b in enumerate(beta)])
    assert np.abs(got - want).max() < TOL


def test_dephasing_2q_rule():
    """Eq. dephasing_2qb_update_rule: unless both principal pairs agree, an
    entry scales by 1 - 4p/3."""
    rng = rng_for(16)
    N, t1, t2, p = 3, 2, 0, 0.41
    beta = D.choi(rand_dm(rng, N))
    got = oracle.dm_apply_kraus(beta.copy(), [t1, t2], synth.kraus_dephasing_2q(p))
    want = np.array([b if (_choi_bit(i, t1) == _choi_bit(i, t1 + N) and _choi_bit(i, t2) == _choi_bit(i, t2 + N))
                     else (1 - 4 * p / 3) * b for i, b in enumerate(beta)])
    assert np.abs(got - want).max() < TOL


def test_depolarising_1q_rule():
    """Eq. depolarising_1qb_amp_update."""
    rng = rng_for(12)
    N, t, p = 3, 2, 0.37
    beta = D.choi(rand_dm(rng, N))
    got = oracle.dm_apply_kraus(beta.copy(), [t], synth.kraus_depolarising_1q(p))
    flip = (1 << t) | (1 << (t + N))
    want = np.array([(1 - 2 * p / 3) * b + (2 * p / 3) * beta[i ^ flip]
                     if _choi_bit(i, t) == _choi_bit(i, t + N) else (1 - 4 * p / 3) * b
                     for i, b in enumerate(beta)])
    assert np.abs(got - want).max() < TOL


def test_depolarising_2q_rule():
    """Eq. 2qb_depolarising_choi_amp_update (the printed equation, which the
    channel's own definition confirms; see test_depolarising_2q_definition)."""
    rng = rng_for(13)
    N, t1, t2, p = 3, 0, 2, 0.29
    beta = D.choi(rand_dm(rng, N))
    got = oracle.dm_apply_kraus(beta.copy(), [t1, t2], synth.kraus_depolarising_2q(p))
    f1 = (1 << t1) | (1 << (t1 + N))
    f2 = (1 << t2) | (1 << (t2 + N))
    want = []
    for i, b in enumerate(beta):
        if _choi_bit(i, t1) == _choi_bit(i, t1 + N) and _choi_bit(i, t2) == _choi_bit(i, t2 + N):
            want.append((1 - 4 * p / 5) * b + (4 * p / 15) * (beta[i ^ f1] + beta[i ^ f2] + beta[i ^ f1 ^ f2]))
        else:
            want.append((1 - 16 * p / 15) * b)
    assert np.abs(got - np.array(want)).max() < TOL


def test_depolarising_2q_definition():
    """(1 - 16p/15) rho + p/15 sum over all 16 Pauli pairs of s rho s."""
    rng = rng_for(14)
    N, t, p = 3, [1, 2], 0.4
    rho = rand_dm(rng, N)
    want = (1 - 16 * p / 15) * rho
    for a in range(4):
        for b in range(4):
            S = D.pauli_operator(N, t, [b, a])
            want = want + (p / 15) * S @ rho @ S.conj().T
    got = oracle.dm_apply_kraus(D.choi(rho), t, synth.kraus_depolarising_2q(p))
    assert np.abs(got - D.choi(want)).max() < TOL


def test_damping_rule():
    """Eq. damping_amps_update."""
    rng = rng_for(15)
    N, t, p = 3, 0, 0.31
    beta = D.choi(rand_dm(rng, N))
    got = oracle.dm_apply_kraus(beta.copy(), [t], synth.kraus_damping_1q(p))
    flip = (1 << t) | (1 << (t + N))
    want = []
    for i, b in enumerate(beta):
        lo, hi = _choi_bit(i, t), _choi_bit(i, t + N)
        if lo == hi == 0:
            want.append(b + p * beta[i ^ flip])
        elif lo != hi:
            want.append(np.sqrt(1 - p) * b)
        else:
            want.append((1 - p) * b)
    assert np.abs(got - np.array(want)).max() < TOL


def test_channel_special_cases():
    rng = rng_for(16)
    N = 3
    psi = rand_state(rng, N)
    rho = np.outer(psi, psi.conj())
    # 1-qubit depolarising at p = 3/4 leaves the target maximally mixed
    out = D.unchoi(oracle.dm_apply_kraus(D.choi(rho), [1], synth.kraus_depolarising_1q(0.75)))
    red = D.partial_trace(N, out, [0, 2])
    assert np.abs(red - np.eye(2) / 2).max() < TOL
    # 2-qubit depolarising at p = 15/16 leaves the pair maximally mixed
    out = D.unchoi(oracle.dm_apply_kraus(D.choi(rho), [0, 2], synth.kraus_depolarising_2q(15 / 16)))
    red = D.partial_trace(N, out, [1])
    assert np.abs(red - np.eye(4) / 4).max() < TOL
    # damping at p = 1 resets the qubit to |0>
    out = D.unchoi(oracle.dm_apply_kraus(D.choi(rho), [2], synth.kraus_damping_1q(1.0)))
    red = D.partial_trace(N, out, [0, 1])
    assert np.abs(red - np.diag([1, 0])).max() < TOL


def test_channels_keep_density_matrix_physical():
    rng = rng_for(17)
    N = 4
    beta = D.choi(rand_dm(rng, N))
    for k in range(30):
        kind = k % 4
        if kind == 0:
            t = [int(rng.integers(0, N))]
            oracle.dm_apply_kraus(beta, t, synth.kraus_depolarising_1q(rng.uniform(0, 0.5)))
        elif kind == 1:
            oracle.dm_apply_kraus(beta, [int(rng.integers(0, N))], synth.kraus_damping_1q(rng.uniform(0, 1)))
        elif kind == 2:
            t = [int(x) for x in rng.permutation(N)[:2]]
            oracle.dm_apply_kraus(beta, t, synth.kraus_random_isometry(rng, 2, 4))
        else:
            t = [int(x) for x in rng.permutation(N)[:2]]
            oracle.dm_apply_gate(beta, [], t, synth.haar_unitary(rng, 4))
    rho = D.unchoi(beta)
    assert abs(oracle.dm_trace(beta) - 1) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-12
    assert np.linalg.eigvalsh(rho).min() > -1e-12


def test_random_isometry_kraus_is_cptp():
    rng = rng_for(18)
    ks = synth.kraus_random_isometry(rng, 2, 4)
    assert np.abs(sum(k.conj().T @ k for k in ks) - np.eye(4)).max() < 1e-12


# ---- partial trace ----------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_partial_trace_matches_einsum(seed):
    rng = rng_for(500 + seed)
    N = int(rng.integers(2, 7))
    n = int(rng.integers(1, N))
    t = [int(x) for x in rng.permutation(N)[:n]]
    rho = synth.random_matrix(rng, 1 << N)          # no Hermiticity assumed
    got = oracle.partial_trace(D.choi(rho), t)
    want = D.choi(D.partial_trace(N, rho, t))
    assert np.abs(got - want).max() < TOL


def test_partial_trace_of_product_and_ghz():
    rng = rng_for(19)
    a, b = rand_dm(rng, 2), rand_dm(rng, 3)
    b = b * 1.7                                     # Tr rho_B = 1.7
    rho = np.kron(b, a)                             # A on qubits 0-1, B on qubits 2-4
    got = D.unchoi(oracle.partial_trace(D.choi(rho), [2, 3, 4]))
    assert np.abs(got - a * np.trace(b)).max() < TOL
    N = 5
    ghz = np.zeros(1 << N, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    red = D.unchoi(oracle.partial_trace(oracle.pure_dm(ghz), [0, 1, 3, 4]))
    assert np.abs(red - np.eye(2) / 2).max() < TOL
    rho = rand_dm(rng, 4)
    assert abs(oracle.dm_trace(oracle.partial_trace(D.choi(rho), [1, 2])) - 1) < TOL


# ---- expectation values, probabilities, purity --------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_expectation_matches_dense(seed):
    rng = rng_for(600 + seed)
    N = int(rng.integers(1, 7))
    codes, coeffs = synth.random_pauli_sum(rng, N, 5)
    H = D.hamiltonian(N, codes, coeffs)
    psi = rand_state(rng, N)
    assert abs(oracle.sv_expec_pauli_sum(psi, codes, coeffs) - psi.conj() @ H @ psi) < 1e-12
    rho = synth.random_matrix(rng, 1 << N)           # general matrix: complex result
    assert abs(oracle.dm_expec_pauli_sum(D.choi(rho), codes, coeffs) - np.trace(H @ rho)) < 1e-11
    # statevector and its density matrix agree
    pure = oracle.pure_dm(psi)
    assert abs(oracle.dm_expec_pauli_sum(pure, codes, coeffs) - oracle.sv_expec_pauli_sum(psi, codes, coeffs)) < 1e-12


def test_expectation_closed_forms():
    N = 6
    ghz = np.zeros(1 << N, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    zz = np.zeros((1, N), np.int32)
    zz[0, 0] = zz[0, N - 1] = 3
    assert abs(oracle.sv_expec_pauli_sum(ghz, zz, [1.0]) - 1) < TOL
    xs = np.ones((1, N), np.int32)
    assert abs(oracle.sv_expec_pauli_sum(oracle.plus_state(N), xs, [1.0]) - 1) < TOL
    assert abs(oracle.dm_expec_pauli_sum(oracle.plus_state(N, density=True), xs, [1.0]) - 1) < TOL


def test_probabilities():
    N = 5
    ghz = np.zeros(1 << N, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    for q in range(N):
        assert abs(oracle.sv_prob_of_outcome(ghz, q, 0) - 0.5) < TOL
    rng = rng_for(20)
    psi = synth.random_state(rng, 1 << N, normalise=False)
    nrm = np.sum(np.abs(psi) ** 2)
    for q in range(N):
        p0, p1 = oracle.sv_prob_of_outcome(psi, q, 0), oracle.sv_prob_of_outcome(psi, q, 1)
        assert abs(p0 + p1 - nrm) < 1e-12
        assert abs(p0 - sum(abs(psi[i]) ** 2 for i in range(1 << N) if not (i >> q) & 1)) < 1e-12
    rho = rand_dm(rng, N)
    for q in range(N):
        want = sum(rho[k, k].real for k in range(1 << N) if (k >> q) & 1)
        assert abs(oracle.dm_prob_of_outcome(D.choi(rho), q, 1) - want) < TOL


def test_purity():
    rng = rng_for(21)
    N = 4
    assert abs(oracle.dm_purity(oracle.pure_dm(rand_state(rng, N))) - 1) < TOL
    mixed = D.choi(np.eye(1 << N) / (1 << N))
    assert abs(oracle.dm_purity(mixed) - 1 / (1 << N)) < TOL
    rho = synth.random_matrix(rng, 1 << N)
    assert abs(oracle.dm_purity(D.choi(rho)) - np.trace(rho @ rho)) < 1e-10
    h = rand_dm(rng, N)
    assert abs(oracle.dm_purity(D.choi(h)) - np.sum(np.abs(h) ** 2)) < TOL


# ---- initial states -------------------------------------------------------------------

def test_initial_states():
    N = 3
    plus = oracle.plus_state(N)
    assert np.abs(oracle.plus_state(N, density=True) - oracle.pure_dm(plus)).max() < TOL
    assert np.abs(oracle.plus_state(N, density=True) - 1 / (1 << N)).max() < TOL
    b = oracle.basis_state(N, 5, density=True)
    assert b[5 * ((1 << N) + 1)] == 1 and np.count_nonzero(b) == 1
    rng = rng_for(22)
    psi = rand_state(rng, N)
    assert np.abs(D.unchoi(oracle.pure_dm(psi)) - np.outer(psi, psi.conj())).max() < TOL


def test_hashed_state():
    L, seed = 9, 77
    full = oracle.hashed_state(L, seed)
    e = (L + 1) // 2
    assert np.all(np.abs(full.real) <= 2.0 ** -e) and np.all(np.abs(full.imag) <= 2.0 ** -e)
    part = oracle.hashed_state(L, seed, start=100, count=50)
    assert np.array_equal(part, full[100:150])
    idx = [0, 3, 511, 260]
    assert np.array_equal(oracle.hashed_amps_at(L, seed, idx), full[idx])
    # value pinned to the published generator: entry 0 uses outputs 0 and 1 of the stream
    u = lambda x: 2.0 * ((x >> 11) * 2.0 ** -53) - 1.0
    assert full[0].real == u(oracle.splitmix64_at(seed, 0)) * 2.0 ** -e


# ---- gradient oracle ---------------------------------------------------------------------

def test_param_shift_gradient_closed_form_and_fd():
    # RY(a)|0>: <Z> = cos a, so dE/da = -sin a
    a = 0.813
    ops = synth.circuits.hea_circuit(1, np.array([a, 0.0]), num_layers=1)
    g = oracle.param_shift_gradient(1, ops, np.array([[3]]), [1.0], 2)
    assert abs(g[0] + np.sin(a)) < 1e-12 and abs(g[1]) < 1e-12
    rng = rng_for(23)
    N, L = 3, 2
    ang = rng.uniform(0, 2 * np.pi, size=2 * N * L)
    codes, coeffs = synth.random_pauli_sum(rng, N, 4)
    ops = synth.circuits.hea_circuit(N, ang, L)
    g = oracle.param_shift_gradient(N, ops, codes, coeffs, ang.size)

    def energy(x):
        psi = oracle.run_ops(oracle.zero_state(N), synth.circuits.hea_circuit(N, x, L))
        return oracle.sv_expec_pauli_sum(psi, codes, coeffs).real

    h = 1e-5
    fd = np.array([(energy(ang + h * e) - energy(ang - h * e)) / (2 * h) for e in np.eye(ang.size)])
    assert np.abs(g - fd).max() < 1e-8


# ---- SWAP, Pauli tensor, phase gadget (statevector and density matrix) ------------

SWAP4 = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)


@pytest.mark.parametrize("seed", range(6))
def test_swap_matches_dense_and_cnot_decomposition(seed):
    rng = rng_for(700 + seed)
    N = int(rng.integers(2, 8))
    t1, t2 = (int(x) for x in rng.permutation(N)[:2])
    psi = rand_state(rng, N)
    want = D.embed(N, [t1, t2], SWAP4) @ psi
    X = D.PAULIS[1]
    cnots = D.gate_operator(N, [t1], [t2], X) @ D.gate_operator(N, [t2], [t1], X) @ D.gate_operator(N, [t1], [t2], X)
    assert np.abs(cnots @ psi - want).max() < TOL
    got = oracle.apply_swap(psi.copy(), t1, t2)
    assert np.abs(got - want).max() < TOL
    # a basis state moves to the index with bits t1 and t2 exchanged
    i = int(rng.integers(0, 1 << N))
    j = i & ~((1 << t1) | (1 << t2))
    j |= ((i >> t1) & 1) << t2 | ((i >> t2) & 1) << t1
    e = np.zeros(1 << N, dtype=complex)
    e[i] = 1
    moved = oracle.apply_swap(e, t1, t2)
    assert moved[j] == 1 and np.count_nonzero(moved) == 1


@pytest.mark.parametrize("seed", range(8))
def test_pauli_tensor_matches_dense(seed):
    rng = rng_for(720 + seed)
    N = int(rng.integers(1, 8))
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(0, 4, size=w)]
    psi = rand_state(rng, N)
    want = D.pauli_operator(N, t, p) @ psi
    got = oracle.apply_pauli_tensor(psi.copy(), t, p)
    assert np.abs(got - want).max() < TOL
    # a Pauli string squares to the identity
    assert np.abs(oracle.apply_pauli_tensor(got, t, p) - psi).max() < TOL


@pytest.mark.parametrize("seed", range(6))
def test_phase_gadget_matches_expm(seed):
    rng = rng_for(740 + seed)
    N = int(rng.integers(1, 8))
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    theta = rng.uniform(-7, 7)
    psi = rand_state(rng, N)
    want = D.gadget_operator(N, t, [3] * w, theta) @ psi
    got = oracle.apply_phase_gadget(psi.copy(), t, theta)
    assert np.abs(got - want).max() < TOL


@pytest.mark.parametrize("seed", range(6))
def test_dm_special_unitaries_match_dense(seed):
    """Pins conj(SWAP) = SWAP, conj(P) = (-1)^m P and
    conj(exp(i theta Z..Z)) = exp(-i theta Z..Z) on the Choi vector."""
    rng = rng_for(760 + seed)
    N = int(rng.integers(2, 6))
    rho = rand_dm(rng, N)
    t1, t2 = (int(x) for x in rng.permutation(N)[:2])
    S = D.embed(N, [t1, t2], SWAP4)
    assert np.abs(oracle.dm_apply_swap(D.choi(rho), t1, t2) - D.choi(S @ rho @ S.conj().T)).max() < TOL
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(1, 4, size=w)]
    p[0] = 2                                         # at least one Y: the sign matters
    P = D.pauli_operator(N, t, p)
    assert np.abs(oracle.dm_apply_pauli_tensor(D.choi(rho), t, p) - D.choi(P @ rho @ P.conj().T)).max() < TOL
    theta = rng.uniform(-4, 4)
    G = D.gadget_operator(N, t, [3] * w, theta)
    assert np.abs(oracle.dm_apply_phase_gadget(D.choi(rho), t, theta) - D.choi(G @ rho @ G.conj().T)).max() < TOL


# ---- argument checks --------------------------------------------------------------------

def test_oracle_rejects_bad_arguments():
    psi = oracle.zero_state(3)
    x = synth.pauli_matrix_2x2(1)
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, [0], [0], x)                 # control is a target
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, [], [3], x)                  # out of range
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, [], [1, 1], np.eye(4))       # duplicate target
    with pytest.raises(ValueError):
        oracle.apply_pauli_gadget(psi, [0], [4], 0.1)        # bad Pauli code
    with pytest.raises(ValueError):
        oracle.partial_trace(oracle.zero_state(2, density=True), [0, 1])   # nothing left
    with pytest.raises(ValueError):
        oracle.apply_swap(psi, 1, 1)                         # same qubit twice
    with pytest.raises(ValueError):
        oracle.apply_pauli_tensor(psi, [0, 1], [1, 5])       # bad Pauli code
    with pytest.raises(ValueError):
        oracle.dm_apply_phase_gadget(oracle.zero_state(2, density=True), [2], 0.1)   # qubit 2 of 2
