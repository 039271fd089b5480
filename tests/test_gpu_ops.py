"""Parity of every HIP operation with the FP64 oracle on the same seeded
inputs, element by element (normalised max-abs amplitude error), for
complex128 (tolerance 1e-12) and complex64 (1e-5)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, amp_err, banner, scalar_tol

pytestmark = pytest.mark.gpu

PRECS = ["c128", "c64"]


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def make(qs, n, prec, density=False, state=None):
    q = qs.Qureg(n, density=density, precision=prec)
    if state is not None:
        q.set_amps(state)
    return q


def rand_sv(rng, n):
    return synth.random_state(rng, 1 << n)


def rand_choi(rng, n, hermitian=True):
    d = 1 << n
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    rho = a @ a.conj().T if hermitian else a
    rho = rho / np.trace(rho) if hermitian else rho / d
    return np.asarray(rho, dtype=np.complex128).flatten(order="F").copy()


# ---- unitaries on statevectors --------------------------------------------------------

GATE_CASES = [
    # (N, num_targets, num_controls)
    (1, 1, 0), (2, 1, 1), (2, 2, 0), (3, 3, 0), (5, 1, 4), (7, 2, 3), (9, 3, 2), (10, 4, 0),
    (11, 5, 1), (12, 6, 0), (13, 6, 3), (14, 1, 0), (16, 2, 2), (17, 4, 4), (18, 5, 0), (20, 1, 1),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", range(len(GATE_CASES)))
def test_gate_parity(qs, prec, case):
    N, nt, ns = GATE_CASES[case]
    banner(f"gate N={N} nt={nt} ns={ns} {prec}")
    rng = np.random.default_rng(1000 + case)
    for rep in range(3):
        qsel = rng.permutation(N)[:nt + ns]
        t, c = [int(x) for x in qsel[:nt]], [int(x) for x in qsel[nt:]]
        M = synth.random_matrix(rng, 1 << nt) / np.sqrt(1 << nt)     # general, not unitary
        psi = rand_sv(rng, N)
        q = make(qs, N, prec, state=psi)
        q.apply_unitary(c, t, M)
        want = oracle.apply_gate(psi.copy(), c, t, M)
        assert amp_err(q.get_amps(), want) < TOL[prec], (t, c)


@pytest.mark.parametrize("prec", PRECS)
def test_low_and_high_targets(qs, prec):
    """Every target position of a 1- and 2-target gate at N = 12."""
    rng = np.random.default_rng(7)
    N = 12
    psi = rand_sv(rng, N)
    q = make(qs, N, prec, state=psi)
    want = psi.copy()
    for t in range(N):
        U = synth.haar_unitary(rng, 2)
        q.apply_unitary([], [t], U)
        oracle.apply_gate(want, [], [t], U)
        t2 = (t + 5) % N
        U = synth.haar_unitary(rng, 4)
        q.apply_unitary([], [t, t2], U)
        oracle.apply_gate(want, [], [t, t2], U)
    assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed", range(8))
def test_gadget_parity(qs, prec, seed):
    rng = np.random.default_rng(2000 + seed)
    N = int(rng.integers(1, 17))
    w = N if seed == 0 else int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(0 if seed % 2 else 1, 4, size=w)]
    if seed == 3:
        p = [3] * w                                   # phase gadget (diagonal)
    theta = rng.uniform(-7, 7)
    banner(f"gadget N={N} w={w} {prec}")
    psi = rand_sv(rng, N)
    q = make(qs, N, prec, state=psi)
    q.apply_pauli_gadget(t, p, theta)
    want = oracle.apply_pauli_gadget(psi.copy(), t, p, theta)
    assert amp_err(q.get_amps(), want) < TOL[prec]


# ---- density matrices ---------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nt,ns", [(1, 0), (2, 0), (1, 1), (2, 1), (3, 0), (1, 2), (3, 2)])
def test_dm_unitary_parity(qs, prec, nt, ns):
    rng = np.random.default_rng(3000 + 10 * nt + ns)
    N = 6
    qsel = rng.permutation(N)[:nt + ns]
    t, c = [int(x) for x in qsel[:nt]], [int(x) for x in qsel[nt:]]
    U = synth.haar_unitary(rng, 1 << nt)
    rho = rand_choi(rng, N)
    q = make(qs, N, prec, density=True, state=rho)
    q.apply_unitary(c, t, U)
    want = oracle.dm_apply_gate(rho.copy(), c, t, U)
    assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed", range(4))
def test_dm_gadget_parity(qs, prec, seed):
    rng = np.random.default_rng(3100 + seed)
    N = 5
    w = int(rng.integers(1, N + 1))
    t = [int(x) for x in rng.permutation(N)[:w]]
    p = [int(x) for x in rng.integers(1, 4, size=w)]
    theta = rng.uniform(-3, 3)
    rho = rand_choi(rng, N)
    q = make(qs, N, prec, density=True, state=rho)
    q.apply_pauli_gadget(t, p, theta)
    want = oracle.dm_apply_pauli_gadget(rho.copy(), t, p, theta)
    assert amp_err(q.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,nops", [(1, 1), (1, 4), (2, 4), (2, 16), (3, 2)])
def test_kraus_and_superop_parity(qs, prec, n, nops):
    rng = np.random.default_rng(3200 + 10 * n + nops)
    N = 6
    t = [int(x) for x in rng.permutation(N)[:n]]
    ks = np.stack([synth.random_matrix(rng, 1 << n) / (2 << n) for _ in range(nops)])
    rho = rand_choi(rng, N)
    q = make(qs, N, prec, density=True, state=rho)
    q.apply_kraus_map(t, ks)
    want = oracle.dm_apply_kraus(rho.copy(), t, ks)
    assert amp_err(q.get_amps(), want) < TOL[prec]
    S = oracle.build_superop(ks)
    q2 = make(qs, N, prec, density=True, state=rho)
    q2.apply_superop(t, S)
    assert amp_err(q2.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_standard_channels_parity(qs, prec):
    rng = np.random.default_rng(3300)
    N = 7
    rho = rand_choi(rng, N)
    q = make(qs, N, prec, density=True, state=rho)
    want = rho.copy()
    chans = [([2], synth.kraus_depolarising_1q(0.04)), ([6], synth.kraus_damping_1q(0.08)),
             ([0], synth.kraus_dephasing_1q(0.3)), ([1, 5], synth.kraus_depolarising_2q(0.2)),
             ([3, 4], synth.kraus_random_isometry(rng, 2, 4))]
    for t, ks in chans:
        q.apply_kraus_map(t, ks)
        oracle.dm_apply_kraus(want, t, ks)
    assert amp_err(q.get_amps(), want) < TOL[prec]


# ---- reductions and partial trace --------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N,n", [(2, 1), (3, 2), (5, 2), (7, 3), (8, 7), (9, 4)])
def test_partial_trace_parity(qs, prec, N, n):
    rng = np.random.default_rng(4000 + 10 * N + n)
    t = [int(x) for x in rng.permutation(N)[:n]]
    rho = rand_choi(rng, N, hermitian=False)
    q = make(qs, N, prec, density=True, state=rho)
    out = q.partial_trace(t)
    want = oracle.partial_trace(rho, t)
    assert amp_err(out.get_amps(), want) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [1, 4, 9, 15])
def test_sv_reductions_parity(qs, prec, N):
    rng = np.random.default_rng(5000 + N)
    psi = synth.random_state(rng, 1 << N, normalise=False)
    q = make(qs, N, prec, state=psi)
    nrm = oracle.sv_total_prob(psi)
    assert abs(q.total_prob() - nrm) < scalar_tol(prec, nrm)
    for qb in range(N):
        for b in (0, 1):
            w = oracle.sv_prob_of_outcome(psi, qb, b)
            assert abs(q.prob_of_outcome(qb, b) - w) < scalar_tol(prec, nrm)
    phi = synth.random_state(rng, 1 << N)
    q2 = make(qs, N, prec, state=phi)
    ip = np.vdot(psi, phi)
    assert abs(q.inner_product(q2) - ip) < scalar_tol(prec, np.sqrt(nrm))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N,T", [(1, 3), (3, 5), (6, 30), (10, 20), (13, 7)])
def test_sv_expectation_parity(qs, prec, N, T):
    rng = np.random.default_rng(5100 + N)
    codes, coeffs = synth.random_pauli_sum(rng, N, T)
    codes[0, :] = 0                                   # identity term
    if T > 2:
        codes[1, :] = rng.choice([0, 3], size=N)      # diagonal term
    if T >= 30:                                      # many terms sharing one flip mask
        codes[2:, :] = np.where(rng.random((T - 2, N)) < 0.5, 3, 0)
        codes[2:, 0] = 1
    psi = rand_sv(rng, N)
    q = make(qs, N, prec, state=psi)
    got = q.expec_pauli_sum(codes, coeffs)
    want = oracle.sv_expec_pauli_sum(psi, codes, coeffs)
    tol = scalar_tol(prec, np.abs(coeffs).sum())
    assert abs(got.real - want.real) < tol and abs(got.imag - want.imag) < tol


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N,T", [(1, 2), (3, 6), (5, 30)])
def test_dm_expectation_parity(qs, prec, N, T):
    rng = np.random.default_rng(5200 + N)
    codes, coeffs = synth.random_pauli_sum(rng, N, T)
    rho = rand_choi(rng, N, hermitian=False)
    q = make(qs, N, prec, density=True, state=rho)
    got = q.expec_pauli_sum(codes, coeffs)
    want = oracle.dm_expec_pauli_sum(rho, codes, coeffs)
    tol = scalar_tol(prec, np.abs(coeffs).sum())
    assert abs(got - want) < tol


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [1, 3, 5, 6, 7])
def test_dm_reductions_parity(qs, prec, N):
    rng = np.random.default_rng(5300 + N)
    rho = rand_choi(rng, N, hermitian=False)
    q = make(qs, N, prec, density=True, state=rho)
    tr = oracle.dm_trace(rho)
    assert abs(q.trace() - tr) < scalar_tol(prec)
    assert abs(q.total_prob() - tr.real) < scalar_tol(prec)
    pur = oracle.dm_purity(rho)
    assert abs(q.purity() - pur) < scalar_tol(prec, abs(pur))
    for qb in range(N):
        assert abs(q.prob_of_outcome(qb, 1) - oracle.dm_prob_of_outcome(rho, qb, 1)) < scalar_tol(prec)


# ---- initial states -------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
def test_initial_states(qs, prec):
    for N in (1, 4, 7):
        q = make(qs, N, prec)
        assert amp_err(q.init_zero().get_amps(), oracle.zero_state(N)) == 0
        assert amp_err(q.init_basis(3 % (1 << N)).get_amps(), oracle.basis_state(N, 3 % (1 << N))) == 0
        assert amp_err(q.init_plus().get_amps(), oracle.plus_state(N)) < TOL[prec]
        d = make(qs, N, prec, density=True)
        assert amp_err(d.init_zero().get_amps(), oracle.zero_state(N, True)) == 0
        assert amp_err(d.init_basis(1).get_amps(), oracle.basis_state(N, 1, True)) == 0
        assert amp_err(d.init_plus().get_amps(), oracle.plus_state(N, True)) < TOL[prec]
        rng = np.random.default_rng(N)
        psi = rand_sv(rng, N)
        q.set_amps(psi)
        assert amp_err(d.init_pure(q).get_amps(), oracle.pure_dm(psi)) < TOL[prec]


def test_hashed_state_bit_exact(qs):
    """The counter-based state is the same function on both sides: bit-exact
    in complex128, correctly rounded in complex64."""
    for bits, dens in ((9, False), (6, True)):
        N = bits // 2 if dens else bits
        q = make(qs, N, "c128", density=dens).init_hashed(12345)
        want = oracle.hashed_state(bits, 12345)
        assert np.array_equal(q.get_amps(), want)
        q = make(qs, N, "c64", density=dens).init_hashed(12345)
        assert np.array_equal(q.get_amps(), want.astype(np.complex64).astype(np.complex128))


# ---- argument errors raised from the GPU library -----------------------------------------

def test_argument_errors(qs):
    q = make(qs, 4, "c128").init_zero()
    x = synth.pauli_matrix_2x2(1)
    with pytest.raises(ValueError):
        q.apply_unitary([0], [0], x)
    with pytest.raises(ValueError):
        q.apply_unitary([], [4], x)
    with pytest.raises(ValueError):
        q.apply_unitary([], [1, 1], np.eye(4))
    with pytest.raises(ValueError):
        q.apply_unitary([], list(range(4)) + [], np.eye(16)[:8])      # wrong matrix size
    with pytest.raises(ValueError):
        q.apply_kraus_map([0], synth.kraus_damping_1q(0.1))           # needs a density matrix
    with pytest.raises(ValueError):
        q.apply_pauli_gadget([0], [5], 0.1)
    d = make(qs, 4, "c128", density=True).init_zero()
    with pytest.raises(ValueError):
        d.partial_trace([0, 1], out=make(qs, 3, "c128", density=True))   # wrong output size
    with pytest.raises(TypeError):
        d.partial_trace([0], out=make(qs, 3, "c64", density=True))
    with pytest.raises(MemoryError):
        qs.native.qs_create_qureg(40, False, qs.QS_C128)              # 2^40 amplitudes, library-owned
