"""Seeded random circuits, matrices and Pauli sums (NumPy PCG64).

Conventions shared by every consumer of these inputs:

* qubit 0 is the least significant bit of an amplitude index;
* a gate on targets ``t`` with matrix ``M`` maps matrix index bit ``q`` to
  qubit ``t[q]`` (the first target is the least significant bit of the
  matrix row/column index), ``M`` is row-major, controls condition on |1>;
* Pauli codes are 0=I, 1=X, 2=Y, 3=Z;
* a Pauli gadget with angle ``theta`` is exp(+i*theta*P);
* depolarising probability ``p`` is the total error probability (p/3 per
  Pauli), damping ``p`` is the decay probability.

An op is a plain dict:

* ``{"op": "unitary", "ctrls": (...), "targs": (...), "matrix": ndarray}``
* ``{"op": "gadget", "targs": (...), "paulis": (...), "theta": float}``
  (optionally ``"param"``: index of the circuit parameter it carries and
  ``"scale"``: d theta / d parameter)
* ``{"op": "kraus", "targs": (...), "kraus": ndarray of shape (M, d, d)}``

Nothing here applies an op to a state.
"""
import numpy as np

PAULI_I, PAULI_X, PAULI_Y, PAULI_Z = 0, 1, 2, 3

# Fixed seeds of the five synthetic workloads.
CONFIG_SEEDS = {1: 20231101, 2: 20231102, 3: 20231103, 4: 20231104, 5: 20231105}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def haar_unitary(rng, d):
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal absorbed (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[np.newaxis, :]


def haar_isometry(rng, rows, cols):
    """Haar-random isometry V (rows x cols, V^dagger V = 1) from the QR of a
    rows x cols complex Ginibre matrix, phases absorbed as above."""
    z = (rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[np.newaxis, :]


def random_matrix(rng, d):
    """General (non-unitary) complex matrix with N(0,1) parts."""
    return rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))


def random_state(rng, num_amps, normalise=True):
    v = rng.standard_normal(num_amps) + 1j * rng.standard_normal(num_amps)
    if normalise:
        v /= np.linalg.norm(v)
    return v


def pauli_matrix_2x2(code):
    return [np.eye(2, dtype=complex),
            np.array([[0, 1], [1, 0]], dtype=complex),
            np.array([[0, -1j], [1j, 0]], dtype=complex),
            np.array([[1, 0], [0, -1]], dtype=complex)][code]


def rotation_y(theta):
    """RY(theta) = exp(-i theta Y / 2)."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=complex)


def rotation_z(theta):
    """RZ(theta) = exp(-i theta Z / 2)."""
    return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]], dtype=complex)


# ---- Kraus lists of the standard channels (inputs to a Kraus map) ----------

def kraus_dephasing_1q(p):
    return np.stack([np.sqrt(1 - p) * pauli_matrix_2x2(0), np.sqrt(p) * pauli_matrix_2x2(3)])


def kraus_dephasing_2q(p):
    """Z on the first, the second or both targets, each with weight p/3;
    matrix index bit 0 is the first target."""
    z, i2 = pauli_matrix_2x2(3), pauli_matrix_2x2(0)
    return np.stack([np.sqrt(1 - p) * np.kron(i2, i2), np.sqrt(p / 3) * np.kron(i2, z),
                     np.sqrt(p / 3) * np.kron(z, i2), np.sqrt(p / 3) * np.kron(z, z)])


def kraus_depolarising_1q(p):
    ks = [np.sqrt(1 - p) * pauli_matrix_2x2(0)]
    ks += [np.sqrt(p / 3) * pauli_matrix_2x2(c) for c in (1, 2, 3)]
    return np.stack(ks)


def kraus_depolarising_2q(p):
    """Two-qubit uniform depolarising: identity with weight 1-p, each of the
    15 non-identity Pauli pairs with weight p/15.  Matrix index bit 0 is the
    first target."""
    ks = []
    for a in range(4):          # Pauli on the second target (high bit)
        for b in range(4):      # Pauli on the first target (low bit)
            w = (1 - p) if (a == 0 and b == 0) else p / 15
            ks.append(np.sqrt(w) * np.kron(pauli_matrix_2x2(a), pauli_matrix_2x2(b)))
    return np.stack(ks)


def kraus_damping_1q(p):
    k1 = np.array([[1, 0], [0, np.sqrt(1 - p)]], dtype=complex)
    k2 = np.array([[0, np.sqrt(p)], [0, 0]], dtype=complex)
    return np.stack([k1, k2])


def kraus_random_isometry(rng, nq=2, num_ops=4):
    """num_ops Kraus operators on nq qubits cut from a Haar isometry of shape
    (num_ops * 2^nq) x 2^nq: K_m = V[m*d:(m+1)*d, :]."""
    d = 1 << nq
    v = haar_isometry(rng, num_ops * d, d)
    return np.stack([v[m * d:(m + 1) * d, :] for m in range(num_ops)])


# ---- Pauli sums --------------------------------------------------------------

def random_pauli_sum(rng, num_qubits, num_terms):
    """Per qubit uniform over {I,X,Y,Z}; coefficients ~ N(0,1).
    Returns (codes [T, N] int32, coeffs [T] float64)."""
    codes = rng.integers(0, 4, size=(num_terms, num_qubits)).astype(np.int32)
    coeffs = rng.standard_normal(num_terms)
    return codes, coeffs


# ---- op helpers --------------------------------------------------------------

def _unitary(ctrls, targs, m):
    return {"op": "unitary", "ctrls": tuple(int(c) for c in ctrls),
            "targs": tuple(int(t) for t in targs), "matrix": np.asarray(m, dtype=complex)}


def _gadget(targs, paulis, theta, **extra):
    d = {"op": "gadget", "targs": tuple(int(t) for t in targs),
         "paulis": tuple(int(p) for p in paulis), "theta": float(theta)}
    d.update(extra)
    return d


def _kraus(targs, ks):
    return {"op": "kraus", "targs": tuple(int(t) for t in targs), "kraus": np.asarray(ks, dtype=complex)}


def op_qubits(op):
    if op["op"] == "unitary":
        return set(op["ctrls"]) | set(op["targs"])
    return set(op["targs"])


def _random_gadget(rng, n, wmin, wmax):
    w = int(rng.integers(wmin, wmax + 1))
    targs = rng.choice(n, size=w, replace=False)
    paulis = rng.integers(1, 4, size=w)
    theta = rng.uniform(0, 2 * np.pi)
    return _gadget(targs, paulis, theta)


# ---- the five workloads ----------------------------------------------------------

def config1_circuit(seed=None, num_qubits=12, num_gates=200):
    """Alternating Haar 1-qubit gate on a uniform target and CNOT/CZ (prob 1/2
    each) on a random ordered pair of distinct qubits, from |0..0>."""
    rng = _rng(CONFIG_SEEDS[1] if seed is None else seed)
    ops = []
    x = pauli_matrix_2x2(1)
    z = pauli_matrix_2x2(3)
    for g in range(num_gates):
        if g % 2 == 0:
            t = int(rng.integers(0, num_qubits))
            ops.append(_unitary((), (t,), haar_unitary(rng, 2)))
        else:
            c, t = rng.choice(num_qubits, size=2, replace=False)
            ops.append(_unitary((c,), (t,), x if rng.random() < 0.5 else z))
    return ops


def config2_circuit(seed=None, num_qubits=28, num_gates=500):
    """Each gate one of (prob 1/3 each): Haar 1-qubit; 2-target Haar U(4) with
    U{0..3} controls; Pauli gadget of weight U{1..N} with theta ~ U(0, 2pi)."""
    rng = _rng(CONFIG_SEEDS[2] if seed is None else seed)
    ops = []
    for _ in range(num_gates):
        kind = int(rng.integers(0, 3))
        if kind == 0:
            t = int(rng.integers(0, num_qubits))
            ops.append(_unitary((), (t,), haar_unitary(rng, 2)))
        elif kind == 1:
            s = int(rng.integers(0, 4))
            qs = rng.choice(num_qubits, size=2 + s, replace=False)
            ops.append(_unitary(qs[2:], qs[:2], haar_unitary(rng, 4)))
        else:
            ops.append(_random_gadget(rng, num_qubits, 1, num_qubits))
    return ops


def config3_circuit(seed=None, num_qubits=14, num_ops=300, num_traced=7):
    """Density-matrix workload: each op one of (prob 1/5 each) Haar 1-qubit,
    Haar 2-qubit, 1-qubit depolarising p~U(0,0.05), damping p~U(0,0.1),
    random 2-qubit Kraus map of 4 operators from a Haar 16x4 isometry.
    Returns (ops, traced_qubits)."""
    rng = _rng(CONFIG_SEEDS[3] if seed is None else seed)
    ops = []
    for _ in range(num_ops):
        kind = int(rng.integers(0, 5))
        if kind == 0:
            t = int(rng.integers(0, num_qubits))
            ops.append(_unitary((), (t,), haar_unitary(rng, 2)))
        elif kind == 1:
            qs = rng.choice(num_qubits, size=2, replace=False)
            ops.append(_unitary((), qs, haar_unitary(rng, 4)))
        elif kind == 2:
            t = int(rng.integers(0, num_qubits))
            ops.append(_kraus((t,), kraus_depolarising_1q(rng.uniform(0, 0.05))))
        elif kind == 3:
            t = int(rng.integers(0, num_qubits))
            ops.append(_kraus((t,), kraus_damping_1q(rng.uniform(0, 0.1))))
        else:
            qs = rng.choice(num_qubits, size=2, replace=False)
            ops.append(_kraus(qs, kraus_random_isometry(rng, 2, 4)))
    traced = sorted(int(q) for q in rng.choice(num_qubits, size=num_traced, replace=False))
    return ops, traced


def hea_circuit(num_qubits, angles, num_layers=6):
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every
    qubit, then CZ(q, q+1) for q = 0..N-2.  RY(a) = exp(-i a Y/2) is the
    gadget exp(i*theta*Y) with theta = -a/2 (likewise RZ).  ``angles`` has
    2*N*num_layers entries, layer-major then (RY block, RZ block)."""
    z = pauli_matrix_2x2(3)
    ops = []
    k = 0
    for _ in range(num_layers):
        for code in (PAULI_Y, PAULI_Z):
            for q in range(num_qubits):
                ops.append(_gadget((q,), (code,), -0.5 * angles[k], param=k, scale=-0.5))
                k += 1
        for q in range(num_qubits - 1):
            ops.append(_unitary((q,), (q + 1,), z))
    return ops


def config4_batch(seed=None, num_circuits=512, nmin=10, nmax=22, num_layers=6, num_terms=20):
    """512 HEA circuits with N ~ U{10..22}; angles ~ U(0, 2pi); per circuit a
    20-term Pauli sum (codes uniform, coefficients N(0,1)).  Returns a list of
    dicts {num_qubits, angles, ops, codes, coeffs}."""
    base = CONFIG_SEEDS[4] if seed is None else seed
    out = []
    for c in range(num_circuits):
        rng = _rng(base * 1000003 + c)
        n = int(rng.integers(nmin, nmax + 1))
        angles = rng.uniform(0, 2 * np.pi, size=2 * n * num_layers)
        codes, coeffs = random_pauli_sum(rng, n, num_terms)
        out.append({"num_qubits": n, "angles": angles, "ops": hea_circuit(n, angles, num_layers),
                    "codes": codes, "coeffs": coeffs, "num_layers": num_layers})
    return out


def config5_circuit(seed=None, num_qubits=34, num_gates=200):
    """Each gate one of (prob 1/2 each): 5-target Haar U(32) with U{0..4}
    controls; Pauli gadget of weight U{1..N}."""
    rng = _rng(CONFIG_SEEDS[5] if seed is None else seed)
    ops = []
    for _ in range(num_gates):
        if rng.random() < 0.5:
            s = int(rng.integers(0, 5))
            qs = rng.choice(num_qubits, size=5 + s, replace=False)
            ops.append(_unitary(qs[5:], qs[:5], haar_unitary(rng, 32)))
        else:
            ops.append(_random_gadget(rng, num_qubits, 1, num_qubits))
    return ops


def count_logical_updates(ops, num_qubits, density=False):
    """Amplitude-updates credited to a circuit under the plain per-gate method:
    2^(N-s) per s-controlled gate, 2^N per Pauli gadget; on a density matrix
    (Choi vector of 2N qubits) 2 * 2^(2N - s) per unitary (two passes, the
    second with the controls shifted by N) and 2^(2N) per Kraus map."""
    total = 0
    for op in ops:
        if op["op"] == "unitary":
            s = len(op["ctrls"])
            total += (2 << (2 * num_qubits - s)) if density else (1 << (num_qubits - s))
        elif op["op"] == "gadget":
            total += (2 << (2 * num_qubits)) if density else (1 << num_qubits)
        else:
            total += 1 << (2 * num_qubits)
    return total
