"""Brute-force dense checker for the oracle (test infrastructure, N <= 10).

Every operator is built as a full 2^N x 2^N matrix out of Kronecker products
and an axis permutation, never from the oracle's index arithmetic, so the
two can disagree when either is wrong.  Density matrices are 2^N x 2^N
NumPy arrays; ``choi(rho)`` stacks columns (entry k + l*2^N = rho[k, l]).
"""
import numpy as np
import scipy.linalg

PAULIS = [np.eye(2, dtype=complex),
          np.array([[0, 1], [1, 0]], dtype=complex),
          np.array([[0, -1j], [1j, 0]], dtype=complex),
          np.array([[1, 0], [0, -1]], dtype=complex)]


def embed(N, qubits, local):
    """Full operator acting as ``local`` on ``qubits`` (bit q of the local
    index <-> qubits[q]) and as identity elsewhere.

    Built as kron(I_rest, local) on the ordering [rest..., qubits reversed]
    (most significant first), then the tensor axes are permuted back to
    qubit order N-1..0."""
    qubits = list(qubits)
    k = len(qubits)
    rest = [q for q in range(N - 1, -1, -1) if q not in qubits]
    order = rest + qubits[::-1]          # qubit held by each tensor axis, MSB first
    big = np.kron(np.eye(1 << (N - k)), local).reshape([2] * (2 * N))
    # axis a (a < N) of the row index holds qubit order[a]; we want axis a to hold qubit N-1-a
    pos = {q: a for a, q in enumerate(order)}
    perm_rows = [pos[N - 1 - a] for a in range(N)]
    perm = perm_rows + [N + p for p in perm_rows]
    return big.transpose(perm).reshape(1 << N, 1 << N)


def controlled(ctrls, targs, M):
    """Local matrix on (targs..., ctrls...) of the controlled gate
    1 + |1><1|^{(x)s} (x) (M - 1), controls in the high bits."""
    s = len(ctrls)
    d = 1 << len(targs)
    proj = np.zeros((1 << s, 1 << s), dtype=complex)
    proj[-1, -1] = 1.0
    return np.eye(d << s, dtype=complex) + np.kron(proj, np.asarray(M, dtype=complex) - np.eye(d))


def gate_operator(N, ctrls, targs, M):
    return embed(N, list(targs) + list(ctrls), controlled(ctrls, targs, M))


def pauli_operator(N, targs, paulis):
    local = np.array([[1.0 + 0j]])
    for code in paulis[::-1]:            # last target is the most significant local bit
        local = np.kron(local, PAULIS[code])
    return embed(N, list(targs), local)


def pauli_string(N, codes):
    """codes[q] is the Pauli on qubit q."""
    return pauli_operator(N, list(range(N)), list(codes))


def gadget_operator(N, targs, paulis, theta):
    """exp(i theta P) by the matrix exponential."""
    return scipy.linalg.expm(1j * theta * pauli_operator(N, targs, paulis))


def hamiltonian(N, codes, coeffs):
    H = np.zeros((1 << N, 1 << N), dtype=complex)
    for c, h in zip(np.asarray(codes).reshape(-1, N), coeffs):
        H += h * pauli_string(N, c)
    return H


def choi(rho):
    return np.asarray(rho, dtype=np.complex128).flatten(order="F").copy()


def unchoi(vec):
    d = int(round(np.sqrt(vec.size)))
    return np.asarray(vec).reshape(d, d, order="F")


def kraus_apply(N, rho, targs, kraus):
    out = np.zeros_like(rho)
    for K in kraus:
        F = embed(N, list(targs), K)
        out += F @ rho @ F.conj().T
    return out


def partial_trace(N, rho, traced):
    """Trace out ``traced`` by reshaping into 2N tensor axes and summing the
    matching row/column axis pairs (einsum), keeping the other qubits in
    their relative order."""
    t = np.asarray(rho).reshape([2] * (2 * N))
    axis_of = lambda q: N - 1 - q                      # row axis of qubit q
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    rows = [letters[a] for a in range(N)]
    cols = [letters[N + a] for a in range(N)]
    for q in traced:
        cols[axis_of(q)] = rows[axis_of(q)]
    keep = [a for a in range(N) if (N - 1 - a) not in traced]
    out = "".join(rows[a] for a in keep) + "".join(cols[a] for a in keep)
    m = N - len(traced)
    return np.einsum("".join(rows) + "".join(cols) + "->" + out, t).reshape(1 << m, 1 << m)
