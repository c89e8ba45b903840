"""Brute-force dense references used only to pin the oracle (n <= 8).

Everything here is written independently of ``oracle.c``: operators are built
as explicit 2^n x 2^n matrices from Kronecker products and a qubit
permutation, and Pauli words as Kronecker products of 2x2 Pauli matrices.
Wire 0 is the most significant index bit (paper Alg. 1).
"""
import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}
P0 = np.diag([1, 0]).astype(complex)
P1 = np.diag([0, 1]).astype(complex)


def kron(*ms):
    out = np.eye(1, dtype=complex)
    for m in ms:
        out = np.kron(out, m)
    return out


def controlled(v, n_ctrls, ctrl_values=None):
    """Block matrix that applies v when the leading control qubits hold
    ctrl_values (tuple of bits, control 0 first) and identity otherwise."""
    if ctrl_values is None:
        ctrl_values = (1,) * n_ctrls
    dv = v.shape[0]
    out = np.zeros((dv << n_ctrls, dv << n_ctrls), dtype=complex)
    for c in range(1 << n_ctrls):
        bits = tuple((c >> (n_ctrls - 1 - j)) & 1 for j in range(n_ctrls))
        blk = v if bits == tuple(ctrl_values) else np.eye(dv)
        out[c * dv:(c + 1) * dv, c * dv:(c + 1) * dv] = blk
    return out


def permutation_matrix(n, order):
    """Matrix P with P |b_0 .. b_{n-1}> = |b_order[0] .. b_order[n-1]>."""
    N = 1 << n
    P = np.zeros((N, N))
    for i in range(N):
        bits = [(i >> (n - 1 - w)) & 1 for w in range(n)]
        j = 0
        for w in order:
            j = (j << 1) | bits[w]
        P[j, i] = 1
    return P


def embed(m, wires, n):
    """Dense 2^n x 2^n operator of the small matrix m acting on wires
    (first listed wire = most significant bit of m's index)."""
    k = len(wires)
    rest = [w for w in range(n) if w not in wires]
    order = list(wires) + rest
    P = permutation_matrix(n, order)
    big = np.kron(m, np.eye(1 << (n - k)))
    return P.T @ big @ P


def pauli_word_matrix(word):
    return kron(*[PAULI[c] for c in word])


def pauli_sum_matrix(obs):
    return sum(c * pauli_word_matrix(w) for c, w in zip(obs.coeffs, obs.words))


def expm(a):
    return scipy.linalg.expm(a)
