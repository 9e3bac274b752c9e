"""Brute-force unitary of a tiny circuit by Kronecker products (tests only).

Independent of the oracle's C code: every layer is built as a dense
2^n x 2^n matrix with numpy.kron (qubit 0 is the most significant factor)
and the layers are multiplied together, U = L_d E_d ... E_1 L_0.
"""
import numpy as np

CZ4 = np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)


def _kron_all(mats):
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(out, m)
    return out


def _two_qubit_full(n, q, g4):
    if q == n - 1:
        return _wrap_full(n, g4)
    left = np.eye(1 << q, dtype=np.complex128)
    right = np.eye(1 << (n - q - 2), dtype=np.complex128)
    return np.kron(np.kron(left, g4), right)


def _wrap_full(n, g4):
    # the ring's wrap pair (n-1, 0): a permutation that brings qubit n-1 to
    # the front, the gate on the first two qubits, and the permutation back
    dim = 1 << n
    perm = np.zeros((dim, dim))
    for i in range(dim):
        bits = [(i >> (n - 1 - j)) & 1 for j in range(n)]
        moved = [bits[n - 1]] + bits[: n - 1]  # new order: q_{n-1}, q_0, ..., q_{n-2}
        perm[sum(b << (n - 1 - j) for j, b in enumerate(moved)), i] = 1.0
    inner = np.kron(g4, np.eye(dim >> 2, dtype=np.complex128))
    return perm.T @ inner @ perm


def unitary(circ):
    n, d = circ.n, circ.d
    assert n <= 7, "brute force only for tiny n"
    U = _kron_all([circ.one_qubit[0, q] for q in range(n)])
    for layer in range(1, d + 1):
        for (l, q, kind, m) in circ.gates:
            if l != layer:
                continue
            g4 = CZ4 if kind == 0 else m
            U = _two_qubit_full(n, q, g4) @ U
        U = _kron_all([circ.one_qubit[layer, q] for q in range(n)]) @ U
    return U


def all_amplitudes(circ):
    """<x|U|0^n> for all x, index x read MSB-first (qubit 0 first)."""
    return unitary(circ)[:, 0].copy()
