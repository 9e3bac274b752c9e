"""Stabilizer-tableau (CHP) probabilities for T-free Clifford circuits.

Tests only.  Aaronson-Gottesman tableau with destabilizers in rows 0..n-1
and stabilizers in rows n..2n-1; gates H, S, CNOT (CZ = H_b CNOT_ab H_b).
The probability of a full bitstring is obtained by measuring qubits in
order with forced outcomes: a random outcome contributes 1/2, a
deterministic one 1 or 0.
"""
import numpy as np


class Tableau:
    def __init__(self, n):
        self.n = n
        self.x = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.z = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.r = np.zeros(2 * n + 1, dtype=np.uint8)
        for i in range(n):
            self.x[i, i] = 1
            self.z[n + i, i] = 1

    def copy(self):
        t = Tableau.__new__(Tableau)
        t.n, t.x, t.z, t.r = self.n, self.x.copy(), self.z.copy(), self.r.copy()
        return t

    def h(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        xa = self.x[:, a].copy()
        self.x[:, a] = self.z[:, a]
        self.z[:, a] = xa

    def s(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.z[:, a] ^= self.x[:, a]

    def cnot(self, a, b):
        self.r ^= self.x[:, a] & self.z[:, b] & (self.x[:, b] ^ self.z[:, a] ^ 1)
        self.x[:, b] ^= self.x[:, a]
        self.z[:, a] ^= self.z[:, b]

    def cz(self, a, b):
        self.h(b)
        self.cnot(a, b)
        self.h(b)

    @staticmethod
    def _g(x1, z1, x2, z2):
        x1 = x1.astype(np.int64); z1 = z1.astype(np.int64)
        x2 = x2.astype(np.int64); z2 = z2.astype(np.int64)
        return np.where((x1 == 1) & (z1 == 1), z2 - x2,
               np.where((x1 == 1) & (z1 == 0), z2 * (2 * x2 - 1),
               np.where((x1 == 0) & (z1 == 1), x2 * (1 - 2 * z2), 0)))

    def rowsum(self, h, i):
        s = 2 * int(self.r[h]) + 2 * int(self.r[i]) + int(
            self._g(self.x[i], self.z[i], self.x[h], self.z[h]).sum())
        self.r[h] = 1 if s % 4 == 2 else 0
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure_forced(self, a, outcome):
        """Measure qubit a, forcing ``outcome``; returns its probability."""
        n = self.n
        ps = [p for p in range(n, 2 * n) if self.x[p, a]]
        if ps:
            p = ps[0]
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self.rowsum(i, p)
            self.x[p - n] = self.x[p]
            self.z[p - n] = self.z[p]
            self.r[p - n] = self.r[p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            self.r[p] = outcome
            return 0.5
        sc = 2 * n
        self.x[sc] = 0
        self.z[sc] = 0
        self.r[sc] = 0
        for i in range(n):
            if self.x[i, a]:
                self.rowsum(sc, i + n)
        return 1.0 if int(self.r[sc]) == outcome else 0.0

    def prob(self, bits):
        t = self.copy()
        p = 1.0
        for a, o in enumerate(bits):
            p *= t.measure_forced(a, int(o))
            if p == 0.0:
                return 0.0
        return p

    def sample(self, rng):
        t = self.copy()
        out = []
        for a in range(self.n):
            o = int(rng.integers(0, 2))
            p = t.copy().measure_forced(a, o)
            if p == 0.0:
                o ^= 1
            t.measure_forced(a, o)
            out.append(o)
        return np.array(out, dtype=np.uint8)


def run_clifford(circ, words):
    """Tableau after a T-free circuit whose one-qubit gates are Clifford words."""
    assert circ.t_mask is None or not circ.t_mask.any()
    t = Tableau(circ.n)
    for layer in range(circ.d + 1):
        for q in range(circ.n):
            for g in words[int(circ.cliff[layer, q])]:
                (t.h if g == "H" else t.s)(q)
        if layer < circ.d:
            for (l, q, kind, _) in circ.gates:
                if l == layer + 1:
                    assert kind == 0
                    t.cz(q, q + 1)
    return t
