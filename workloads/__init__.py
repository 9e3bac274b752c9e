"""Seeded synthetic inputs for the temporal-boundary amplitude engine.

This module is shared by the CPU oracle and by the GPU path.  It builds
inputs only: circuits given as explicit gate matrices, output bitstrings and
request streams.  It contains none of the contraction arithmetic.

Circuit family (Sec. 2.1 of arXiv 2608.13110): ``n`` qubits on an open chain,
``d`` entangling layers of nearest-neighbour CZ gates whose pattern alternates
between the pairs (1,2),(3,4),... and (2,3),(4,5),... (1-based), d + 1
layers of one-qubit gates (one ahead of the first entangling layer, one
behind each), and T gates inserted at some (qubit, one-qubit-layer) sites.

Conventions (0-based everywhere):
  * qubit ``q`` is row ``q`` of the chain; gate ``(l, q)`` acts on ``(q, q+1)``.
  * one-qubit layer ``L_l`` (l = 0..d) acts after entangling layer ``l``
    (``L_0`` acts on |0^n> before layer 1).
  * layer 1 uses the pairs whose upper qubit ``q`` has parity ``first_parity``
    (default 1, i.e. the 1-based pattern (2,3),(4,5),... as printed first in
    the paper's pattern equation); later layers alternate.
  * a T gate at site (q, l) replaces ``L_l[q]`` by ``T @ L_l[q]``.
  * bitstring byte ``j`` is the output value of qubit ``j``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "GATE_CZ", "GATE_DENSE4", "Circuit", "clifford_table", "T_GATE",
    "brickwork_circuit", "restrict", "random_bitstrings", "rng_for",
    "config_circuit", "CONFIGS", "serving_requests", "random_rank2_gate",
    "random_unitary_2x2", "with_gate_values", "ring_circuit",
]

GATE_CZ = 0
GATE_DENSE4 = 1

T_GATE = np.array([[1.0, 0.0], [0.0, np.exp(1j * np.pi / 4)]], dtype=np.complex128)
_H = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)
_S = np.array([[1.0, 0.0], [0.0, 1j]], dtype=np.complex128)


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator seeded by an integer tuple, e.g. (config_id, seed)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _normalise_phase(m: np.ndarray) -> np.ndarray:
    flat = m.reshape(-1)
    for v in flat:
        if abs(v) > 1e-9:
            return m * (abs(v) / v)
    return m


_CLIFF_CACHE: Optional[Tuple[np.ndarray, List[str]]] = None


def clifford_table() -> Tuple[np.ndarray, List[str]]:
    """The 24 one-qubit Cliffords modulo global phase.

    Breadth-first search over words in {H, S} starting from the identity;
    each matrix is normalised so that its first nonzero entry (row-major) is
    real and positive, and duplicates are dropped.  Order = discovery order.
    Returns (matrices (24,2,2) complex128, words) where ``words[i]`` lists
    the gates in time order (``"HS"`` means H first, then S), so the matrix
    equals the product of the word up to a global phase.
    """
    global _CLIFF_CACHE
    if _CLIFF_CACHE is not None:
        return _CLIFF_CACHE[0].copy(), list(_CLIFF_CACHE[1])
    mats: List[np.ndarray] = []
    words: List[str] = []

    def key(m: np.ndarray) -> Tuple:
        r = np.round(m.reshape(-1), 9)
        return tuple((float(z.real) + 0.0, float(z.imag) + 0.0) for z in r)

    seen = {}
    start = np.eye(2, dtype=np.complex128)
    frontier = [(start, "")]
    seen[key(_normalise_phase(start))] = 0
    mats.append(_normalise_phase(start))
    words.append("")
    while frontier:
        nxt = []
        for m, w in frontier:
            for g, name in ((_H, "H"), (_S, "S")):
                m2 = g @ m
                k2 = key(_normalise_phase(m2))
                if k2 not in seen:
                    seen[k2] = len(mats)
                    mats.append(_normalise_phase(m2))
                    words.append(w + name)
                    nxt.append((m2, w + name))
        frontier = nxt
    arr = np.stack(mats)
    assert arr.shape == (24, 2, 2), arr.shape
    _CLIFF_CACHE = (arr, words)
    return arr.copy(), list(words)


@dataclasses.dataclass
class Circuit:
    """Explicit open-chain brickwork circuit.

    one_qubit: complex128 (d+1, n, 2, 2); ``one_qubit[l, q]`` is ``L_l`` on q,
               row-major [out][in].
    gates:     list of (layer, q, kind, matrix) with layer in 1..d acting on
               (q, q+1); ``matrix`` is a 4x4 complex128 for DENSE4 (basis
               index 2*x_q + x_{q+1}, row-major [out][in]) and None for CZ.
               On a ring, q = n-1 is the wrap pair (n-1, 0).
    cliff:     optional (d+1, n) Clifford indices used to build one_qubit.
    t_mask:    optional (d+1, n) bool, True where a T follows the Clifford.
    """

    n: int
    d: int
    one_qubit: np.ndarray
    gates: List[Tuple[int, int, int, Optional[np.ndarray]]]
    cliff: Optional[np.ndarray] = None
    t_mask: Optional[np.ndarray] = None
    first_parity: int = 1
    label: str = ""

    @property
    def width(self) -> int:
        return (self.d + 1) // 2

    def n_cz(self) -> int:
        return sum(1 for g in self.gates if g[2] == GATE_CZ)

    def n_t(self) -> int:
        return 0 if self.t_mask is None else int(self.t_mask.sum())

    def gate_arrays(self):
        """Flat arrays (layer, q, kind, mats(n_g,4,4)) for C entry points.

        ``mats`` is all-zero for CZ gates: consumers apply CZ by its kind.
        """
        ng = len(self.gates)
        layer = np.array([g[0] for g in self.gates], dtype=np.int32)
        q = np.array([g[1] for g in self.gates], dtype=np.int32)
        kind = np.array([g[2] for g in self.gates], dtype=np.int32)
        mats = np.zeros((ng, 4, 4), dtype=np.complex128)
        for i, g in enumerate(self.gates):
            if g[2] == GATE_DENSE4:
                mats[i] = g[3]
        return layer, q, kind, mats


def brickwork_pairs(n: int, layer: int, first_parity: int = 1) -> List[int]:
    """Upper qubits of the CZ pairs in entangling layer ``layer`` (1-based)."""
    par = (first_parity + layer - 1) % 2
    return [q for q in range(par, n - 1, 2)]


def brickwork_circuit(n: int, d: int, n_t: int, rng: np.random.Generator,
                      first_parity: int = 1, label: str = "") -> Circuit:
    """Doped-Clifford brickwork circuit with seeded uniform Clifford layers.

    Each of the (d+1)*n one-qubit sites gets a uniform draw from the 24
    Cliffords; ``n_t`` distinct sites are drawn uniformly without replacement
    and get a T applied after their Clifford.
    """
    if n < 2 or d < 1:
        raise ValueError("need n >= 2 and d >= 1")
    sites = (d + 1) * n
    if not 0 <= n_t <= sites:
        raise ValueError("n_t out of range")
    mats, _ = clifford_table()
    cliff = rng.integers(0, 24, size=(d + 1, n))
    t_flat = np.zeros(sites, dtype=bool)
    if n_t:
        t_flat[rng.choice(sites, size=n_t, replace=False)] = True
    t_mask = t_flat.reshape(d + 1, n)
    one = mats[cliff]
    one[t_mask] = np.einsum("ij,njk->nik", T_GATE, one[t_mask])
    gates = []
    for layer in range(1, d + 1):
        for q in brickwork_pairs(n, layer, first_parity):
            gates.append((layer, q, GATE_CZ, None))
    return Circuit(n=n, d=d, one_qubit=one, gates=gates, cliff=cliff,
                   t_mask=t_mask, first_parity=first_parity, label=label)


def ring_circuit(n: int, d: int, n_t: int, rng: np.random.Generator, label: str = "") -> Circuit:
    """Doped-Clifford brickwork circuit on a ring of even n >= 4: the
    open-chain pattern plus a CZ on the wrap pair (n-1, 0) in every layer
    whose pairs start at qubit 1 (the layers that leave qubits 0 and n-1
    free), d/2 of them for even d.  The wrap gate is listed with q = n-1."""
    if n < 4 or n % 2:
        raise ValueError("the ring needs an even n >= 4")
    c = brickwork_circuit(n, d, n_t, rng, first_parity=1, label=label)
    gates = list(c.gates)
    for layer in range(1, d + 1):
        if brickwork_pairs(n, layer, 1)[:1] == [1]:
            gates.append((layer, n - 1, GATE_CZ, None))
    return dataclasses.replace(c, gates=sorted(gates, key=lambda g: (g[0], g[1])))


def restrict(c: Circuit, n2: int) -> Circuit:
    """The same circuit on qubits 0..n2-1 with all layers kept.

    Gates touching a removed qubit are dropped (T gates on removed qubits go
    with their site).
    """
    if not 2 <= n2 <= c.n:
        raise ValueError("bad restriction size")
    gates = [g for g in c.gates if g[1] + 1 < n2]
    return Circuit(n=n2, d=c.d, one_qubit=c.one_qubit[:, :n2].copy(), gates=gates,
                   cliff=None if c.cliff is None else c.cliff[:, :n2].copy(),
                   t_mask=None if c.t_mask is None else c.t_mask[:, :n2].copy(),
                   first_parity=c.first_parity, label=f"{c.label}|q<{n2}")


def with_gate_values(c: Circuit, rng: np.random.Generator) -> Circuit:
    """Same topology, new uniformly random unitary one-qubit gates."""
    one = np.stack([[random_unitary_2x2(rng) for _ in range(c.n)] for _ in range(c.d + 1)])
    return dataclasses.replace(c, one_qubit=one, cliff=None, t_mask=None)


def random_bitstrings(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """(count, n) uint8 uniform output bitstrings."""
    return rng.integers(0, 2, size=(count, n), dtype=np.uint8)


def random_unitary_2x2(rng: np.random.Generator) -> np.ndarray:
    z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    qm, r = np.linalg.qr(z)
    return qm * (np.diag(r) / np.abs(np.diag(r)))


def random_unitary_4x4(rng: np.random.Generator) -> np.ndarray:
    """A Haar-random two-qubit unitary (QR of a complex Gaussian with the
    phases of R's diagonal divided out); operator Schmidt rank 4 with
    probability one."""
    z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    qm, r = np.linalg.qr(z)
    return qm * (np.diag(r) / np.abs(np.diag(r)))


def generic_brickwork_circuit(n: int, d: int, rng: np.random.Generator, first_parity: int = 1,
                              label: str = "") -> Circuit:
    """Open-chain brickwork in which every entangler is an independent
    Haar-random two-qubit unitary (bond dimension four) and every one-qubit
    site an independent Haar-random 2x2: the hardened circuit family of
    Sec. 6.2 (generic gates in place of CZ)."""
    if n < 2 or d < 1:
        raise ValueError("need n >= 2 and d >= 1")
    one = np.stack([[random_unitary_2x2(rng) for _ in range(n)] for _ in range(d + 1)])
    gates = []
    for layer in range(1, d + 1):
        for q in brickwork_pairs(n, layer, first_parity):
            gates.append((layer, q, GATE_DENSE4, random_unitary_4x4(rng)))
    return Circuit(n=n, d=d, one_qubit=one, gates=gates, first_parity=first_parity, label=label)


SWAP_GATE = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def swap_network_circuit(n: int, d: int, rng: np.random.Generator, first_parity: int = 1,
                         label: str = "") -> Circuit:
    """Open-chain brickwork whose entanglers are SWAP gates dressed with
    Haar-random one-qubit gates, (A (x) B) SWAP (C (x) D): operator Schmidt
    rank four, yet U|0^n> stays a product state, so every amplitude has a
    closed form at any n.  One-qubit sites are Haar-random."""
    one = np.stack([[random_unitary_2x2(rng) for _ in range(n)] for _ in range(d + 1)])
    gates = []
    for layer in range(1, d + 1):
        for q in brickwork_pairs(n, layer, first_parity):
            a, b, c, e = (random_unitary_2x2(rng) for _ in range(4))
            gates.append((layer, q, GATE_DENSE4, np.kron(a, b) @ SWAP_GATE @ np.kron(c, e)))
    return Circuit(n=n, d=d, one_qubit=one, gates=gates, first_parity=first_parity, label=label)


def random_rank2_gate(rng: np.random.Generator, kind: str = "zz") -> np.ndarray:
    """A two-qubit unitary of operator Schmidt rank 2 (basis 2*x_q + x_{q+1}).

    kind "zz":    (a1 (x) b1) exp(i theta Z(x)Z) (a2 (x) b2) with random locals.
    kind "cnot_down": CNOT with the upper qubit as control.
    kind "cnot_up":   CNOT with the lower qubit as control.
    kind "cphase":    diag(1, 1, 1, e^{i phi}).
    """
    if kind == "zz":
        th = rng.uniform(0.1, 1.4)
        zz = np.diag(np.exp(1j * th * np.array([1, -1, -1, 1]))).astype(np.complex128)
        a1, b1, a2, b2 = (random_unitary_2x2(rng) for _ in range(4))
        return np.kron(a1, b1) @ zz @ np.kron(a2, b2)
    if kind == "cnot_down":
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
    if kind == "cnot_up":
        return np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=np.complex128)
    if kind == "cphase":
        return np.diag([1, 1, 1, np.exp(1j * rng.uniform(0, 2 * np.pi))]).astype(np.complex128)
    raise ValueError(kind)


# The workload shapes (n, d, T count, open legs, batches).  Config 0 is the
# tiny all-amplitude case; 1 medium; 2 precision; 3 serving; 4 full width.
CONFIGS = {
    0: dict(name="tiny", n=12, d=12, n_t=8, k=3, batches=512),
    1: dict(name="medium", n=40, d=40, n_t=60, k=6, batches=64, restrict_n=24),
    2: dict(name="precision", n=70, d=56, n_t=400, k=8, batches=16, restrict_n=22),
    3: dict(name="serving", requests=512),
    4: dict(name="full_width", n=70, d=66, n_t=468, k=8, batches=8, restrict_n=24),
    # the paper's production shape on one device: n = d = 70, w = 35, the
    # IBM instance's T density (468 T, 0.096 per qubit-layer site)
    5: dict(name="width35", n=70, d=70, n_t=468, k=8, batches=2, restrict_n=22),
}


def config_circuit(cid: int, seed: int = 1) -> Circuit:
    cfg = CONFIGS[cid]
    return brickwork_circuit(cfg["n"], cfg["d"], cfg["n_t"], rng_for(cid, seed, 0),
                             label=f"{cfg['name']}:seed{seed}")


def config_bitstrings(cid: int, seed: int = 1, count: Optional[int] = None) -> np.ndarray:
    cfg = CONFIGS[cid]
    return random_bitstrings(cfg["n"], count or cfg["batches"], rng_for(cid, seed, 1))


def serving_requests(count: int = 512, seed: int = 1, rate_hz: float = 100.0,
                     n_range: Sequence[int] = (24, 56), d_range: Sequence[int] = (20, 48),
                     k_max: int = 8):
    """Poisson stream of amplitude requests of mixed shape.

    Each request: arrival time (s), circuit (n ~ U{n_range}, d ~ U even in
    d_range, T count = round(0.1*n*d/2)), one bitstring, k ~ U{0..k_max}.
    """
    rng = rng_for(3, seed, 0)
    t = 0.0
    out = []
    d_choices = list(range(d_range[0], d_range[1] + 1, 2))
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.choice(d_choices))
        n_t = int(round(0.1 * n * d / 2))
        k = int(rng.integers(0, k_max + 1))
        circ = brickwork_circuit(n, d, n_t, rng_for(3, seed, 1000 + i), label=f"req{i}")
        bits = random_bitstrings(n, 1, rng_for(3, seed, 5000 + i))
        out.append(dict(id=i, arrival=t, circuit=circ, bits=bits, k=k))
    return out
