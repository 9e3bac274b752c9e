"""The oracle: plain, slow, obviously correct CPU FP64 reference.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library (``paper_2608_13110_amd``) never imports, links or calls it,
and this package imports nothing from the product.  The two share only the
seeded input generators in ``workloads``.

Contents
--------
``statevector``  full 2^n FP64 state of U|0^n> (C, ``sv.c``), following the
                 amplitude definition psi(x) = <x|U|0^n> of Sec. 2.2 with
                 U = L_d E_d ... E_1 L_0 (Sec. 2.1); a gate listed at
                 q = n-1 acts on the ring's wrap pair (n-1, 0) (Sec. 6.3).
``amplitudes``   the batch tensor Z[b] = <a, b|U|0^n> of the batched
                 contraction (Sec. 4.3, its Require/Ensure lines): b are the
                 last k qubits, index b read MSB-first over qubits n-k..n-1.
``logxeb``       the log-XEB estimator of Sec. 5.2 (Eq. normalized-log-xeb),
                 with its empirical standard error and 95 % interval.
``product_amplitudes`` <x|U|0^n> for circuits whose entanglers are all
                 SWAP gates dressed with one-qubit gates (G = (P (x) Q) SWAP),
                 at any n: U|0^n> stays a product state, tracked qubit by
                 qubit (operator Schmidt rank 4 entanglers with a closed form,
                 for checks of the bond-dimension-four path at full width).
``tv_conditional`` total-variation distance of the conditional
                 distributions p(b|a), the accuracy metric of Sec. 5.1.
``batched_sample`` the batched sampler of Sec. 4.2: one suffix b per batch
                 from p(b|a) = p(a, b) / Q_a, by inverse CDF of a given
                 uniform; with ``batched_distribution`` (q_k and its TV).
``frugal_accept`` frugal rejection of Sec. 4.1: accept x with probability
                 min(1, z_x / M), z_x = 2^n p(x), for a given uniform; with
                 ``frugal_distribution`` (q_M and its TV) and the
                 Porter-Thomas closed forms ``frugal_alpha``, ``frugal_tv``,
                 ``batched_tv``.

Every function here has pins in ``tests/test_oracle.py`` (brute-force
Kronecker products, a stabilizer tableau for T-free Cliffords, the closed
form of a T right before measurement, normalisation, and the paper's printed
log-XEB interval).  None is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EULER_GAMMA = 0.57721566490153286060651209008240243


def build(force: bool = False) -> str:
    """Compile ``sv.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_statevector.restype = ctypes.c_int
        lib.oracle_statevector.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def statevector(circ, mutation: int = 0) -> np.ndarray:
    """Full state U|0^n> as complex128 of length 2^n (qubit j = bit n-1-j)."""
    lib = _load()
    n, d = circ.n, circ.d
    one = np.ascontiguousarray(circ.one_qubit, dtype=np.complex128)
    layer, q, kind, mats = circ.gate_arrays()
    mats = np.ascontiguousarray(mats, dtype=np.complex128)
    psi = np.empty(1 << n, dtype=np.complex128)
    rc = lib.oracle_statevector(n, d, one.ctypes.data, len(layer), layer.ctypes.data,
                                q.ctypes.data, kind.ctypes.data, mats.ctypes.data,
                                int(mutation), psi.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_statevector rejected the circuit")
    return psi


def prefix_index(bits: np.ndarray, k: int) -> np.ndarray:
    """State index of (a, b=0) for each bitstring row: MSB-first, last k zeroed."""
    bits = np.asarray(bits, dtype=np.int64)
    n = bits.shape[1]
    weights = (1 << np.arange(n - 1, -1, -1, dtype=np.int64))
    idx = bits @ weights
    return idx & ~np.int64((1 << k) - 1)


def amplitudes(circ, bitstrings: np.ndarray, k: int, psi: Optional[np.ndarray] = None,
               mutation: int = 0) -> np.ndarray:
    """Z[batch, b] = <a, b|U|0^n> for each bitstring's prefix a (last k bits open).

    Returns complex128 of shape (batches, 2^k); b is read MSB-first over the
    qubits n-k..n-1, so column b is the state index a*2^k + b.
    """
    if psi is None:
        psi = statevector(circ, mutation)
    base = prefix_index(bitstrings, k)
    cols = np.arange(1 << k, dtype=np.int64)
    return psi[base[:, None] + cols[None, :]]


SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def product_amplitudes(circ, bitstrings: np.ndarray) -> np.ndarray:
    """<x|U|0^n> (one per bitstring row) when every entangler is G = (P (x) Q)
    SWAP (basis 2*x_q + x_{q+1}).  The state is then a product of one-qubit
    states s_0 (x) ... (x) s_{n-1} at every layer (Sec. 2.1's U applied layer
    by layer): a one-qubit gate L maps s_q to L s_q, and G maps (s_q, s_{q+1})
    to (P s_{q+1}, Q s_q).  P (x) Q = G SWAP is recovered as the rank-one
    factor of its realignment R[2a+a'][2b+b'] = (G SWAP)[2a+b][2a'+b'] (the
    largest singular pair); a gate whose realignment is not rank one is
    refused.  The amplitude is prod_q s_q[x_q].
    """
    n, d = circ.n, circ.d
    one = np.asarray(circ.one_qubit, dtype=np.complex128)
    factors = {}
    for (layer, q, kind, m) in circ.gates:
        if m is None:
            raise ValueError("product_amplitudes needs dressed-SWAP entanglers, not CZ")
        k = np.asarray(m, dtype=np.complex128) @ SWAP
        r = k.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
        u, sv, vh = np.linalg.svd(r)
        if sv[1] > 1e-9 * sv[0]:
            raise ValueError("entangler is not a dressed SWAP")
        factors[(layer, q)] = ((u[:, 0] * sv[0]).reshape(2, 2), vh[0].reshape(2, 2))
    s = np.zeros((n, 2), dtype=np.complex128)
    s[:, 0] = 1.0
    s = np.einsum("qij,qj->qi", one[0], s)
    for layer in range(1, d + 1):
        for (l, q), (P, Q) in factors.items():
            if l == layer:
                s[q], s[q + 1] = P @ s[q + 1], Q @ s[q]
        s = np.einsum("qij,qj->qi", one[layer], s)
    bits = np.asarray(bitstrings, dtype=np.int64)
    return np.prod(s[np.arange(n)[None, :], bits], axis=1)


def logxeb(probs: np.ndarray, n: int):
    """Log-XEB estimate (Sec. 5.2, Eq. normalized-log-xeb).

    F = gamma + n ln 2 + (1/N) sum_i ln p(x_i).  SE is the sample standard
    deviation of ln p over sqrt(N) (the draws treated as independent); the
    95 % interval is F -/+ 1.96 SE.  Returns (F, SE, lo, hi), all FP64.
    """
    lp = np.log(np.asarray(probs, dtype=np.float64))
    N = lp.size
    f = EULER_GAMMA + n * math.log(2.0) + float(lp.mean())
    se = float(lp.std(ddof=1) / math.sqrt(N)) if N > 1 else float("nan")
    return f, se, f - 1.96 * se, f + 1.96 * se


def ci95(f: float, se: float):
    """The 95 % interval F -/+ 1.96 SE used with the log-XEB estimate."""
    return f - 1.96 * se, f + 1.96 * se


def tv_conditional(za: np.ndarray, zb: np.ndarray) -> np.ndarray:
    """Per-batch total variation between conditional distributions p(b|a).

    ``za``, ``zb``: (batches, 2^k) amplitudes.  p(b|a) = |Z[b]|^2 / sum_b |Z[b]|^2.
    """
    pa = np.abs(np.asarray(za, dtype=np.complex128)) ** 2
    pb = np.abs(np.asarray(zb, dtype=np.complex128)) ** 2
    pa = pa / pa.sum(axis=1, keepdims=True)
    pb = pb / pb.sum(axis=1, keepdims=True)
    return 0.5 * np.abs(pa - pb).sum(axis=1)


# ---------------------------------------------------------------------------
# Samplers on top of the amplitudes (Sec. 4.1, Sec. 4.2).  The random numbers
# are inputs (uniforms in [0, 1)), so a sample is a function of its inputs.

def batched_sample(amps: np.ndarray, u: np.ndarray):
    """Batched sampling, Sec. 4.2, steps 3-4: for each batch (prefix a) the
    probabilities p(a, b) = |Z[b]|^2, their sum Q_a, and the suffix b drawn
    from p(b | a) = p(a, b) / Q_a by inverse CDF: the smallest b with
    p(a, 0) + ... + p(a, b) > u Q_a (b = 2^k - 1 if rounding leaves none).

    amps: (batches, 2^k) complex; u: (batches,) uniforms.  FP64 throughout,
    the prefix sums taken left to right.  Returns (b int64, Q float64).
    """
    p = np.abs(np.asarray(amps, dtype=np.complex128)) ** 2
    q = p.sum(axis=1)
    out = np.empty(p.shape[0], dtype=np.int64)
    for i in range(p.shape[0]):
        target = float(u[i]) * q[i]
        acc = 0.0
        b = p.shape[1] - 1
        for j in range(p.shape[1]):
            acc += p[i, j]
            if acc > target:
                b = j
                break
        out[i] = b
    return out, q


def batched_distribution(p_full: np.ndarray, k: int):
    """The output distribution of the batched sampler with uniform prefixes
    (Sec. 4.2): q_k(a, b) = p(a, b) / (A Q_a), A = 2^(n-k); returns (q_k,
    TV(q_k, p)) with the TV summed over all (a, b) by its definition."""
    p = np.asarray(p_full, dtype=np.float64)
    B = 1 << k
    A = p.size // B
    pa = p.reshape(A, B)
    qa = pa.sum(axis=1, keepdims=True)
    q = (pa / (A * qa)).reshape(-1)
    return q, 0.5 * float(np.abs(q - p).sum())


def frugal_accept(amps: np.ndarray, n: int, M: float, u: np.ndarray):
    """Frugal rejection, Sec. 4.1, steps 2-3: z_x = 2^n |amp_x|^2 and the
    candidate is accepted when u < min(1, z_x / M).  Returns (accept bool,
    z float64)."""
    z = np.ldexp(np.abs(np.asarray(amps, dtype=np.complex128)) ** 2, n)
    return np.asarray(u, dtype=np.float64) < np.minimum(1.0, z / M), z


def frugal_distribution(p_full: np.ndarray, M: float):
    """The distribution q_M of accepted candidates (uniform candidates,
    acceptance min(1, z_x / M), Sec. 4.1), its acceptance probability and
    TV(q_M, p)."""
    p = np.asarray(p_full, dtype=np.float64)
    acc = np.minimum(1.0, p * p.size / M)
    alpha = float(acc.mean())
    q = acc / acc.sum()
    return q, alpha, 0.5 * float(np.abs(q - p).sum())


def frugal_alpha(M: float) -> float:
    """Mean acceptance under Porter-Thomas z ~ Exp(1): (1 - e^-M) / M."""
    return (1.0 - math.exp(-M)) / M


def frugal_tv(M: float) -> float:
    """TV of frugal rejection under Porter-Thomas: exp(-M / (1 - e^-M))."""
    return math.exp(-M / (1.0 - math.exp(-M)))


def batched_tv(k: int) -> float:
    """Expected TV of batched sampling under Porter-Thomas: 1/sqrt(2 pi 2^k)."""
    return 1.0 / math.sqrt(2.0 * math.pi * (1 << k))
