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
                 U = L_d E_d ... E_1 L_0 (Sec. 2.1).
``amplitudes``   the batch tensor Z[b] = <a, b|U|0^n> of the batched
                 contraction (Sec. 4.3, its Require/Ensure lines): b are the
                 last k qubits, index b read MSB-first over qubits n-k..n-1.
``logxeb``       the log-XEB estimator of Sec. 5.2 (Eq. normalized-log-xeb),
                 with its empirical standard error and 95 % interval.
``tv_conditional`` total-variation distance of the conditional
                 distributions p(b|a), the accuracy metric of Sec. 5.1.

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
