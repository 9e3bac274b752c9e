"""Shared test helpers: circuits, tolerances, library symbol list."""
import os
import re

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    """Every function declared in include/*.h."""
    syms = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            syms |= set(re.findall(r"^\s*(?:int|void|uint64_t|const char\*)\s+(tnc_\w+)\s*\(", txt, re.M))
    return sorted(syms)


def mixed_circuit(n, d, seed, first_parity=1, dense=0.0, n_t=None):
    """Doped-Clifford brickwork; a fraction `dense` of the CZ replaced by
    other rank-2 entanglers (ZZ-type, CNOT either way, CPhase)."""
    rng = W.rng_for(201, seed)
    c = W.brickwork_circuit(n, d, max(1, n * d // 10) if n_t is None else n_t, rng,
                            first_parity=first_parity)
    if dense:
        gates = []
        kinds = ["zz", "cnot_up", "cnot_down", "cphase"]
        for (l, q, kind, m) in c.gates:
            if rng.random() < dense:
                gates.append((l, q, W.GATE_DENSE4, W.random_rank2_gate(rng, kinds[int(rng.integers(4))])))
            else:
                gates.append((l, q, kind, m))
        c.gates = gates
    return c


def amp_errors(got, ref, n):
    """Per-amplitude error relative to max(|ref|, 2^(-n/2)) and the batch
    relative l2 error ||got-ref|| / ||ref|| (rows = batches)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    floor = 2.0 ** (-n / 2)
    per = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
    l2 = np.linalg.norm(got - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(per.max()), float(l2.max())


# complex64 boundary updates: per amplitude |err| <= 1e-5 * max(|ref|, 2^-n/2)
TOL_C64 = 1e-5
