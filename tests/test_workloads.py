"""Generator checks against the circuit family of Sec. 2.1 (CPU only)."""
import numpy as np

import workloads as W


def test_cz_counts_match_paper():
    # Sec. 2.1: the n=70 circuit alternates 34 and 35 CZ per layer, 2415 at d=70
    c = W.brickwork_circuit(70, 70, 468, W.rng_for(1, 1))
    per_layer = [sum(1 for g in c.gates if g[0] == l) for l in range(1, 71)]
    assert sorted(set(per_layer)) == [34, 35]
    assert all(per_layer[i] != per_layer[i + 1] for i in range(69))
    assert c.n_cz() == 2415 and c.n_t() == 468


def test_first_layer_pattern():
    c = W.brickwork_circuit(10, 3, 0, W.rng_for(1, 2))
    assert [g[1] for g in c.gates if g[0] == 1] == [1, 3, 5, 7]   # 1-based (2,3),(4,5),...
    assert [g[1] for g in c.gates if g[0] == 2] == [0, 2, 4, 6, 8]


def test_clifford_table():
    mats, words = W.clifford_table()
    assert len(words) == 24
    for m in mats:
        assert np.allclose(m @ m.conj().T, np.eye(2))
    # distinct modulo global phase
    for i in range(24):
        for j in range(i):
            ov = abs(np.trace(mats[i].conj().T @ mats[j])) / 2
            assert ov < 1 - 1e-9


def test_seeded_and_restrict():
    a = W.config_circuit(4, 1)
    b = W.config_circuit(4, 1)
    assert np.array_equal(a.one_qubit, b.one_qubit) and a.n_t() == 468
    r = W.restrict(a, 24)
    assert r.n == 24 and r.d == 66
    assert all(g[1] + 1 < 24 for g in r.gates)
    assert np.array_equal(r.one_qubit, a.one_qubit[:, :24])


def test_serving_stream_shapes():
    reqs = W.serving_requests(count=40, seed=1)
    for r in reqs:
        c = r["circuit"]
        assert 24 <= c.n <= 56 and 20 <= c.d <= 48 and c.d % 2 == 0
        assert c.n_t() == round(0.1 * c.n * c.d / 2)
        assert 0 <= r["k"] <= 8
    t = [r["arrival"] for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
