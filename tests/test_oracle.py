"""Pins for the oracle (CPU only).

Each check ties the oracle to something other than itself: a brute-force
Kronecker-product unitary, a stabilizer tableau on T-free Clifford circuits,
the closed form of a T gate right before measurement, unitarity, and the
log-XEB interval printed in the paper.  ``test_planted_mistakes_are_caught``
shows that plausible mistakes planted in the oracle fail these pins.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.pinlib import brute, tableau

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _random_general_circuit(n, d, seed, dense_frac=0.3):
    rng = W.rng_for(101, seed)
    c = W.brickwork_circuit(n, d, 0, rng)
    c = W.with_gate_values(c, rng)
    gates = []
    for (l, q, kind, m) in c.gates:
        u = rng.random()
        if u < dense_frac / 2:
            gates.append((l, q, W.GATE_DENSE4, W.random_rank2_gate(rng, "zz")))
        elif u < dense_frac:
            z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
            gates.append((l, q, W.GATE_DENSE4, np.linalg.qr(z)[0]))
        else:
            gates.append((l, q, kind, m))
    c.gates = gates
    return c


@pytest.mark.parametrize("n,d,seed", [(2, 1, 1), (2, 4, 2), (3, 3, 3), (4, 5, 4), (5, 6, 5),
                                      (6, 7, 6), (6, 4, 7), (5, 9, 8)])
def test_matches_bruteforce(n, d, seed):
    c = _random_general_circuit(n, d, seed)
    ref = brute.all_amplitudes(c)
    got = oracle.statevector(c)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("n,d", [(4, 4), (4, 7), (6, 5), (6, 8)])
def test_ring_matches_bruteforce(n, d):
    # the ring's wrap pair (n-1, 0) (Sec. 6.3), doped Cliffords and random
    # one-qubit unitaries, against Kronecker products with a qubit permutation
    c = W.ring_circuit(n, d, 3, W.rng_for(120, n, d))
    assert sum(1 for g in c.gates if g[1] == n - 1) == d // 2 + (d % 2)
    for cc in (c, W.with_gate_values(c, W.rng_for(121, n, d))):
        assert np.max(np.abs(oracle.statevector(cc) - brute.all_amplitudes(cc))) < 1e-13


@pytest.mark.parametrize("first_parity", [0, 1])
def test_doped_clifford_bruteforce(first_parity):
    c = W.brickwork_circuit(6, 8, 5, W.rng_for(102, first_parity), first_parity=first_parity)
    assert np.max(np.abs(oracle.statevector(c) - brute.all_amplitudes(c))) < 1e-13


def test_normalised():
    c = W.brickwork_circuit(14, 14, 12, W.rng_for(103, 1))
    psi = oracle.statevector(c)
    assert abs(float(np.vdot(psi, psi).real) - 1.0) < 1e-12


@pytest.mark.parametrize("n,d,seed", [(8, 8, 1), (10, 11, 2), (9, 12, 3)])
def test_clifford_all_probabilities_match_tableau(n, d, seed):
    c = W.brickwork_circuit(n, d, 0, W.rng_for(104, seed))
    _, words = W.clifford_table()
    tab = tableau.run_clifford(c, words)
    p = np.abs(oracle.statevector(c)) ** 2
    for x in range(1 << n):
        bits = [(x >> (n - 1 - j)) & 1 for j in range(n)]
        pt = tab.prob(bits)
        assert abs(p[x] - pt) < 1e-12, (x, p[x], pt)
        if p[x] > 1e-12:
            r = -math.log2(p[x])
            assert abs(r - round(r)) < 1e-9


def test_clifford_sampled_probabilities_match_tableau():
    n, d = 18, 18
    c = W.brickwork_circuit(n, d, 0, W.rng_for(105, 1))
    _, words = W.clifford_table()
    tab = tableau.run_clifford(c, words)
    psi = oracle.statevector(c)
    rng = W.rng_for(105, 2)
    xs = [tab.sample(rng) for _ in range(24)] + list(W.random_bitstrings(n, 24, rng))
    nonzero = 0
    for bits in xs:
        idx = int(oracle.prefix_index(bits[None, :], 0)[0])
        pt = tab.prob(bits)
        assert abs(abs(psi[idx]) ** 2 - pt) < 1e-12
        nonzero += pt > 0
    assert nonzero >= 24


@pytest.mark.parametrize("q", [0, 3, 7])
def test_t_right_before_measurement_is_a_phase(q):
    c = W.brickwork_circuit(8, 9, 6, W.rng_for(106, q))
    psi = oracle.statevector(c)
    c2 = W.Circuit(n=c.n, d=c.d, one_qubit=c.one_qubit.copy(), gates=list(c.gates))
    c2.one_qubit[c.d, q] = W.T_GATE @ c2.one_qubit[c.d, q]
    psi2 = oracle.statevector(c2)
    xq = (np.arange(1 << c.n) >> (c.n - 1 - q)) & 1
    assert np.max(np.abs(psi2 - psi * np.exp(1j * np.pi / 4 * xq))) < 1e-14


def test_amplitude_batches_index_convention():
    c = W.brickwork_circuit(7, 6, 3, W.rng_for(107, 1))
    psi = brute.all_amplitudes(c)
    bits = W.random_bitstrings(7, 5, W.rng_for(107, 2))
    for k in (0, 1, 3, 7):
        z = oracle.amplitudes(c, bits, k)
        for i, row in enumerate(bits):
            for b in range(1 << k):
                full = list(row[: 7 - k]) + [(b >> (k - 1 - j)) & 1 for j in range(k)]
                x = sum(v << (6 - j) for j, v in enumerate(full))
                assert abs(z[i, b] - psi[x]) < 1e-14


def _golden(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_logxeb_interval_matches_paper():
    g = _golden("logxeb_interval.txt")
    lo, hi = oracle.ci95(g["F"], g["SE"])
    # F, SE and the bounds are each printed to 5 decimals (half-unit 0.5e-5),
    # so the recomputed bounds agree to within 0.5e-5 * (1 + 1.96 + 1).
    tol = 0.5e-5 * (1 + 1.96 + 1)
    assert abs(lo - g["LO"]) <= tol and abs(hi - g["HI"]) <= tol
    assert abs(0.5 * (g["LO"] + g["HI"]) - g["F"]) <= 1e-5


def test_logxeb_closed_forms():
    n = 20
    # uniform probabilities 2^-n give ln p + n ln 2 = 0, so F = gamma exactly
    f, se, _, _ = oracle.logxeb(np.full(100, 2.0 ** -n), n)
    assert abs(f - oracle.EULER_GAMMA) < 1e-12 and se < 1e-12
    # Porter-Thomas z ~ Exp(1): E[ln z] = -gamma, so uniform draws give F ~ 0
    z = W.rng_for(108, 1).exponential(size=200000)
    f, se, _, _ = oracle.logxeb(z * 2.0 ** -n, n)
    assert abs(f) < 5 * se
    # exact sampling draws z with density z e^-z: E[ln z] = 1 - gamma, so F ~ 1
    z = W.rng_for(108, 2).gamma(2.0, size=200000)
    f, se, _, _ = oracle.logxeb(z * 2.0 ** -n, n)
    assert abs(f - 1.0) < 5 * se


def test_logxeb_standard_error_worked_example():
    # ln p = -1, -2, -3, -4: mean -5/2, sample variance (ddof = 1)
    # (1.5^2 + 0.5^2 + 0.5^2 + 1.5^2) / 3 = 5/3, so SE = sqrt(5/3) / sqrt(4)
    # (Sec. 5.2: the standard error of the mean of ln p over N draws)
    n = 7
    f, se, lo, hi = oracle.logxeb(np.exp(-np.arange(1.0, 5.0)), n)
    assert abs(se - math.sqrt(5.0 / 3.0) / 2.0) < 1e-12
    assert abs(f - (oracle.EULER_GAMMA + n * math.log(2.0) - 2.5)) < 1e-12
    assert abs(lo - (f - 1.96 * se)) < 1e-12 and abs(hi - (f + 1.96 * se)) < 1e-12


def test_logxeb_standard_error_matches_repetition_spread():
    # Porter-Thomas draws z ~ Exp(1) (uniform bitstrings, Sec. 4.1): ln z has
    # variance pi^2 / 6, so the estimate over N draws spreads by
    # sqrt(pi^2 / (6 N)) across independent repetitions; the reported SE of
    # each repetition must match that spread (an SE without its 1/sqrt(N)
    # would be sqrt(N) = 7 times too large)
    n, N, reps = 16, 49, 4000
    z = W.rng_for(108, 3).exponential(size=(reps, N))
    est = [oracle.logxeb(row * 2.0 ** -n, n) for row in z]
    fs = np.array([e[0] for e in est])
    ses = np.array([e[1] for e in est])
    closed = math.sqrt(math.pi ** 2 / 6.0 / N)
    assert abs(fs.std(ddof=1) / closed - 1.0) < 0.05
    assert abs(ses.mean() / closed - 1.0) < 0.05


def test_tv_conditional():
    z = np.array([[1.0, 0.0], [1.0, 1.0]], dtype=np.complex128)
    w = np.array([[0.0, 1.0], [1.0, 1.0j]], dtype=np.complex128)
    assert np.allclose(oracle.tv_conditional(z, w), [1.0, 0.0])


def test_tv_conditional_normalises_each_row():
    # p(b|a) divides by the row's own marginal Q_a (Sec. 5.1): rows that
    # differ only by a scale have TV 0, and |Z| = (3, 0) against (3, 3)
    # gives p(b|a) = (1, 0) against (1/2, 1/2), TV 1/2
    z = np.array([[3.0, 0.0], [0.5, 0.25j], [2.0, 1.0]], dtype=np.complex128)
    w = np.array([[3.0, 3.0], [5.0, 2.5j], [2e-6, 1e-6j]], dtype=np.complex128)
    assert np.allclose(oracle.tv_conditional(z, w), [0.5, 0.0, 0.0], atol=1e-12)


def _pins_pass(mutation):
    """True if every pin used here still passes for the mutated oracle."""
    ok = True
    c = _random_general_circuit(5, 6, 11, dense_frac=0.0)
    ok &= np.max(np.abs(oracle.statevector(c, mutation) - brute.all_amplitudes(c))) < 1e-12
    cc = W.brickwork_circuit(8, 8, 0, W.rng_for(109, 1))
    _, words = W.clifford_table()
    tab = tableau.run_clifford(cc, words)
    p = np.abs(oracle.statevector(cc, mutation)) ** 2
    for x in range(0, 256, 7):
        bits = [(x >> (7 - j)) & 1 for j in range(8)]
        ok &= abs(p[x] - tab.prob(bits)) < 1e-12
    return bool(ok)


def test_unmutated_oracle_passes_pins():
    assert _pins_pass(0)


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5])
def test_planted_mistakes_are_caught(mutation):
    assert not _pins_pass(mutation)


# ---------------------------------------------------------------------------
# Samplers (Sec. 4.1, Sec. 4.2)

def _paper_pin(key):
    with open(os.path.join(GOLD, "paper_pins.txt")) as f:
        for line in f:
            if line.startswith(key + " "):
                return line.split()[1:]
    raise KeyError(key)


def test_batched_sample_is_the_inverse_cdf():
    # uniforms on a fine grid land on every b in proportion to p(b|a), to
    # within one grid step: the sampler draws from the conditional
    rng = np.random.default_rng(501)
    k, N = 4, 4096
    amps = rng.standard_normal((3, 1 << k)) + 1j * rng.standard_normal((3, 1 << k))
    amps[1, 5] = 0.0  # a zero-probability suffix is never drawn
    u = (np.arange(N) + 0.5) / N
    for i in range(3):
        b, q = oracle.batched_sample(np.repeat(amps[i:i + 1], N, axis=0), u)
        p = np.abs(amps[i]) ** 2
        assert np.allclose(q, p.sum(), rtol=1e-15, atol=0)
        counts = np.bincount(b, minlength=1 << k)
        assert np.all(np.abs(counts - N * p / p.sum()) <= 1.0)
        if i == 1:
            assert counts[5] == 0
    # u just below 1 takes the last suffix with p > 0; u = 0 the first
    b, _ = oracle.batched_sample(amps[:1], np.array([np.nextafter(1.0, 0.0)]))
    assert b[0] == np.flatnonzero(np.abs(amps[0]) > 0)[-1]
    b, _ = oracle.batched_sample(amps[:1], np.array([0.0]))
    assert b[0] == np.flatnonzero(np.abs(amps[0]) > 0)[0]


def test_batched_tv_equals_prefix_marginal_form():
    # Sec. 4.2, Eq. tv_norm: summing |q_k - p| over (a, b) equals
    # (1/2) sum_a |Q_a - 1/A|, for any distribution
    rng = np.random.default_rng(502)
    for k in (1, 3, 6):
        p = rng.random(1 << 12) ** 3
        p /= p.sum()
        q, tv = oracle.batched_distribution(p, k)
        A = p.size >> k
        qa = p.reshape(A, -1).sum(axis=1)
        assert abs(q.sum() - 1.0) < 1e-12
        assert abs(tv - 0.5 * np.abs(qa - 1.0 / A).sum()) < 1e-12


def test_batched_tv_porter_thomas():
    # Porter-Thomas probabilities: E TV = 1/sqrt(2 pi 2^k) (Sec. 4.2); the
    # paper prints 2.5e-2 for k = 8
    k = 8
    printed = float(_paper_pin("BATCHED_TV")[1])
    assert abs(oracle.batched_tv(k) - printed) < 0.05e-2
    rng = np.random.default_rng(503)
    p = rng.exponential(size=1 << 21)
    p /= p.sum()
    _, tv = oracle.batched_distribution(p, k)
    # 2^13 prefixes: the mean of |N(0, s)| over them is within ~1 % (3 sd)
    assert abs(tv / oracle.batched_tv(k) - 1.0) < 0.03


def test_frugal_rejection_closed_forms():
    # Sec. 4.1: acceptance (1 - e^-M)/M and TV exp(-M/(1 - e^-M)) under
    # Porter-Thomas; the paper prints TV ~ 4.5e-5 at M = 10
    printed = float(_paper_pin("FRUGAL_TV")[1])
    assert abs(oracle.frugal_tv(10.0) / printed - 1.0) < 0.02
    assert abs(oracle.frugal_alpha(10.0) - (1 - math.exp(-10)) / 10) < 1e-15
    rng = np.random.default_rng(504)
    p = rng.exponential(size=1 << 22)
    p /= p.sum()
    for M in (2.0, 3.0, 5.0):
        _, alpha, tv = oracle.frugal_distribution(p, M)
        assert abs(alpha / oracle.frugal_alpha(M) - 1.0) < 0.005
        assert abs(tv / oracle.frugal_tv(M) - 1.0) < 0.05
    # M -> 0 accepts every candidate (q_M = uniform); a huge M reproduces p
    _, alpha, _ = oracle.frugal_distribution(p, 1e-9)
    assert alpha == 1.0
    q, _, tv = oracle.frugal_distribution(p, 1e9)
    assert tv < 1e-12


def test_frugal_accept_rate_on_a_grid():
    rng = np.random.default_rng(505)
    n, M, N = 10, 4.0, 2048
    amps = (rng.standard_normal(6) + 1j * rng.standard_normal(6)) * 2.0 ** (-n / 2)
    u = (np.arange(N) + 0.5) / N
    for a in amps:
        acc, z = oracle.frugal_accept(np.full(N, a), n, M, u)
        assert np.allclose(z, 2.0 ** n * abs(a) ** 2, rtol=1e-15, atol=0)
        assert abs(acc.mean() - min(1.0, z[0] / M)) <= 1.0 / N


# oracle.product_amplitudes (dressed-SWAP networks, any n): brute force on
# small chains, and refusal of gates whose G SWAP is not a product
@pytest.mark.parametrize("n,d,fp", [(2, 2, 1), (5, 6, 0), (8, 8, 1), (11, 10, 0), (14, 12, 1)])
def test_product_oracle_matches_state_vector(n, d, fp):
    # pin of oracle.product_amplitudes: brute force on small chains
    c = W.swap_network_circuit(n, d, W.rng_for(411, n, d), fp)
    bits = W.random_bitstrings(n, 16, W.rng_for(412, n))
    ref = oracle.amplitudes(c, bits, 0)[:, 0]
    assert np.max(np.abs(oracle.product_amplitudes(c, bits) - ref)) < 1e-13


def test_product_oracle_refuses_entangling_gates():
    c = W.generic_brickwork_circuit(4, 4, W.rng_for(413))
    with pytest.raises(ValueError):
        oracle.product_amplitudes(c, W.random_bitstrings(4, 2, W.rng_for(414)))
