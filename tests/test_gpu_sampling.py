"""GPU tests of the samplers on top of the amplitudes (Sec. 4.1, Sec. 4.2),
through the C ABI, against the oracle on the same seeded inputs.

A sampled index is decided by comparing a prefix sum with u Q_a in FP64 on
both sides; the two sides add in different orders, so indices must agree
wherever u Q_a is farther than a few ulps from a prefix-sum boundary, and
elsewhere the GPU's index must still be a valid draw.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2608_13110_amd import lib
    lib()
    yield


def _inputs(nb, k, seed):
    rng = np.random.default_rng(seed)
    amps = (rng.standard_normal((nb, 1 << k)) + 1j * rng.standard_normal((nb, 1 << k))) * 2.0 ** (-k / 2)
    u = rng.random(nb)
    return amps, u


def _check_draws(amps, u, b_gpu, q_gpu):
    b_ref, q_ref = oracle.batched_sample(amps, u)
    assert np.allclose(q_gpu, q_ref, rtol=1e-13, atol=0)
    p = np.abs(amps) ** 2
    cdf = np.cumsum(p, axis=1)
    for i in range(len(u)):
        if q_ref[i] == 0.0:  # no mass: both sides give the last suffix
            assert b_gpu[i] == b_ref[i] == p.shape[1] - 1
            continue
        t = u[i] * q_ref[i]
        lo = cdf[i, b_ref[i] - 1] if b_ref[i] > 0 else 0.0
        margin = min(abs(t - lo), abs(cdf[i, b_ref[i]] - t))
        if margin > 1e-12 * q_ref[i]:
            assert b_gpu[i] == b_ref[i], (i, b_gpu[i], b_ref[i])
        else:  # a boundary case: the GPU's draw must still be valid
            g = b_gpu[i]
            glo = cdf[i, g - 1] if g > 0 else 0.0
            assert glo - 1e-12 * q_ref[i] <= t <= cdf[i, g] + 1e-12 * q_ref[i]
            assert p[i, g] > 0


@pytest.mark.parametrize("k,nb", [(0, 5), (1, 7), (3, 64), (8, 300), (9, 33), (10, 40)])
def test_batched_sampler_matches_oracle(k, nb):
    from paper_2608_13110_amd import sample_batched
    amps, u = _inputs(nb, k, 601 + k)
    if k >= 3:
        amps[1, :] = 0.0          # Q_a = 0: the last suffix, as in the oracle
        amps[2, : (1 << k) // 2] = 0.0
        u[3] = 0.0
        u[4] = np.nextafter(1.0, 0.0)
    print(f"  [gpu] batched sampler k={k} batches={nb}", flush=True)
    b, q = sample_batched(torch.from_numpy(amps).cuda(), torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    b, q = b.cpu().numpy(), q.cpu().numpy()
    if k >= 3:
        assert b[1] == (1 << k) - 1 and q[1] == 0.0
        assert b[2] >= (1 << k) // 2
    _check_draws(amps, u, b, q)


def test_frugal_rejection_matches_oracle():
    from paper_2608_13110_amd import frugal_accept
    rng = np.random.default_rng(611)
    n, M, N = 30, 6.0, 100000
    amps = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * 2.0 ** (-(n + 1) / 2)
    u = rng.random(N)
    print("  [gpu] frugal rejection", flush=True)
    acc, z = frugal_accept(torch.from_numpy(amps).cuda(), n, M, torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    acc, z = acc.cpu().numpy().astype(bool), z.cpu().numpy()
    acc_ref, z_ref = oracle.frugal_accept(amps, n, M, u)
    assert np.allclose(z, z_ref, rtol=1e-15, atol=0)
    edge = np.abs(u - np.minimum(1.0, z_ref / M)) < 1e-12
    assert np.array_equal(acc[~edge], acc_ref[~edge])
    # z = 2^n |amp|^2 is Exp(1)-distributed here: acceptance near (1 - e^-M)/M
    assert abs(acc.mean() / oracle.frugal_alpha(M) - 1.0) < 0.03


def test_batched_tv_of_porter_thomas_batches():
    # Sec. 4.2: with Porter-Thomas probabilities the batched sampler's TV,
    # (1/2) sum_a |Q_a - 1/A| with Q_a summed on the GPU, is 1/sqrt(2 pi 2^k)
    from paper_2608_13110_amd import sample_batched
    rng = np.random.default_rng(612)
    k, A = 8, 4096
    z = rng.exponential(size=(A, 1 << k))
    z /= z.sum()
    amps = np.sqrt(z) * np.exp(2j * np.pi * rng.random(z.shape))
    u = rng.random(A)
    b, q = sample_batched(torch.from_numpy(amps).cuda(), torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    tv = 0.5 * np.abs(q.cpu().numpy() - 1.0 / A).sum()
    assert abs(tv / oracle.batched_tv(k) - 1.0) < 0.05


def test_sampling_from_circuit_amplitudes():
    # end to end: uniform prefixes, the GPU's k = 3 batches of a circuit, one
    # suffix per batch; the same draws from the oracle's amplitudes agree
    # wherever u Q_a is not within the amplitudes' FP32-level error of a
    # prefix-sum boundary
    from paper_2608_13110_amd import Plan, sample_batched
    c = W.config_circuit(0)
    k, nb = 3, 256
    bits = W.random_bitstrings(c.n, nb, W.rng_for(613, 1))
    u = W.rng_for(613, 2).random(nb)
    z = Plan.from_circuit(c).amplitudes(torch.from_numpy(bits).cuda(), k)
    b, q = sample_batched(z, torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    b = b.cpu().numpy()
    ref = oracle.amplitudes(c, bits, k)
    b_ref, q_ref = oracle.batched_sample(ref, u)
    assert np.allclose(q.cpu().numpy(), q_ref, rtol=2 * H.TOL_C64, atol=2 * H.TOL_C64 * 2.0 ** -c.n)
    cdf = np.cumsum(np.abs(ref) ** 2, axis=1)
    typical = 2.0 ** (k - c.n)  # mean of Q_a
    live = 0
    for i in range(nb):
        # prefixes of a doped-Clifford circuit can have Q_a = 0 exactly; both
        # sides then sample rounding residue, which decides nothing
        if q_ref[i] < 1e-6 * typical:
            continue
        live += 1
        t = u[i] * q_ref[i]
        dist = np.min(np.abs(cdf[i] - t))
        if dist > 1e-4 * q_ref[i]:
            assert b[i] == b_ref[i]
    assert live > nb // 4
