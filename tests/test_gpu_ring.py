"""GPU tests of the ring geometry (Sec. 6.3) by slicing its wrap-pair CZ
bonds: the sum over 2^m open-chain slices (run in grouped launches of up to
1024 slices), through the C ABI, against the FP64 oracle's state vector of
the ring itself."""
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


@pytest.mark.parametrize("n,d,k,opts", [(6, 6, 0, None), (8, 8, 2, None), (10, 9, 2, None),
                                        (12, 12, 3, dict(max_tile_bits=6, low_bits=2, reg_bits=3)),
                                        (16, 16, 4, None), (20, 20, 4, dict(max_tile_bits=8)),
                                        # 4096 slices: four groups of 1024
                                        (24, 24, 2, None)])
def test_ring_matches_oracle(n, d, k, opts):
    from paper_2608_13110_amd import RingPlan
    c = W.ring_circuit(n, d, n, W.rng_for(140, n, d))
    bits = W.random_bitstrings(n, 3, W.rng_for(141, n, d))
    rp = RingPlan.from_circuit(c, opts)
    info = rp.info(k, len(bits))
    print(f"  [gpu] ring n={n} d={d} k={k}: {info['slices']} slices of width {info['width']}", flush=True)
    got = rp.amplitudes(torch.from_numpy(bits).cuda(), k)
    torch.cuda.synchronize()
    ref = oracle.amplitudes(c, bits, k)
    per, l2 = H.amp_errors(got.cpu().numpy(), ref, n)
    assert per < H.TOL_C64 and l2 < H.TOL_C64, (per, l2)
    rp.close()


def test_ring_equals_host_emulation_of_its_slices():
    from paper_2608_13110_amd import RingPlan
    c = W.with_gate_values(W.ring_circuit(10, 10, 0, W.rng_for(142, 1)), W.rng_for(142, 2))
    bits = W.random_bitstrings(10, 2, W.rng_for(142, 3))
    rp = RingPlan.from_circuit(c, dict(max_tile_bits=6, low_bits=2, reg_bits=3))
    got = rp.amplitudes(torch.from_numpy(bits).cuda(), 2).cpu().numpy()
    emu = rp.debug_emulate_device(bits, 2)
    per, l2 = H.amp_errors(got, emu, 10)
    assert per < 1e-6
