"""The allocation-free entry point (tnc_amplitudes_noalloc) against
tnc_amplitudes, through the C ABI on the GPU.

Both run the same recorded launches on the same tables, the only difference
being where the workspace lives (the library's per-GPU scratch array against
a caller buffer), so the results must agree bit for bit.
"""
import numpy as np
import pytest

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


def _both(plan, bits, k, storage=0):
    print(f"  [gpu] noalloc n={plan.n} d={plan.d} k={k} batches={len(bits)} storage={storage}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).cuda()
    plan.prepare(k)
    ref = plan.amplitudes(d, k, storage=storage)
    got = plan.amplitudes_noalloc(d, k, storage=storage)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_equals_workspace_path_two_calls():
    from paper_2608_13110_amd import Plan
    # a larger input first (several tiles per pass, fused phases), then a
    # smaller one: the second call reuses the scratch the first one wrote
    big = H.mixed_circuit(20, 38, 61, dense=0.2)
    small = H.mixed_circuit(12, 22, 62)
    for c, k, nb, opts in ((big, 6, 5, dict(max_tile_bits=12, reg_bits=4, math=2)), (small, 3, 2, None)):
        bits = W.random_bitstrings(c.n, nb, W.rng_for(410, c.n))
        got, ref = _both(Plan.from_circuit(c, opts), bits, k)
        assert np.array_equal(got, ref)


def test_noalloc_16bit_storage_and_groups():
    # 16-bit storage; and more batches than fit the scratch at once at
    # width 20 (they run in groups)
    from paper_2608_13110_amd import Plan, lib
    c = H.mixed_circuit(16, 30, 63, dense=0.2)
    bits = W.random_bitstrings(c.n, 3, W.rng_for(411, 1))
    got, ref = _both(Plan.from_circuit(c), bits, 4, storage=1)
    assert np.array_equal(got, ref)
    c = W.restrict(W.config_circuit(1), 22)  # d = 40: 2^20-entry tensors
    p = Plan.from_circuit(c)
    per = p.workspace_bytes(5, 1)
    nb = int(lib().tnc_noalloc_scratch_bytes() // per) + 2
    bits = W.random_bitstrings(c.n, nb, W.rng_for(411, 2))
    got, ref = _both(p, bits, 5)
    assert np.array_equal(got, ref)


def test_noalloc_needs_prepared_tables_and_bounds_its_scratch():
    from paper_2608_13110_amd import TNC_E_INVALID, TNC_E_NOMEM, Plan, TncError
    c = H.mixed_circuit(12, 22, 64)
    p = Plan.from_circuit(c)
    bits = torch.zeros((1, c.n), dtype=torch.uint8, device="cuda")
    with pytest.raises(TncError) as e:  # k = 2 never prepared: nothing may be uploaded here
        p.amplitudes_noalloc(bits, 2)
    assert e.value.code == TNC_E_INVALID
    big = W.brickwork_circuit(26, 48, 10, W.rng_for(412, 1))  # 2^24-entry tensor: above the scratch
    pb = Plan.from_circuit(big)
    pb.prepare(2)
    with pytest.raises(TncError) as e:
        pb.amplitudes_noalloc(torch.zeros((1, 26), dtype=torch.uint8, device="cuda"), 2)
    assert e.value.code == TNC_E_NOMEM
