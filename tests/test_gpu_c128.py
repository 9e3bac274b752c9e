"""The complex128 reference path on the GPU, and the paper's accuracy metric.

The reference path (tnc_debug_amplitudes_c128) applies every update of the
same plan in FP64 on a complex128 tensor, one launch per update, then the
same FP64 join and late phase.  It is pinned to the FP64 oracle on
restrictions, then used where no state vector fits: the complex64 path at
full n is compared with it by the total variation of the conditional
distributions p(b|a), the accuracy measure of Sec. 5.1.
"""
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


def _run(plan, bits, k, c128):
    print(f"  [gpu] {'c128' if c128 else 'c64'} n={plan.n} d={plan.d} k={k} batches={len(bits)}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).cuda()
    out = plan.debug_amplitudes_c128(d, k) if c128 else plan.amplitudes(d, k)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,d,fp,k", [(10, 20, 1, 0), (11, 21, 0, 3), (14, 28, 1, 5), (9, 19, 0, 2)])
def test_c128_path_matches_oracle_small(n, d, fp, k):
    from paper_2608_13110_amd import Plan
    c = H.mixed_circuit(n, d, 13 * n + d, first_parity=fp, dense=0.3)
    bits = W.random_bitstrings(n, 4, W.rng_for(413, n, d))
    got = _run(Plan.from_circuit(c), bits, k, True)
    ref = oracle.amplitudes(c, bits, k)
    per, _ = H.amp_errors(got, ref, n)
    assert per < 1e-11, per


def test_c128_path_matches_oracle_precision_restriction():
    # the precision shape (d = 56, w = 28) on 22 qubits: FP64 throughout
    from paper_2608_13110_amd import Plan
    c = W.restrict(W.config_circuit(2), 22)
    bits = W.config_bitstrings(2)[:2, :22]
    got = _run(Plan.from_circuit(c), bits, 8, True)
    ref = oracle.amplitudes(c, bits, 8)
    per, _ = H.amp_errors(got, ref, c.n)
    assert per < 1e-10, per


def test_c64_against_c128_at_full_n():
    # the precision workload itself (n = 70, d = 56, w = 28, 400 T, k = 8):
    # no state vector fits; the complex64 path against the complex128 one,
    # per amplitude and by the TV of p(b|a) (Sec. 5.1)
    from paper_2608_13110_amd import Plan
    c = W.config_circuit(2)
    bits = W.config_bitstrings(2)[:2]
    p = Plan.from_circuit(c)
    z64 = _run(p, bits, 8, False)
    z128 = _run(p, bits, 8, True)
    per, l2 = H.amp_errors(z64, z128, c.n)
    tv = oracle.tv_conditional(z64, z128)
    print(f"  c64 vs c128: per-amplitude {per:.2e}, l2 {l2:.2e}, TV of conditionals {tv.max():.2e}", flush=True)
    assert per < H.TOL_C64 and tv.max() < H.TOL_C64, (per, tv)
