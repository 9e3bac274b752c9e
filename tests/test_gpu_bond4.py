"""GPU parity of the bond-dimension-four path (Sec. 6.2, "Effect of bond
dimension"): generic Haar-random two-qubit entanglers, lowered to dense 4x4
updates of a (d-1)-slot temporal boundary tensor, or of the n-qubit state
when that is narrower, through the C ABI against the FP64 oracle.

Tolerance as for bond two: every amplitude within 1e-5 * max(|ref|, 2^(-n/2))
(complex64 updates, FP64 late phase).  Where no state vector fits (width 33,
n = 34) the circuit is a dressed-SWAP network, whose amplitudes the oracle
gives in closed form at any n (oracle.product_amplitudes).
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


def gpu_amps(plan, bits, **kw):
    print(f"  [gpu] bond-4 n={plan.n} d={plan.d} batches={len(bits)} {kw}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).cuda()
    out = plan.amplitudes(d, 0, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# the tile options the autotuner of the bond-4 workload chooses among
FULL_OPTIONS = dict(max_tile_bits=13, low_bits=5, reg_bits=4)

GENERIC = [
    # n, d, first parity, batches, options
    (2, 2, 1, 3, None),
    (3, 4, 0, 2, None),
    (6, 6, 1, 5, None),
    (9, 10, 0, 4, dict(max_tile_bits=6, low_bits=2, reg_bits=3)),
    (12, 12, 1, 4, dict(max_tile_bits=6, low_bits=1, reg_bits=5)),
    (16, 14, 0, 3, dict(max_tile_bits=7, low_bits=3, reg_bits=2)),
    (20, 18, 1, 2, None),
    (22, 22, 0, 2, dict(reg_bits=4, math=2)),
    (22, 20, 1, 2, FULL_OPTIONS),
    (24, 22, 0, 2, dict(max_tile_bits=12, reg_bits=4, reg_adapt=1)),
    (24, 24, 1, 2, dict(max_tile_bits=13, low_bits=5, reg_bits=5)),
    # matrix-core unit phases, in 64-thread-wave tiles and full-size tiles
    (20, 18, 1, 2, dict(max_tile_bits=9, low_bits=3, reg_bits=3, math=2)),
    (24, 22, 0, 2, dict(max_tile_bits=13, low_bits=4, reg_bits=4, math=2)),
    (22, 20, 1, 2, dict(max_tile_bits=13, low_bits=5, reg_bits=5, math=2)),
    # spatial sweeps (the n-qubit state is the narrower boundary)
    (2, 4, 1, 3, None),
    (5, 9, 0, 2, None),
    (12, 20, 1, 2, dict(max_tile_bits=6, low_bits=2, reg_bits=3)),
    (20, 26, 0, 2, FULL_OPTIONS),
]


@pytest.mark.parametrize("n,d,fp,nb,opt", GENERIC)
def test_generic_brickwork_matches_oracle(n, d, fp, nb, opt):
    from paper_2608_13110_amd import Plan
    c = W.generic_brickwork_circuit(n, d, W.rng_for(501, n, d, fp), first_parity=fp)
    p = Plan.from_circuit(c, opt)
    assert p.info(0)["bond"] == 4 and p.info(0)["width"] == (min(n, d - 1) if d % 2 == 0 else n)
    bits = W.random_bitstrings(n, nb, W.rng_for(502, n, d))
    ref = oracle.amplitudes(c, bits, 0)
    got = gpu_amps(p, bits)
    per, l2 = H.amp_errors(got, ref, n)
    assert per < H.TOL_C64, (per, l2)


@pytest.mark.parametrize("storage,tol", [(1, 1e-2), (2, 5e-2)])
def test_sixteen_bit_storage(storage, tol):
    from paper_2608_13110_amd import Plan
    c = W.generic_brickwork_circuit(16, 14, W.rng_for(503, storage))
    p = Plan.from_circuit(c, dict(max_tile_bits=7, low_bits=3, reg_bits=4))
    bits = W.random_bitstrings(16, 3, W.rng_for(504))
    ref = oracle.amplitudes(c, bits, 0)
    got = gpu_amps(p, bits, storage=storage)
    _, l2 = H.amp_errors(got, ref, 16)
    assert l2 < tol


def test_forced_bond_four_matches_bond_two():
    # CZ and rank-2 entanglers lowered both ways give the same amplitudes
    from paper_2608_13110_amd import Plan
    c = H.mixed_circuit(14, 12, 505, first_parity=1, dense=0.4)
    bits = W.random_bitstrings(14, 4, W.rng_for(506))
    ref = oracle.amplitudes(c, bits, 0)
    got4 = gpu_amps(Plan.from_circuit(c, dict(bond=4)), bits)
    got2 = gpu_amps(Plan.from_circuit(c), bits)
    assert H.amp_errors(got4, ref, 14)[0] < H.TOL_C64
    assert H.amp_errors(got2, ref, 14)[0] < H.TOL_C64


@pytest.mark.parametrize("math", [0, 2])
@pytest.mark.parametrize("n,d,nb", [(26, 26, 8), (34, 34, 1)])
def test_swap_network_at_width(n, d, nb, math):
    # width 25 with several batches, and the full width-33 workload of the
    # bench (2^33 complex64 entries, 64 GiB per batch) in its tile options,
    # with dense phases on the vector ALUs and with unit phases
    from paper_2608_13110_amd import Plan
    c = W.swap_network_circuit(n, d, W.rng_for(507, n, d), 1)
    p = Plan.from_circuit(c, dict(FULL_OPTIONS, math=math))
    assert p.info(0)["width"] == d - 1
    bits = W.random_bitstrings(n, nb, W.rng_for(508, n))
    ref = oracle.product_amplitudes(c, bits)
    got = gpu_amps(p, bits)[:, 0]
    per, l2 = H.amp_errors(got[:, None], ref[:, None], n)
    assert per < H.TOL_C64, (per, l2)
