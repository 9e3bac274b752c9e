"""Bond-dimension-four lowering (Sec. 6.2, "Effect of bond dimension") on the
CPU: the constructive width and the path estimate the paper prints, the
plan's own tables executed on the host in FP64, and the device tables run
through the host emulation of the pass kernel (dense 4x4 phases), all
against the oracle on generic-unitary brickworks."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2608_13110_amd import Plan
from tests import helpers as H

# (n, d, first parity): temporal sweeps (n >= d - 1, even d) with both cut
# types at the top, from rows of one crossing (d = 2) up to several passes
# per row; spatial sweeps (n < d - 1, or n <= d at odd d), n = 2 included
GENERIC = [(2, 2, 1), (2, 2, 0), (3, 2, 1), (3, 4, 0), (4, 4, 1), (5, 6, 0), (6, 6, 1), (7, 8, 0),
           (8, 8, 1), (9, 10, 0), (10, 6, 1), (12, 12, 0), (16, 14, 1),
           (2, 4, 1), (2, 3, 0), (3, 6, 0), (5, 8, 1), (4, 9, 0), (7, 7, 1), (9, 13, 0), (12, 20, 1)]

TILES = [dict(max_tile_bits=6, low_bits=2, reg_bits=3), dict(max_tile_bits=6, low_bits=1, reg_bits=5),
         dict(max_tile_bits=7, low_bits=3, reg_bits=2), dict(max_tile_bits=8, low_bits=4, reg_bits=4), None,
         dict(max_tile_bits=7, low_bits=2, reg_bits=4, math=2),
         dict(max_tile_bits=8, low_bits=3, reg_bits=4, reg_adapt=1),
         # matrix-core unit phases (a wavefront step as one 8x8)
         dict(max_tile_bits=9, low_bits=3, reg_bits=3, math=2),
         dict(max_tile_bits=10, low_bits=3, reg_bits=4, math=2)]


@pytest.mark.parametrize("n", [3, 8, 12, 20])
def test_width_matches_the_bond_four_construction(n):
    # Sec. 6.2: W = min(n, d-1) for even d and min(n, d) for odd d (odd d
    # with n > d, the temporal sweep of odd depth, is not lowered)
    for d in range(2, 2 * n + 3):
        if d % 2 and n > d:
            continue
        p = Plan.from_circuit(W.generic_brickwork_circuit(n, d, W.rng_for(401, n, d)))
        inf = p.info(0)
        assert inf["bond"] == 4
        assert inf["width"] == (min(n, d - 1) if d % 2 == 0 else min(n, d)), (n, d)


def test_cost_point_matches_paper():
    # Sec. 6.2: (W, log2 C) = (69, 83.19) for the chi=4 path at n = d = 70
    # (planned only: a 2^69-entry tensor is far beyond one device)
    p = Plan.from_circuit(W.generic_brickwork_circuit(70, 70, W.rng_for(402, 1)))
    inf = p.info(0)
    assert inf["bond"] == 4
    assert inf["width"] == 69
    assert abs(inf["log2_cost"] - 83.19) < 0.01
    assert inf["workspace_per_batch"] == 0


@pytest.mark.parametrize("n,d,fp", GENERIC)
def test_host_execution_matches_oracle(n, d, fp):
    c = W.generic_brickwork_circuit(n, d, W.rng_for(403, n, d, fp), first_parity=fp)
    p = Plan.from_circuit(c)
    bits = W.random_bitstrings(n, 6, W.rng_for(404, n, d))
    ref = oracle.amplitudes(c, bits, 0)
    got = p.debug_execute_host(bits, 0)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("opt", TILES)
@pytest.mark.parametrize("n,d,fp", [(12, 12, 1), (16, 14, 0), (13, 16, 1), (20, 18, 0), (12, 20, 1), (15, 17, 0)])
def test_device_emulation_matches_oracle(n, d, fp, opt):
    c = W.generic_brickwork_circuit(n, d, W.rng_for(405, n, d, fp), first_parity=fp)
    p = Plan.from_circuit(c, opt)
    bits = W.random_bitstrings(n, 4, W.rng_for(406, n, d))
    ref = oracle.amplitudes(c, bits, 0)
    got = p.debug_emulate_device(bits, 0)
    per, l2 = H.amp_errors(got, ref, n)
    assert per < H.TOL_C64, (per, l2)


def test_unit_phases_are_planned_with_matrix_cores():
    c = W.generic_brickwork_circuit(20, 18, W.rng_for(407, 2))
    p = Plan.from_circuit(c, dict(max_tile_bits=10, low_bits=3, reg_bits=4, math=2))
    assert sum(q["fused_phases"] for q in p.passes(0)) > 0
    p0 = Plan.from_circuit(c, dict(max_tile_bits=10, low_bits=3, reg_bits=4))
    assert sum(q["fused_phases"] for q in p0.passes(0)) == 0


def test_dense_phases_hold_one_or_two_updates():
    c = W.generic_brickwork_circuit(20, 18, W.rng_for(407, 1))
    for opt in TILES:
        p = Plan.from_circuit(c, opt)
        for ps in p.passes(0):
            assert ps["phases"] >= 1
        # every pass of a bond-4 plan is planned (the tables are validated
        # against the kernel forms when the info is built)
        assert p.info(0)["n_passes"] == len(p.passes(0))


def test_forced_bond_four_on_rank_two_entanglers():
    # the bond-4 lowering holds any entangler; on CZ / rank-2 gates it must
    # give the same amplitudes as the bond-2 one
    c = H.mixed_circuit(10, 10, 77, first_parity=0, dense=0.5)
    bits = W.random_bitstrings(10, 4, W.rng_for(408))
    ref = oracle.amplitudes(c, bits, 0)
    p4 = Plan.from_circuit(c, dict(bond=4))
    assert p4.info(0)["bond"] == 4 and p4.info(0)["width"] == 9
    assert np.max(np.abs(p4.debug_execute_host(bits, 0) - ref)) < 1e-12
    per, _ = H.amp_errors(p4.debug_emulate_device(bits, 0), ref, 10)
    assert per < H.TOL_C64


@pytest.mark.parametrize("storage", [1, 2])
def test_sixteen_bit_storage_emulation(storage):
    c = W.generic_brickwork_circuit(12, 12, W.rng_for(409, storage))
    bits = W.random_bitstrings(12, 4, W.rng_for(410))
    ref = oracle.amplitudes(c, bits, 0)
    p = Plan.from_circuit(c, dict(max_tile_bits=6, low_bits=2, reg_bits=4))
    got = p.debug_emulate_device(bits, 0, storage=storage)
    _, l2 = H.amp_errors(got, ref, 12)
    assert l2 < (1e-2 if storage == 1 else 5e-2)


def test_swap_network_through_the_bond_four_path():
    # the dressed-SWAP family used for full-width checks on the device, at an
    # emulated size
    c = W.swap_network_circuit(18, 16, W.rng_for(415), 1)
    bits = W.random_bitstrings(18, 6, W.rng_for(416))
    ref = oracle.product_amplitudes(c, bits)
    p = Plan.from_circuit(c, dict(max_tile_bits=8, low_bits=3, reg_bits=4))
    assert p.info(0)["bond"] == 4
    got = p.debug_emulate_device(bits, 0)[:, 0]
    per, _ = H.amp_errors(got[:, None], ref[:, None], 18)
    assert per < H.TOL_C64
