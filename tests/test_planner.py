"""Planner checks on the CPU: the paper's width, cost and partition claims,
invariance, error handling, and the lowering itself (the plan's own tables
executed on the host in FP64, and the device tables run through a host
emulation of the pass kernel's thread/LDS mapping) against the oracle."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2608_13110_amd import EXPORTED, TNC_E_DOMAIN, TNC_E_INVALID, TNC_E_RANK, Plan, TncError, lib
from tests import helpers as H
from tests.pinlib import tableau

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_header_symbol():
    L = lib()
    syms = H.header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    assert set(EXPORTED) == set(syms)


@pytest.mark.parametrize("n", [4, 5, 8, 12])
def test_width_matches_prop_constructive_memory(n):
    # Prop. constructive-memory: W = ceil(d/2) for n >= 4, 7 <= d <= 2n;
    # Prop. batched width: the same for 1 <= k <= floor(d/4).
    for d in range(7, 2 * n + 1):
        p = Plan.from_circuit(W.brickwork_circuit(n, d, 1, W.rng_for(301, n, d)))
        assert p.info(0)["width"] == math.ceil(d / 2)
        for k in range(1, min(d // 4, n - 1) + 1):
            assert p.info(k)["width"] == math.ceil(d / 2)


def test_cost_point_matches_paper():
    # Sec. 6.2 / 6.3: (W, log2 C) = (35, 48.22) for the open chi=2 path at n=d=70
    p = Plan.from_circuit(W.brickwork_circuit(70, 70, 468, W.rng_for(302, 1)))
    inf = p.info(0)
    assert inf["width"] == 35
    assert abs(inf["log2_cost"] - 48.22) < 0.05


def test_partition_example_matches_paper():
    # Sec. 4.3, figure fig:batched-regions: n=d=10, k=2
    p = Plan.from_circuit(W.brickwork_circuit(10, 10, 4, W.rng_for(303, 1)))
    inf = p.info(2)
    assert (inf["fixed_rows"], inf["early_layers"], inf["late_layers"]) == (8, 4, 6)


def test_width_and_cost_do_not_depend_on_gate_values():
    # Sec. 1: absorbing one-qubit gates leaves the shape of the network as
    # it is, so the planned width and cost must not move when the gate
    # values change or when T gates are added, removed or moved.
    ref = None
    for seed, nt in [(1, 0), (2, 30), (3, 300), (4, 700)]:
        c = W.brickwork_circuit(40, 33, nt, W.rng_for(304, seed))
        if seed == 4:
            c = W.with_gate_values(c, W.rng_for(304, 9))
        sig = [Plan.from_circuit(c).info(k) for k in (0, 3, 8)]
        if ref is None:
            ref = sig
        assert sig == ref


def test_rank_and_domain_errors():
    c = W.brickwork_circuit(6, 6, 0, W.rng_for(305, 1))
    z = W.rng_for(305, 2).normal(size=(4, 4)) + 1j * W.rng_for(305, 3).normal(size=(4, 4))
    u = np.linalg.qr(z)[0]
    bad = list(c.gates)
    bad[0] = (bad[0][0], bad[0][1], W.GATE_DENSE4, u)
    # a rank-4 entangler: refused under bond dimension 2, lowered with bond
    # dimension 4 otherwise (even depth, k = 0 only; Sec. 6.2)
    with pytest.raises(TncError) as e:
        Plan(c.n, c.d, c.one_qubit, bad, options=dict(bond=2))
    assert e.value.code == TNC_E_RANK
    p4 = Plan(c.n, c.d, c.one_qubit, bad)
    assert p4.info(0)["bond"] == 4 and p4.info(0)["width"] == c.d - 1
    with pytest.raises(TncError) as e:
        p4.info(1)
    assert e.value.code == TNC_E_DOMAIN
    # odd depth: the spatial sweep covers n <= d; n > d is not lowered
    c7 = W.brickwork_circuit(9, 7, 0, W.rng_for(305, 4))
    bad7 = list(c7.gates)
    bad7[0] = (bad7[0][0], bad7[0][1], W.GATE_DENSE4, u)
    with pytest.raises(TncError) as e:
        Plan(c7.n, c7.d, c7.one_qubit, bad7)
    assert e.value.code == TNC_E_DOMAIN
    with pytest.raises(TncError) as e:
        Plan(c.n, c.d, c.one_qubit, list(c.gates), options=dict(bond=3))
    assert e.value.code == TNC_E_INVALID
    off = list(c.gates) + [(1, 0, W.GATE_CZ, None)] if c.gates[0][1] == 1 else list(c.gates) + [(1, 1, W.GATE_CZ, None)]
    with pytest.raises(TncError) as e:
        Plan(c.n, c.d, c.one_qubit, off)
    assert e.value.code == TNC_E_INVALID
    p = Plan.from_circuit(c)
    for k in (-1, 4, 6):
        with pytest.raises(TncError) as e:
            p.info(k)
        assert e.value.code == TNC_E_DOMAIN
    with pytest.raises(TncError) as e:
        Plan(3, 1, np.zeros((2, 3, 2, 2)), [])
    assert e.value.code == TNC_E_DOMAIN


def test_width_limits():
    # bond two: widths up to 40 are planned (a 2^40-entry tensor is the
    # device limit), wider ones refused; bond four: widths up to 69 are
    # planned, above 40 for the path estimate only (no workspace)
    ok = Plan.from_circuit(W.brickwork_circuit(82, 80, 4, W.rng_for(309, 1)))
    assert ok.info(0)["width"] == 40 and ok.info(0)["workspace_per_batch"] > 0
    with pytest.raises(TncError) as e:
        Plan.from_circuit(W.brickwork_circuit(84, 82, 4, W.rng_for(309, 2)))
    assert e.value.code == TNC_E_DOMAIN
    p4 = Plan.from_circuit(W.generic_brickwork_circuit(44, 44, W.rng_for(309, 3)))
    assert p4.info(0)["width"] == 43 and p4.info(0)["workspace_per_batch"] == 0
    with pytest.raises(TncError) as e:
        p4.workspace_bytes(0, 1)
    assert e.value.code == TNC_E_DOMAIN
    with pytest.raises(TncError) as e:
        Plan.from_circuit(W.generic_brickwork_circuit(72, 72, W.rng_for(309, 4)))
    assert e.value.code == TNC_E_DOMAIN


CASES = [(2, 2, 1), (2, 5, 0), (3, 2, 0), (3, 7, 1), (4, 4, 0), (5, 6, 1), (6, 7, 0), (7, 8, 1),
         (8, 9, 0), (9, 12, 1), (10, 15, 0), (12, 12, 1), (13, 20, 0)]


@pytest.mark.parametrize("n,d,fp", CASES)
@pytest.mark.parametrize("dense", [0.0, 0.5])
def test_host_execution_matches_oracle(n, d, fp, dense):
    c = H.mixed_circuit(n, d, 100 * n + d, first_parity=fp, dense=dense)
    p = Plan.from_circuit(c)
    psi = oracle.statevector(c)
    bits = W.random_bitstrings(n, 5, W.rng_for(306, n, d))
    for k in range(0, min(n - 1, d // 2, 8) + 1):
        ref = oracle.amplitudes(c, bits, k, psi=psi)
        got = p.debug_execute_host(bits, k)
        assert np.max(np.abs(got - ref)) < 1e-12, k


TILES = [dict(max_tile_bits=6, low_bits=2, reg_bits=3), dict(max_tile_bits=6, low_bits=1, reg_bits=5),
         dict(max_tile_bits=7, low_bits=3, reg_bits=2), dict(max_tile_bits=8, low_bits=4, reg_bits=4), None,
         # late removals folded into the join launch (the default for large tensors:
         # 3 from 2^26 entries, 5 from 2^30, 7 at 2^35)
         dict(late_fold=3), dict(late_fold=1, max_tile_bits=8, low_bits=3, reg_bits=4),
         dict(late_fold=5), dict(late_fold=7, max_tile_bits=8, low_bits=4, reg_bits=4, math=2),
         # passes narrowed to reg_bits - 1 where that costs no phase
         dict(reg_adapt=1, max_tile_bits=8, low_bits=4, reg_bits=5),
         dict(reg_adapt=1, max_tile_bits=9, low_bits=3, reg_bits=4, math=2),
         # runs of three updates fused into 8x8 products on the matrix cores
         dict(math=2, max_tile_bits=9, low_bits=3, reg_bits=3), dict(math=2, max_tile_bits=10, low_bits=4, reg_bits=4),
         dict(math=2, max_tile_bits=11, low_bits=4, reg_bits=5, late_fold=3)]


@pytest.mark.parametrize("opts", TILES)
@pytest.mark.parametrize("n,d,fp", [(10, 20, 0), (11, 21, 1), (12, 24, 1), (9, 19, 0)])
def test_device_emulation_matches_oracle(opts, n, d, fp):
    c = H.mixed_circuit(n, d, 7 * n + d, first_parity=fp, dense=0.3)
    p = Plan.from_circuit(c, opts)
    psi = oracle.statevector(c)
    bits = W.random_bitstrings(n, 3, W.rng_for(307, n, d))
    for k in sorted({0, 1, d // 4, min(n - 1, d // 2, 6)}):
        ref = oracle.amplitudes(c, bits, k, psi=psi)
        got = p.debug_emulate_device(bits, k)
        per, l2 = H.amp_errors(got, ref, n)
        assert per < H.TOL_C64 and l2 < H.TOL_C64, (k, per, l2)


def test_device_emulation_large_tiles():
    # 2^14-entry tiles (512 threads of 32 entries) with 64-byte low runs
    c = H.mixed_circuit(17, 32, 171, dense=0.3)
    bits = W.random_bitstrings(17, 2, W.rng_for(311, 1))
    for k in (0, 4):
        ref = oracle.amplitudes(c, bits, k)
        got = Plan.from_circuit(c, dict(max_tile_bits=14, low_bits=3)).debug_emulate_device(bits, k)
        per, l2 = H.amp_errors(got, ref, 17)
        assert per < H.TOL_C64 and l2 < H.TOL_C64, (k, per, l2)


@pytest.mark.parametrize("n,d", [(30, 12), (40, 9), (24, 16)])
def test_emulation_matches_tableau_at_full_size(n, d):
    # T-free Clifford circuits at n beyond the state vector: |psi|^2 from the
    # lowering must equal the stabilizer-tableau probability.
    c = W.brickwork_circuit(n, d, 0, W.rng_for(308, n, d))
    _, words = W.clifford_table()
    tab = tableau.run_clifford(c, words)
    p = Plan.from_circuit(c, dict(max_tile_bits=6, low_bits=2, reg_bits=3))
    rng = W.rng_for(308, 1)
    xs = np.stack([tab.sample(rng) for _ in range(6)] + list(W.random_bitstrings(n, 6, rng)))
    got = p.debug_emulate_device(xs, 0)[:, 0]
    for x, a in zip(xs, got):
        pt = tab.prob(x)
        assert abs(abs(a) ** 2 - pt) <= 1e-5 * max(pt, 2.0 ** -n)


# 16-bit block-scaled storage in the host emulation: the error is the storage
# format's (FP16 keeps 11 significant bits, BF16 8), well above complex64's
# and well below O(1).  Bounds: measured errors of these circuits with a
# margin of about 2x.
@pytest.mark.parametrize("storage,bound", [(1, (1.5e-2, 6e-3)), (2, (1.2e-1, 5e-2))])
@pytest.mark.parametrize("opts,n,d,k", [
    (None, 14, 29, 2),
    (dict(max_tile_bits=10, low_bits=4, reg_bits=4), 16, 30, 4),
    (dict(max_tile_bits=8, low_bits=2, reg_bits=3), 12, 24, 4),
    (dict(max_tile_bits=6, low_bits=2, reg_bits=1), 10, 21, 1),
])
def test_emulated_block_scaled_storage(storage, bound, opts, n, d, k):
    c = H.mixed_circuit(n, d, 7 * n + d, dense=0.3)
    bits = W.random_bitstrings(n, 3, W.rng_for(309, n, d))
    ref = oracle.amplitudes(c, bits, k)
    got = Plan.from_circuit(c, opts).debug_emulate_device(bits, k, storage)
    per, l2 = H.amp_errors(got, ref, n)
    assert np.isfinite(got).all()
    assert per < bound[0] and l2 < bound[1], (per, l2)
    # and it is a real rounding error, not an exact result
    assert l2 > 1e-6


def test_block_scaled_storage_is_rejected_with_one_low_slot():
    c = H.mixed_circuit(14, 28, 98)
    p = Plan.from_circuit(c, dict(max_tile_bits=8, low_bits=1, reg_bits=3))
    with pytest.raises(TncError):
        p.debug_emulate_device(W.random_bitstrings(14, 1, W.rng_for(310)), 2, 1)


def test_fused_phases_restrictions():
    # the update forms are 0 (vector ALUs) and 2 (fused matrix-core phases);
    # any other value, and unknown option names, are rejected
    c = H.mixed_circuit(14, 28, 98)
    for bad in (1, 3, -1):
        with pytest.raises(TncError):
            Plan.from_circuit(c, dict(math=bad, max_tile_bits=10, reg_bits=4))
    with pytest.raises(ValueError):
        Plan.from_circuit(c, dict(math=2, max_tile_bits=10, reg_bits=4, pipeline=1))
    p = Plan.from_circuit(c, dict(math=2, max_tile_bits=10, low_bits=4, reg_bits=4))
    # with 16-bit storage the fused phases run on the decoded tile, to the
    # storage mode's own accuracy
    bits16 = W.random_bitstrings(14, 2, W.rng_for(312))
    per16, _ = H.amp_errors(p.debug_emulate_device(bits16, 2, 1), oracle.amplitudes(c, bits16, 2), 14)
    assert per16 < 2e-2
    # fused phases take over the first three updates of staircases of three
    # or more, and hold two targets in lane bits, so their staircases run up
    # to two updates longer: the same updates in fewer phases than the
    # vector-ALU plan, different FP32 rounding (so the fused path did run),
    # the same amplitudes
    q = Plan.from_circuit(c, dict(max_tile_bits=10, low_bits=4, reg_bits=4))
    base = q.info(2)
    assert p.info(2)["n_ops"] == base["n_ops"] and p.info(2)["n_phases"] < base["n_phases"]
    bits = W.random_bitstrings(14, 2, W.rng_for(313))
    a, b = p.debug_emulate_device(bits, 2), q.debug_emulate_device(bits, 2)
    assert not np.array_equal(a, b)
    per, l2 = H.amp_errors(a, b, 14)
    assert per < H.TOL_C64 and l2 < H.TOL_C64


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_serving_arena_allocator(seed):
    # the serving loop's first-fit device-arena allocator, on the host
    from paper_2608_13110_amd import _check
    _check(lib().tnc_debug_arena_check(seed, 5000))


def test_sampler_entry_points_validate_on_the_host():
    # argument errors come back as status codes before any device work
    L = lib()
    assert L.tnc_sample_batched(None, 0, 3, None, None, None, None) == 0
    assert L.tnc_sample_batched(None, 4, 11, None, None, None, None) == TNC_E_INVALID
    assert L.tnc_sample_batched(None, 4, 3, None, None, None, None) == TNC_E_INVALID
    assert L.tnc_frugal_accept(None, 0, 10, 2.0, None, None, None, None) == 0
    assert L.tnc_frugal_accept(None, 8, 10, 0.0, None, None, None, None) == TNC_E_INVALID
    assert L.tnc_frugal_accept(None, 8, 10, float("inf"), None, None, None, None) == TNC_E_INVALID
    assert L.tnc_frugal_accept(None, 8, 0, 2.0, None, None, None, None) == TNC_E_INVALID


def test_ring_slicing_matches_oracle_in_emulation():
    # the ring (Sec. 6.3) as the sum of its 2^m open-chain slices, emulated on
    # the host, against the oracle's ring state vector; and the slice count
    import oracle as O
    from paper_2608_13110_amd import RingPlan
    for n, d, k in [(6, 6, 0), (8, 8, 2), (10, 9, 2)]:
        c = W.ring_circuit(n, d, 4, W.rng_for(130, n, d))
        for cc in (c, W.with_gate_values(c, W.rng_for(131, n, d))):
            rp = RingPlan.from_circuit(cc, dict(max_tile_bits=6, low_bits=2, reg_bits=3))
            assert rp.info(k)["slices"] == 1 << sum(1 for g in cc.gates if g[1] == n - 1)
            bits = W.random_bitstrings(n, 3, W.rng_for(132, n))
            per, l2 = H.amp_errors(rp.debug_emulate_device(bits, k), O.amplitudes(cc, bits, k), n)
            assert per < H.TOL_C64 and l2 < H.TOL_C64, (n, d, k, per, l2)


def test_ring_rejects_bad_wrap_gates():
    from paper_2608_13110_amd import RingPlan
    c = W.ring_circuit(8, 8, 0, W.rng_for(133, 1))
    dense = [(l, q, W.GATE_DENSE4 if q == 7 else kind, np.eye(4, dtype=complex) if q == 7 else m)
             for (l, q, kind, m) in c.gates]
    with pytest.raises(TncError):
        RingPlan(c.n, c.d, c.one_qubit, dense)
    clash = list(c.gates) + [(2, 7, W.GATE_CZ, None)]  # layer 2 uses qubit 0 in the chain
    with pytest.raises(TncError):
        RingPlan(c.n, c.d, c.one_qubit, clash)


LDS_CASES = [(cid, o) for cid in (2, 4) for o in (None, dict(max_tile_bits=12, math=2), dict(reg_bits=4, math=2),
                                                   dict(max_tile_bits=13, low_bits=5, reg_bits=4, math=2),
                                                   dict(max_tile_bits=12, reg_adapt=1),
                                                   dict(max_tile_bits=14, low_bits=3))]
LDS_CASES += [(5, dict(max_tile_bits=13, low_bits=5, reg_bits=4, math=2)), (5, dict(max_tile_bits=12, math=2))]


@pytest.mark.parametrize("cid,opts", LDS_CASES)
def test_lds_placement_is_conflict_free(cid, opts):
    # every register phase of the precision, full-width and width-35 plans in
    # the tile options the benchmark chooses from: the 16 lanes of a bank
    # cycle of an 8-byte LDS access meet 16 different slots modulo 16, and
    # the 32 lanes of a 32-lane cycle 32 modulo 32 (late_fold = -1 only skips
    # the host fold of the join, which does not touch the pass tables)
    p = Plan.from_circuit(W.config_circuit(cid), dict(opts or {}, late_fold=-1))
    st = p.debug_lds_conflicts(8)
    assert st["phases"] > 100
    assert st["conflicted_16"] == 0 and st["conflicted_32"] == 0, st


def test_memory_cap_bounds_the_workspace():
    # tnc_options.mem_cap_bytes (the boundary's memory cap): a batch whose
    # workspace exceeds it is refused with TNC_E_NOMEM; below it the plan is
    # unchanged
    from paper_2608_13110_amd import TNC_E_NOMEM
    c = W.brickwork_circuit(16, 20, 8, W.rng_for(307, 1))
    free = Plan.from_circuit(c)
    per = free.workspace_bytes(3, 1)
    assert Plan.from_circuit(c, dict(mem_cap_bytes=per)).workspace_bytes(3, 4) == 4 * per
    with pytest.raises(TncError) as e:
        Plan.from_circuit(c, dict(mem_cap_bytes=per - 1)).workspace_bytes(3, 1)
    assert e.value.code == TNC_E_NOMEM
    bits = W.random_bitstrings(16, 3, W.rng_for(307, 2))
    capped = Plan.from_circuit(c, dict(mem_cap_bytes=per))
    assert np.array_equal(capped.debug_execute_host(bits, 3), free.debug_execute_host(bits, 3))
