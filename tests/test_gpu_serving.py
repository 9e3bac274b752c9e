"""GPU tests of the serving loop and the autotuner, through the C ABI.

Every served result must equal the same request run alone through
tnc_amplitudes (the same kernels and plan options, so bit for bit), and the
FP64 oracle within the complex64 tolerance.
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


def alone(req, storage=0):
    from paper_2608_13110_amd import Plan
    c = req["circuit"]
    bits = torch.from_numpy(np.ascontiguousarray(req["bits"], dtype=np.uint8)).cuda()
    out = Plan.from_circuit(c).amplitudes(bits, req["k"], storage=storage)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def small_stream(count, seed):
    return W.serving_requests(count=count, seed=seed, n_range=(12, 20), d_range=(12, 30), k_max=6)


def test_served_mix_equals_alone_and_oracle():
    from paper_2608_13110_amd import Server
    reqs = small_stream(12, 7)
    ref = [alone(r) for r in reqs]
    with Server(arena_bytes=1 << 30, n_streams=4, n_planners=4, small_bits=16) as srv:
        for rnd in range(2):  # the second round replays the captured graphs
            print(f"  [gpu] served round {rnd}: {len(reqs)} requests", flush=True)
            ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
            for r, rid, z in zip(reqs, ids, ref):
                got, st = srv.wait(rid)
                assert np.array_equal(got, z), (r["id"], rnd)
                assert st["total_ms"] >= st["run_ms"] >= 0.0
        summ = srv.summary()
    assert summ["completed"] == 2 * len(reqs)
    assert summ["plan_cache_hits"] >= len(reqs)
    assert summ["graph_launches"] + summ["plain_launches"] == 2 * len(reqs)
    assert summ["graph_failures"] == 0
    assert summ["graph_launches"] >= len(reqs)  # every second-round request replays its graph
    assert summ["latency_ms_p99"] >= summ["latency_ms_p50"] > 0.0
    for r, z in zip(reqs, ref):
        o = oracle.amplitudes(r["circuit"], r["bits"], r["k"])
        per, l2 = H.amp_errors(z, o, r["circuit"].n)
        assert per < H.TOL_C64, (r["id"], per)


def test_served_requests_overlap_and_respect_the_arena():
    # an arena that holds one of the largest requests (or a few smaller
    # ones) at once: requests wait for memory, none fails, every result is
    # still the alone result
    from paper_2608_13110_amd import Plan, Server
    reqs = W.serving_requests(count=8, seed=11, n_range=(22, 26), d_range=(36, 40), k_max=4)
    ref = [alone(r) for r in reqs]
    wss = [Plan.from_circuit(r["circuit"]).workspace_bytes(r["k"], 1) for r in reqs]
    arena = int(1.5 * max(wss)) + (16 << 20)
    with Server(arena_bytes=arena, n_streams=4, n_planners=2, small_bits=0) as srv:
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
        for rid, z in zip(ids, ref):
            got, st = srv.wait(rid)
            assert np.array_equal(got, z)
            assert st["mode"] == 0
        summ = srv.summary()
    assert summ["completed"] == len(reqs)
    # never more requests in flight than the arena holds
    assert 1 <= summ["max_inflight"] <= min(4, arena // min(wss))


def test_served_storage_modes_and_batches():
    from paper_2608_13110_amd import Server
    reqs = small_stream(4, 13)
    with Server(arena_bytes=1 << 29, n_streams=2, small_bits=16) as srv:
        for r in reqs:
            bits = W.random_bitstrings(r["circuit"].n, 3, W.rng_for(407, r["id"]))
            for storage in (0, 1):
                rr = dict(r, bits=bits)
                z = alone(rr, storage)
                got, _ = srv.wait(srv.submit(r["circuit"], bits, r["k"], storage))
                assert np.array_equal(got, z)


def test_autotune_picks_a_candidate():
    from paper_2608_13110_amd import autotune
    cands = [dict(), dict(max_tile_bits=12), dict(max_tile_bits=12, reg_bits=4), dict(max_tile_bits=10, reg_bits=4)]
    best, times = autotune(24, 36, 4, cands, reps=2)
    assert 0 <= best < len(cands)
    assert np.all(np.isfinite(times)) and times[best] == times.min()


def test_served_with_tuned_option_forms():
    # the tuner's table may pick fused matrix-core phases or the prefetching
    # blocks per width: served results still equal the same plan options run
    # alone (bit for bit) and the oracle
    from paper_2608_13110_amd import Plan, Server
    reqs = W.serving_requests(count=6, seed=17, n_range=(16, 20), d_range=(24, 30), k_max=4)
    tuning = {}
    for r in reqs:
        h = (r["circuit"].d + 1) // 2
        tuning[h] = dict(math=2) if h % 2 == 0 else dict(max_tile_bits=12, reg_bits=4, math=2)
    with Server(arena_bytes=1 << 30, n_streams=2, n_planners=2, small_bits=16) as srv:
        for h, o in tuning.items():
            srv.set_tuning(h, o)
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
        for r, rid in zip(reqs, ids):
            got, _ = srv.wait(rid)
            h = (r["circuit"].d + 1) // 2
            bits = torch.from_numpy(np.ascontiguousarray(r["bits"], dtype=np.uint8)).cuda()
            alone_z = Plan.from_circuit(r["circuit"], tuning[h]).amplitudes(bits, r["k"])
            torch.cuda.synchronize()
            assert np.array_equal(got, alone_z.cpu().numpy()), r["id"]
            o = oracle.amplitudes(r["circuit"], r["bits"], r["k"])
            per, _ = H.amp_errors(got, o, r["circuit"].n)
            assert per < H.TOL_C64, (r["id"], per)


def test_small_requests_of_one_width_run_grouped():
    # many small requests of one width queued behind a single stream: the
    # dispatcher takes them as groups, merges their launches into grouped
    # launches, and every result is still the alone result bit for bit (the
    # grouped kernels run the same code on the same arguments) and the
    # oracle's within the complex64 tolerance
    from paper_2608_13110_amd import Server
    reqs = []
    for i, (n, k) in enumerate([(12, 0), (14, 3), (16, 5), (13, 2), (18, 4), (15, 1), (12, 6), (17, 3)]):
        c = H.mixed_circuit(n, 24, 500 + i, dense=0.2)
        bits = W.random_bitstrings(n, 1 + i % 3, W.rng_for(409, i))
        reqs.append(dict(id=i, circuit=c, bits=bits, k=k))
    ref = [alone(r) for r in reqs]
    # a batching window long enough for every request to be planned
    with Server(arena_bytes=1 << 30, n_streams=1, n_planners=4, small_bits=16, max_group=8,
                group_window_us=2000000) as srv:
        print(f"  [gpu] grouped: {len(reqs)} requests of width 12", flush=True)
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
        modes = []
        for r, rid, z in zip(reqs, ids, ref):
            got, st = srv.wait(rid)
            assert np.array_equal(got, z), r["id"]
            modes.append(st["mode"])
        summ = srv.summary()
    assert summ["completed"] == len(reqs)
    assert summ["groups"] >= 1 and summ["grouped_requests"] >= 2 and summ["grouped_launches"] >= 1, summ
    assert modes.count(2) == summ["grouped_requests"]
    for r, z in zip(reqs, ref):
        o = oracle.amplitudes(r["circuit"], r["bits"], r["k"])
        per, _ = H.amp_errors(z, o, r["circuit"].n)
        assert per < H.TOL_C64, (r["id"], per)


def test_grouping_disabled_runs_each_request_alone():
    from paper_2608_13110_amd import Server
    reqs = small_stream(5, 23)
    ref = [alone(r) for r in reqs]
    with Server(arena_bytes=1 << 29, n_streams=1, small_bits=16, max_group=1) as srv:
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
        for rid, z in zip(ids, ref):
            got, st = srv.wait(rid)
            assert np.array_equal(got, z) and st["mode"] != 2
        assert srv.summary()["groups"] == 0
