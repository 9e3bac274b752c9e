#!/usr/bin/env python3
"""Benchmark of the temporal-boundary amplitude engine on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload full_width|precision]

A step is one pass of the whole hot path (row-0 build-up, the fixed sweep,
the join and the late phase) over one amplitude batch of the workload,
inputs resident in HBM.  Default workload: the one-GPU full-width shape
(n = 70, d = 66, w = 33: a 2^33-entry complex64 boundary tensor, 468 T gates,
k = 8 open legs -> 256 amplitudes per batch, 8 seeded bitstring batches used
round robin).  The precision shape (n = 70, d = 56, w = 28, 400 T, 16 batches)
is measured beside it.  Prints one JSON line.

`roofline` is for the dominant kernel (the sweep pass): algorithmic bytes per
launch (read + write of the 2^h complex64 boundary tensor) over its average
duration measured with HIP events on its launch stream; `traffic` is the
counter-based HBM bytes per launch recorded in profiles/ for the current
kernel source (null when absent or stale).  `cpu_baseline` times the oracle
(FP64 state vector) on a bounded restriction of the same circuit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 78.6    # non-packed FP32 (256 CU x 64 lanes x 2 x 2.4 GHz)
METRIC = "amplitudes/s and boundary-tensor HBM GB/s (% of peak) at w=28/33; p99 latency"

WORKLOADS = {
    "full_width": dict(cid=4, k=8, desc="full_width n=70 d=66 w=33 T=468 k=8 (2^33 c64 boundary), 1 batch/step"),
    "precision": dict(cid=2, k=8, desc="precision n=70 d=56 w=28 T=400 k=8 (2^28 c64 boundary), 1 batch/step"),
    # not the default: one batch needs 279 GB of the 288 GB of HBM
    "width35": dict(cid=5, k=8, desc="width35 n=70 d=70 w=35 T=468 k=8 (2^35 c64 boundary, 256 GiB), 1 batch/step"),
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "device_tables.hpp", "lds_layout.hpp"):
        with open(os.path.join(ROOT, "paper_2608_13110_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str):
    """HBM bytes per pass launch from the committed counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_pass_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


_T0 = time.time()


def log(msg: str):
    """A progress line on stderr (the JSON result line goes to stdout)."""
    print(f"[bench {time.time() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


# tile candidates the autotuner times for the large workloads
MAIN_CANDIDATES = [dict(), dict(max_tile_bits=12, math=2), dict(reg_bits=4, math=2),
                   dict(max_tile_bits=13, low_bits=5, reg_bits=4, math=2)]


def pass_classes(plan, k, launches, h, bytes_per_entry=8, flops_per_op=14.0):
    """Pass launches of the timed steps grouped by window class (low slots,
    window start, window length): count per batch, updates, phases, average
    ms, the fraction of the HBM peak (algorithmic bytes 2 * 2^h * entry
    bytes per launch) and the fraction of the FP32 vector peak (algorithmic
    flops: flops_per_op per entry and update, matrix-core work included)."""
    passes = plan.passes(k)
    ms = [m for c, m in launches if c == 1]
    if not passes or len(ms) % len(passes):
        return None
    groups = {}
    for i, m in enumerate(ms):
        p = passes[i % len(passes)]
        key = (p["low_bits"], p["win_lo"], p["win_len"])
        g = groups.setdefault(key, {"ms": [], "updates": p["updates"], "phases": p["phases"],
                                    "fused_phases": p["fused_phases"], "n": 0})
        g["ms"].append(m)
    for i, p in enumerate(passes):
        groups[(p["low_bits"], p["win_lo"], p["win_len"])]["n"] += 1
    nbytes = 2.0 * bytes_per_entry * (1 << h)
    out = []
    for key, g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["ms"])):
        avg = sum(g["ms"]) / len(g["ms"])
        ups = [q["updates"] for q in passes if (q["low_bits"], q["win_lo"], q["win_len"]) == key]
        phs = [q["phases"] for q in passes if (q["low_bits"], q["win_lo"], q["win_len"]) == key]
        flops = sum(ups) / len(ups) * flops_per_op * (1 << h)
        out.append({"window": list(key), "passes_per_batch": g["n"],
                    "updates_avg": round(sum(ups) / len(ups), 2), "phases_avg": round(sum(phs) / len(phs), 2),
                    "ms_avg": round(avg, 3), "hbm_frac": round(nbytes / (avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                    "alu_frac": round(flops / (avg / 1e3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4)})
    return out


def run_workload(name, steps, warmup, torch, W, Plan, profile_begin, profile_end, fixed=None):
    from paper_2608_13110_amd import autotune, profile_launches
    spec = WORKLOADS[name]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits_all = W.config_bitstrings(spec["cid"])
    options, tune_ms = (fixed or {}), None
    if fixed is None:
        best, times = autotune(circ.n, circ.d, k, MAIN_CANDIDATES, reps=1)
        options, tune_ms = MAIN_CANDIDATES[best], [round(float(t), 1) for t in times]
    t0 = time.time()
    plan = Plan.from_circuit(circ, options or None)
    plan.prepare(k)
    prep_s = time.time() - t0
    info = plan.info(k)
    dev_bits = torch.from_numpy(bits_all).cuda()
    out = torch.empty((len(bits_all), 1 << k), dtype=torch.complex128, device="cuda")
    ws = torch.empty(plan.workspace_bytes(k, 1), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(i):
        j = i % len(bits_all)
        plan.amplitudes(dev_bits[j:j + 1], k, out=out[j:j + 1], workspace=ws, stream=stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    profile_begin()
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(steps):
        evs[i][0].record(stream)
        step(warmup + i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    prof = profile_end()
    classes = pass_classes(plan, k, profile_launches(), info["boundary_bits"])
    lat_ms = [a.elapsed_time(b) for a, b in evs]
    amps = steps * (1 << k)
    pass_gbs = prof["pass_bytes"] / (prof["pass_ms"] / 1e3) / 1e9 if prof["pass_ms"] > 0 else 0.0
    h = info["boundary_bits"]
    # algorithmic FLOPs of the sweep: every update is a complex 2x2 on each
    # pair of entries, 14 real flops per entry
    sweep_flops = info["n_ops"] * 14.0 * (1 << h) * steps
    return dict(
        workload=spec["desc"], k=k, h=h, steps=steps, wall_s=wall, prep_s=prep_s,
        amplitudes_per_s=amps / wall, ms_per_step=1e3 * wall / steps,
        latency_ms_p50=pct(lat_ms, 50), latency_ms_p99=pct(lat_ms, 99),
        pass_launches=prof["pass_launches"], pass_ms=prof["pass_ms"], late_ms=prof["late_ms"],
        init_ms=prof["init_ms"], pass_gbs=pass_gbs, pass_bytes_per_launch=prof["pass_bytes"] / max(1, prof["pass_launches"]),
        pass_avg_ms=prof["pass_ms"] / max(1, prof["pass_launches"]),
        sweep_tflops=sweep_flops / (prof["pass_ms"] / 1e3) / 1e12 if prof["pass_ms"] > 0 else 0.0,
        n_passes=info["n_passes"], n_ops=info["n_ops"], log2_cost=info["log2_cost"],
        tile_options=options, autotune_ms=tune_ms, pass_classes=classes,
    )


def sampling_bench(torch, W, Plan, batches=16, M=10.0):
    """Samplers on the precision workload's batches (Sec. 4.1, Sec. 4.2):
    one batched sample per contraction (uniform prefix, suffix from p(b|a))
    and frugal rejection on the same amplitudes.  Reports samples per second
    of the whole path, the sampler kernel's time, and two Porter-Thomas
    checks: the mean |A Q_a - 1| against sqrt(2/(pi B)), and the frugal
    acceptance against (1 - e^-M)/M."""
    import math
    import numpy as np
    from paper_2608_13110_amd import frugal_accept, sample_batched
    spec = WORKLOADS["precision"]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits = torch.from_numpy(W.config_bitstrings(spec["cid"])[:batches]).cuda()
    rng = np.random.default_rng(707)
    u = torch.from_numpy(rng.random(batches)).cuda()
    uf = torch.from_numpy(rng.random(batches << k)).cuda()
    plan = Plan.from_circuit(circ)
    plan.prepare(k)
    ws = torch.empty(plan.workspace_bytes(k, 1), dtype=torch.uint8, device="cuda")
    out = torch.empty((batches, 1 << k), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    plan.amplitudes(bits[:1], k, out=out[:1], workspace=ws, stream=stream)
    sample_batched(out[:1], u[:1])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    sampler_ms = 0.0
    for i in range(batches):
        plan.amplitudes(bits[i:i + 1], k, out=out[i:i + 1], workspace=ws, stream=stream)
        e0.record(stream)
        b, q = sample_batched(out[i:i + 1], u[i:i + 1])
        e1.record(stream)
        e1.synchronize()
        sampler_ms += e0.elapsed_time(e1)
    wall = time.time() - t0
    b, q = sample_batched(out, u)
    acc, _ = frugal_accept(out, circ.n, M, uf)
    torch.cuda.synchronize()
    A_dev = np.abs(q.cpu().numpy() * 2.0 ** (circ.n - k) - 1.0)
    return {"workload": spec["desc"] + f", {batches} uniform prefixes",
            "batched_samples_per_s": round(batches / wall, 3),
            "sampler_kernel_us": round(1e3 * sampler_ms / batches, 2),
            "mean_abs_AQ_minus_1": round(float(A_dev.mean()), 4),
            "porter_thomas_mean_abs_AQ_minus_1": round(math.sqrt(2.0 / (math.pi * (1 << k))), 4),
            "frugal_M": M, "frugal_acceptance": round(float(acc.float().mean().item()), 4),
            "porter_thomas_acceptance": round((1.0 - math.exp(-M)) / M, 4)}


def ring_bench(torch, W, n=20, d=20, k=4):
    """A ring of n = d = 20 (Sec. 6.3) by slicing its d/2 wrap-pair CZ bonds:
    2^10 open-chain slices of width 10, summed on the device; one batch of
    2^k amplitudes after a warmup batch."""
    from paper_2608_13110_amd import RingPlan
    c = W.ring_circuit(n, d, n * d // 10, W.rng_for(150, n, d))
    bits = torch.from_numpy(W.random_bitstrings(n, 1, W.rng_for(151, n, d))).cuda()
    t0 = time.time()
    rp = RingPlan.from_circuit(c)
    plan_s = time.time() - t0
    info = rp.info(k, 1)
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    out = torch.empty((1, 1 << k), dtype=torch.complex128, device="cuda")
    rp.amplitudes(bits, k, out=out, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.time()
    rp.amplitudes(bits, k, out=out, workspace=ws)
    torch.cuda.synchronize()
    wall = time.time() - t0
    rp.close()
    return {"workload": f"ring n={n} d={d} T={n * d // 10} k={k}, 1 batch",
            "slices": info["slices"], "slice_width": info["width"], "plan_s": round(plan_s, 2),
            "s_per_batch": round(wall, 4), "amplitudes_per_s": round((1 << k) / wall, 2),
            "slices_per_s": round(info["slices"] / wall, 1)}


# The paper's steady-state time per contraction at this shape (n = d = 70,
# w = 35, k = 8) on one node of 8 H100s, the tensor sharded over them (Sec. 5.2)
PAPER_W35_S_PER_CONTRACTION_8XH100 = 32.16


def width35_bench(torch, W, Plan, profile_begin, profile_end, storage=0, ref=None):
    """One batch of the width-35 shape on this one GPU: the 2^35-entry
    tensor in place (256 GiB in complex64, 128 GiB in the 16-bit modes), the
    join output shrunk by folding seven late removals.  No warmup step (a
    second batch would double the time); the plan and its tables are prepared
    before the timed region.  ref: the complex64 amplitudes of the same batch
    (16-bit storage reports its error against them)."""
    spec = WORKLOADS["width35"]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits = torch.from_numpy(W.config_bitstrings(spec["cid"])[:1]).cuda()
    opts = dict(max_tile_bits=13, low_bits=5, reg_bits=4, math=2)
    t0 = time.time()
    plan = Plan.from_circuit(circ, opts)
    plan.prepare(k)
    prep_s = time.time() - t0
    info = plan.info(k)
    torch.cuda.empty_cache()
    ws_bytes = plan.workspace_bytes(k, 1, storage)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.empty((1, 1 << k), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    profile_begin()
    t0 = time.time()
    plan.amplitudes(bits, k, out=out, workspace=ws, storage=storage)
    torch.cuda.synchronize()
    wall = time.time() - t0
    prof = profile_end()
    del ws
    torch.cuda.empty_cache()
    z = out.cpu().numpy()
    r = {"workload": spec["desc"], "storage": ("c64", "f16_blockscale", "bf16_blockscale")[storage],
         "tile_options": opts, "s_per_batch": round(wall, 3),
         "amplitudes_per_s": round((1 << k) / wall, 3), "passes": info["n_passes"],
         "workspace_gb": round(ws_bytes / 1e9, 1), "prepare_s": round(prep_s, 1),
         "pass_gbs": round(prof["pass_bytes"] / (prof["pass_ms"] / 1e3) / 1e9, 1),
         "pass_avg_ms": round(prof["pass_ms"] / max(1, prof["pass_launches"]), 3),
         "late_ms": round(prof["late_ms"], 1),
         "paper_s_per_contraction_8xH100": PAPER_W35_S_PER_CONTRACTION_8XH100,
         "paper_amplitudes_per_s_8xH100": round((1 << k) / PAPER_W35_S_PER_CONTRACTION_8XH100, 3)}
    if ref is not None:
        r["max_rel_err_vs_c64"] = _rel_err(z, ref, circ.n)
    return r, z


def storage_modes(torch, W, Plan, profile_begin, profile_end, batches=16):
    """The precision workload's batches with complex64 storage and with the
    FP16 / BF16 block-scaled storage modes: throughput, pass bandwidth
    (algorithmic bytes of each mode) and p99 per batch, and each 16-bit
    mode's amplitude error against the complex64 result."""
    import numpy as np
    spec = WORKLOADS["precision"]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits = torch.from_numpy(W.config_bitstrings(spec["cid"])[:batches]).cuda()
    plan = Plan.from_circuit(circ)
    plan.prepare(k)
    stream = torch.cuda.current_stream()
    res, ref = {}, None
    for name, storage in (("c64", 0), ("f16_blockscale", 1), ("bf16_blockscale", 2)):
        ws = torch.empty(plan.workspace_bytes(k, 1, storage), dtype=torch.uint8, device="cuda")
        out = torch.empty((batches, 1 << k), dtype=torch.complex128, device="cuda")
        plan.amplitudes(bits[:1], k, out=out[:1], workspace=ws, stream=stream, storage=storage)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(batches)]
        profile_begin()
        t0 = time.time()
        for i in range(batches):
            evs[i][0].record(stream)
            plan.amplitudes(bits[i:i + 1], k, out=out[i:i + 1], workspace=ws, stream=stream, storage=storage)
            evs[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.time() - t0
        prof = profile_end()
        lat = [a.elapsed_time(b) for a, b in evs]
        z = out.cpu().numpy()
        r = {"amplitudes_per_s": round(batches * (1 << k) / wall, 3),
             "latency_ms_p50": round(pct(lat, 50), 3), "latency_ms_p99": round(pct(lat, 99), 3),
             "pass_gbs": round(prof["pass_bytes"] / (prof["pass_ms"] / 1e3) / 1e9, 1),
             "bytes_per_entry": 8 if storage == 0 else 4}
        if ref is None:
            ref = z
        else:
            floor = 2.0 ** (-circ.n / 2)
            r["max_rel_err_vs_c64"] = float(np.max(np.abs(z - ref) / np.maximum(np.abs(ref), floor)))
            r["l2_rel_err_vs_c64"] = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
        res[name] = r
        del ws
        torch.cuda.empty_cache()
    res["workload"] = WORKLOADS["precision"]["desc"].replace("1 batch/step", f"{batches} batches")
    return res


BOND4 = dict(n=34, d=34, desc="bond4 n=34 d=34 w=33 (2^33 c64 boundary), Haar-random two-qubit gates, "
                                "k=0, 1 batch/step")
BOND4_CANDIDATES = [dict(max_tile_bits=13, low_bits=5, reg_bits=4), dict(max_tile_bits=13, low_bits=5, reg_bits=5),
                    dict(max_tile_bits=13, low_bits=5, reg_bits=4, math=2),
                    dict(max_tile_bits=13, low_bits=4, reg_bits=4, math=2),
                    dict(max_tile_bits=13, low_bits=5, reg_bits=5, math=2)]


def bond4_bench(torch, W, Plan, profile_begin, profile_end, steps=3):
    """Entanglers of operator Schmidt rank 4 (Sec. 6.2, Effect of bond
    dimension): a generic-gate brickwork at n = d = 34 has a 33-slot boundary
    tensor (the same 64 GiB as the width-33 bond-2 workload), updated by
    dense 4x4s.  Tile options are picked by timing one batch of each
    candidate; then `steps` batches are timed.  Also reports the planner's
    (W, log2 C) at n = d = 70 (planned only) against the paper's (69, 83.19)."""
    from paper_2608_13110_amd import profile_launches
    circ = W.generic_brickwork_circuit(BOND4["n"], BOND4["d"], W.rng_for(34, 34, 1))
    bits = torch.from_numpy(W.random_bitstrings(circ.n, steps + 1, W.rng_for(34, 34, 2))).cuda()
    out = torch.empty((steps + 1, 1), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    tune = []
    ws = None
    for opt in BOND4_CANDIDATES:
        p = Plan.from_circuit(circ, opt or None)
        p.prepare(0)
        if ws is None or ws.numel() < p.workspace_bytes(0, 1):
            ws = None
            ws = torch.empty(p.workspace_bytes(0, 1), dtype=torch.uint8, device="cuda")
        p.amplitudes(bits[:1], 0, out=out[:1], workspace=ws, stream=stream)
        torch.cuda.synchronize()
        t0 = time.time()
        p.amplitudes(bits[:1], 0, out=out[:1], workspace=ws, stream=stream)
        torch.cuda.synchronize()
        tune.append(round(1e3 * (time.time() - t0), 1))
    best = min(range(len(tune)), key=lambda i: tune[i])
    options = BOND4_CANDIDATES[best]
    plan = Plan.from_circuit(circ, options or None)
    plan.prepare(0)
    info = plan.info(0)
    passes = plan.passes(0)
    dense = sum(q["updates"] for q in passes) - info["n_ops"]  # a dense update holds two table ops
    h = info["boundary_bits"]
    plan.amplitudes(bits[:1], 0, out=out[:1], workspace=ws, stream=stream)
    torch.cuda.synchronize()
    profile_begin()
    t0 = time.time()
    for i in range(steps):
        plan.amplitudes(bits[1 + i:2 + i], 0, out=out[1 + i:2 + i], workspace=ws, stream=stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    prof = profile_end()
    classes = pass_classes(plan, 0, profile_launches(), h, flops_per_op=15.0)
    pass_s = prof["pass_ms"] / 1e3
    # algorithmic FLOPs per entry: 30 for a dense 4x4 (4 complex products,
    # 3 complex sums), 14 for a 2x2
    flops = ((info["n_ops"] - dense) * 14.0 + dense * 30.0) * (1 << h) * steps
    pass_gbs = prof["pass_bytes"] / pass_s / 1e9 if pass_s > 0 else 0.0
    p70 = Plan.from_circuit(W.generic_brickwork_circuit(70, 70, W.rng_for(70, 70, 1))).info(0)
    del ws
    return {"workload": BOND4["desc"], "tile_options": options, "candidates": BOND4_CANDIDATES,
            "candidates_ms_per_batch": tune, "width": info["width"], "log2_cost": round(info["log2_cost"], 3),
            "passes": info["n_passes"], "dense_updates": dense, "updates": info["n_ops"],
            "s_per_batch": round(wall / steps, 3), "amplitudes_per_s": round(steps / wall, 4),
            "pass_avg_ms": round(prof["pass_ms"] / max(1, prof["pass_launches"]), 3),
            "pass_gbs": round(pass_gbs, 1), "hbm_frac": round(pass_gbs / HBM_PEAK_GBS, 4),
            "alu_tflops": round(flops / pass_s / 1e12, 2) if pass_s > 0 else None,
            "alu_frac": round(flops / pass_s / 1e12 / FP32_VALU_PEAK_TFLOPS, 4) if pass_s > 0 else None,
            "late_ms": round(prof["late_ms"] / steps, 1), "pass_classes": classes,
            "planned_n70_d70": {"width": p70["width"], "log2_cost": round(p70["log2_cost"], 3),
                                "paper": {"width": 69, "log2_cost": 83.19}}}


def storage_full_width(torch, W, Plan, profile_begin, profile_end, options):
    """One batch of the full-width workload (w = 33) in each storage mode,
    with the tile options the autotuner chose for complex64: time per batch,
    pass time and bandwidth (each mode's own algorithmic bytes), and the
    16-bit modes' error against the complex64 amplitudes."""
    spec = WORKLOADS["full_width"]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits = torch.from_numpy(W.config_bitstrings(spec["cid"])[:1]).cuda()
    plan = Plan.from_circuit(circ, options or None)
    plan.prepare(k)
    res, ref = {"workload": spec["desc"], "tile_options": options}, None
    for name, storage in (("c64", 0), ("f16_blockscale", 1), ("bf16_blockscale", 2)):
        torch.cuda.empty_cache()
        ws = torch.empty(plan.workspace_bytes(k, 1, storage), dtype=torch.uint8, device="cuda")
        out = torch.empty((1, 1 << k), dtype=torch.complex128, device="cuda")
        torch.cuda.synchronize()
        profile_begin()
        t0 = time.time()
        plan.amplitudes(bits, k, out=out, workspace=ws, storage=storage)
        torch.cuda.synchronize()
        wall = time.time() - t0
        prof = profile_end()
        z = out.cpu().numpy()
        r = {"s_per_batch": round(wall, 3), "amplitudes_per_s": round((1 << k) / wall, 3),
             "pass_avg_ms": round(prof["pass_ms"] / max(1, prof["pass_launches"]), 3),
             "pass_gbs": round(prof["pass_bytes"] / (prof["pass_ms"] / 1e3) / 1e9, 1),
             "late_ms": round(prof["late_ms"], 1)}
        if ref is None:
            ref = z
        else:
            r["max_rel_err_vs_c64"] = _rel_err(z, ref, circ.n)
            r["tv_conditional_vs_c64"] = float(_tv_conditional(z, ref).max())
        res[name] = r
        del ws
    torch.cuda.empty_cache()
    return res


TUNE_CANDIDATES = [dict(), dict(max_tile_bits=12), dict(max_tile_bits=12, reg_adapt=1),
                   dict(max_tile_bits=12, reg_bits=4), dict(max_tile_bits=11, reg_bits=4), dict(math=2),
                   dict(reg_bits=4, math=2)]


def serving_bench(torch, W, count=512, load=0.8):
    """The serving stream: Poisson arrivals of mixed-shape requests.

    Autotunes the tile options per width, measures sequential plain launches
    back to back (one request at a time on one stream, no graphs, no groups:
    the capacity C), then runs the same stream at arrival rate load x C twice:
    through the sequential path (a request starts when it has arrived and the
    previous one is done) and through the server.  Plans are prepared before
    either run (the server's by a warm-up pass); latency is arrival -> done.
    """
    import threading
    import numpy as np
    from paper_2608_13110_amd import Plan, Server, autotune
    reqs = W.serving_requests(count=count, seed=1)
    widths = sorted({(r["circuit"].d + 1) // 2 for r in reqs})
    tuning = {}
    for h in widths:
        best, times = autotune(40, 2 * h, 4, TUNE_CANDIDATES, reps=2)
        tuning[h] = TUNE_CANDIDATES[best]
    # sequential plain launches with the same tuned plans
    plans = [Plan.from_circuit(r["circuit"], tuning[(r["circuit"].d + 1) // 2]) for r in reqs]
    for p_, r in zip(plans, reqs):
        p_.prepare(r["k"])
    stream = torch.cuda.current_stream()

    def run_one(p_, r):
        bits = torch.from_numpy(np.ascontiguousarray(r["bits"], dtype=np.uint8)).cuda()
        out = p_.amplitudes(bits, r["k"], stream=stream)
        return out.cpu()

    log("serving: sequential capacity")
    service = []
    for p_, r in zip(plans, reqs):
        t0 = time.perf_counter()
        run_one(p_, r)
        service.append(time.perf_counter() - t0)
    seq_total = sum(service)
    amps = sum(1 << r["k"] for r in reqs)
    capacity = count / seq_total
    rate = load * capacity
    gaps = np.array([r["arrival"] for r in reqs])
    arrivals = gaps / gaps[-1] * (count / rate)
    # the sequential path under the same arrivals, measured
    log(f"serving: sequential under arrivals at {rate:.0f} requests/s")
    seq_lat = []
    t0 = time.perf_counter()
    for p_, r, a in zip(plans, reqs, arrivals):
        dt = a - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        run_one(p_, r)
        seq_lat.append(1e3 * (time.perf_counter() - t0 - a))
    seq_arr_s = time.perf_counter() - t0
    del plans
    torch.cuda.empty_cache()
    with Server(arena_bytes=16 << 30, n_streams=8, n_planners=8, small_bits=20) as srv:
        for h, o in tuning.items():
            srv.set_tuning(h, o)
        log("serving: server warm-up")
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]  # warm-up: plans, graphs
        for i in ids:
            srv.wait(i)
        warm = srv.summary()
        res = [None] * count
        submit_t = [0.0] * count

        def producer(t0):
            for i, (r, a) in enumerate(zip(reqs, arrivals)):
                dt = a - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                submit_t[i] = time.perf_counter() - t0 - a
                res[i] = srv.submit(r["circuit"], r["bits"], r["k"])

        log("serving: served under arrivals")
        t0 = time.perf_counter()
        th = threading.Thread(target=producer, args=(t0,))
        th.start()
        lat = []
        for i in range(count):
            while res[i] is None:
                time.sleep(1e-4)
            _, st = srv.wait(res[i])
            # arrival -> done: the producer's own lateness plus submit -> done
            lat.append(1e3 * submit_t[i] + st["total_ms"])
        th.join()
        served_s = time.perf_counter() - t0
        summ = srv.summary()
        # saturated: the whole stream at once (capacity of the served path)
        log("serving: saturated")
        t1 = time.perf_counter()
        ids = [srv.submit(r["circuit"], r["bits"], r["k"]) for r in reqs]
        for i in ids:
            srv.wait(i)
        sat_s = time.perf_counter() - t1
        sat = srv.summary()

    def delta(a, b, key):
        return b[key] - a[key]

    return {
        "workload": f"{count} Poisson requests, n in 24..56, even d in 20..48 (w 10..24), k in 0..8, "
                    f"1 bitstring each; arrival rate {load} x sequential capacity",
        "amplitudes": amps,
        "sequential": {"amplitudes_per_s": round(amps / seq_arr_s, 1), "requests_per_s": round(count / seq_arr_s, 1),
                       "capacity_requests_per_s": round(capacity, 1),
                       "latency_ms_p50": round(pct(seq_lat, 50), 3), "latency_ms_p99": round(pct(seq_lat, 99), 3)},
        "served": {"amplitudes_per_s": round(amps / served_s, 1), "requests_per_s": round(count / served_s, 1),
                   "latency_ms_p50": round(pct(lat, 50), 3), "latency_ms_p99": round(pct(lat, 99), 3),
                   "max_inflight": summ["max_inflight"], "graph_failures": summ["graph_failures"],
                   "graph_launches": delta(warm, summ, "graph_launches"),
                   "plain_launches": delta(warm, summ, "plain_launches"),
                   "groups": delta(warm, summ, "groups"), "grouped_requests": delta(warm, summ, "grouped_requests")},
        "saturated": {"amplitudes_per_s": round(amps / sat_s, 1), "requests_per_s": round(count / sat_s, 1),
                      "vs_sequential": round(seq_total / sat_s, 3),
                      "groups": delta(summ, sat, "groups"), "grouped_requests": delta(summ, sat, "grouped_requests"),
                      "grouped_launches": delta(summ, sat, "grouped_launches"),
                      "graph_launches": delta(summ, sat, "graph_launches")},
        "tuning": {str(h): o for h, o in tuning.items()},
    }


def _tv_conditional(za, zb):
    """Per-batch TV between the conditional distributions p(b|a) of two
    amplitude batches (rows), the accuracy measure of Sec. 5.1; zb is the
    reference.  A prefix a of probability zero (exact zeros of near-Clifford
    circuits, held as rounding residue) has no conditional distribution: rows
    whose reference mass is below 1e-10 of the largest row's are left out."""
    import numpy as np
    pa = np.abs(za) ** 2
    pb = np.abs(zb) ** 2
    mb = pb.sum(axis=1)
    keep = mb > 1e-10 * mb.max()
    pa = pa[keep] / pa[keep].sum(axis=1, keepdims=True)
    pb = pb[keep] / mb[keep][:, None]
    return 0.5 * np.abs(pa - pb).sum(axis=1)


def _rel_err(got, ref, n):
    import numpy as np
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 ** (-n / 2))))


def accuracy_bench(torch, W, Plan, batches=2):
    """The paper's accuracy measure (Sec. 5.1) at full size: the complex64
    path against the complex128 reference path (unfused FP64 updates, same
    plan) on the precision workload, n = 70, d = 56, w = 28, k = 8."""
    spec = WORKLOADS["precision"]
    k = spec["k"]
    circ = W.config_circuit(spec["cid"])
    bits = torch.from_numpy(W.config_bitstrings(spec["cid"])[:batches]).cuda()
    plan = Plan.from_circuit(circ)
    z64 = plan.amplitudes(bits, k).cpu().numpy()
    t0 = time.time()
    z128 = plan.debug_amplitudes_c128(bits, k).cpu().numpy()
    dt = time.time() - t0
    tv = _tv_conditional(z64, z128)
    return {"workload": spec["desc"].replace("1 batch/step", f"{batches} batches"),
            "c64_vs_c128_tv_conditional_max": float(tv.max()),
            "c64_vs_c128_max_rel_err": _rel_err(z64, z128, circ.n),
            "c128_reference_s_per_batch": round(dt / batches, 2),
            "paper_c64_vs_c128_tv_bound": 9.0e-7}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, torch, Plan):
    """The oracle (FP64 state vector, OpenMP) on bounded restrictions of the
    workloads, with all host threads and with one; the GPU's complex64
    amplitudes of the same restrictions are compared with its results."""
    import ctypes
    import numpy as np
    import oracle
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        gomp = None
    all_threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    # (name, config id, restriction, batches, k, thread counts)
    plan_ = [("tiny n=12 d=12", 0, 12, 512, 3, (all_threads, 1)),
             ("precision restricted n=22 d=56", 2, 22, 16, 8, (all_threads, 1)),
             ("medium restricted n=24 d=40", 1, 24, 64, 6, (all_threads, 1)),
             ("full_width restricted n=24 d=66", 4, 24, 8, 8, (all_threads, 1))]
    out = []
    head = None
    for name, cid, m, nb, k, threads in plan_:
        log(f"cpu baseline: {name}")
        circ = W.restrict(W.config_circuit(cid), m)
        if cid == 0:
            x = np.arange(1 << (m - k))
            bits = np.concatenate([((x[:, None] >> np.arange(m - k - 1, -1, -1)[None, :]) & 1).astype(np.uint8),
                                   np.zeros((len(x), k), np.uint8)], axis=1)
        else:
            bits = np.ascontiguousarray(W.config_bitstrings(cid)[:nb, :m])
        rec = {"instance": name, "amplitudes": int(len(bits) << k)}
        z = None
        for th in threads:
            log(f"cpu baseline: {name}, {th} thread(s)")
            if gomp is not None:
                gomp.omp_set_num_threads(int(th))
            t0 = time.time()
            psi = oracle.statevector(circ)
            t1 = time.time()
            z = oracle.amplitudes(circ, bits, k, psi=psi)
            t2 = time.time()
            rec[f"threads_{th}"] = {"s_full_state": round(t1 - t0, 3),
                                    "amplitudes_per_s": round(len(bits) * (1 << k) / (t2 - t0), 1),
                                    "state_entries_per_s": round((1 << m) / (t1 - t0), 1)}
        if gomp is not None:
            gomp.omp_set_num_threads(all_threads)
        gp = Plan.from_circuit(circ)
        ws = torch.empty(gp.workspace_bytes(k, 1), dtype=torch.uint8, device="cuda")  # batches run in groups
        g = gp.amplitudes(torch.from_numpy(bits).cuda(), k, workspace=ws).cpu().numpy()
        del ws
        rec["gpu_c64_vs_oracle_max_rel_err"] = _rel_err(g, z, m)
        rec["gpu_c64_vs_oracle_tv_conditional_max"] = float(_tv_conditional(g, z).max()) if k >= 1 else None
        out.append(rec)
        if cid == 4:
            head = rec
    hv = head[f"threads_{all_threads}"]
    return {"value": hv["amplitudes_per_s"], "unit": "amplitudes/s", "cores": all_threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "sample": "FP64 state vector of the full-width circuit restricted to qubits 0..23 (n=24, d=66, all "
                      "67 one-qubit layers), 8 batches x 256 requested amplitudes, all host threads; n=70 itself "
                      "does not fit a state vector",
            "instances": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="full_width")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-storage", action="store_true", help="skip the 16-bit storage comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-width35", action="store_true", help="skip the width-35 batch (279 GB of HBM)")
    ap.add_argument("--no-bond4", action="store_true", help="skip the bond-dimension-4 workload")
    ap.add_argument("--bond4-only", action="store_true",
                    help="only the bond-dimension-4 workload (its own JSON line; profiling runs)")
    ap.add_argument("--options", default=None,
                    help="tile options as JSON (e.g. '{\"max_tile_bits\": 12}') instead of autotuning "
                         "(profiling runs fix them so that only the timed configuration launches)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (reference "
                         "dispatches for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the contraction is "
              f"not sharded in this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2608_13110_amd import Plan, profile_begin, profile_end
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                          "dispatches": 5}), flush=True)
        return
    if args.bond4_only:
        log("bond dimension 4 only")
        print(json.dumps({"bond4": bond4_bench(torch, W, Plan, profile_begin, profile_end)}), flush=True)
        return
    fixed = json.loads(args.options) if args.options else None
    log(f"main workload {args.workload}: autotune and {args.steps} timed steps")
    main_r = run_workload(args.workload, args.steps, args.warmup, torch, W, Plan, profile_begin, profile_end, fixed)
    log(f"main workload done: {main_r['ms_per_step']:.1f} ms per step")
    torch.cuda.empty_cache()
    secondary = None
    if not args.no_secondary:
        other = "precision" if args.workload == "full_width" else "full_width"
        steps2 = 16 if other == "precision" else 2
        log(f"secondary workload {other}")
        secondary = run_workload(other, steps2, 1, torch, W, Plan, profile_begin, profile_end)
        torch.cuda.empty_cache()
    # the side sections report their own failure instead of losing the line
    storage = None
    if not args.no_storage:
        try:
            log("storage modes at w = 28")
            storage = storage_modes(torch, W, Plan, profile_begin, profile_end)
        except Exception as e:  # noqa: BLE001
            storage = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    sampling = None
    if not args.no_secondary:
        try:
            log("samplers")
            sampling = sampling_bench(torch, W, Plan)
        except Exception as e:  # noqa: BLE001
            sampling = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    serving = None
    if not args.no_serving:
        try:
            log("serving stream")
            serving = serving_bench(torch, W)
        except Exception as e:  # noqa: BLE001
            serving = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    ring = None
    if not args.no_secondary:
        try:
            log("ring")
            ring = ring_bench(torch, W)
        except Exception as e:  # noqa: BLE001
            ring = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    accuracy = None
    if not args.no_secondary:
        try:
            log("accuracy: complex64 against complex128")
            accuracy = accuracy_bench(torch, W, Plan)
        except Exception as e:  # noqa: BLE001
            accuracy = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    storage33 = None
    if not args.no_storage and args.workload == "full_width":
        try:
            log("storage modes at w = 33")
            storage33 = storage_full_width(torch, W, Plan, profile_begin, profile_end, main_r["tile_options"])
        except Exception as e:  # noqa: BLE001
            storage33 = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    bond4 = None
    if not args.no_bond4:
        try:
            log("bond dimension 4 (generic two-qubit gates), w = 33")
            bond4 = bond4_bench(torch, W, Plan, profile_begin, profile_end)
        except Exception as e:  # noqa: BLE001
            bond4 = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    width35 = None
    if not args.no_width35 and args.workload != "width35":
        try:
            log("width 35, complex64")
            width35, z35 = width35_bench(torch, W, Plan, profile_begin, profile_end)
            if not args.no_storage:
                log("width 35, FP16 block-scaled")
                width35["f16_blockscale"], _ = width35_bench(torch, W, Plan, profile_begin, profile_end, 1, z35)
        except Exception as e:  # noqa: BLE001
            width35 = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    traffic = recorded_traffic(args.workload)
    roofline = {
        "bound": "hbm", "achieved": round(main_r["pass_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(main_r["pass_gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "k_pass", "bytes_per_launch": main_r["pass_bytes_per_launch"],
        "avg_launch_ms": round(main_r["pass_avg_ms"], 4),
        "alu": {"achieved_tflops": round(main_r["sweep_tflops"], 2), "peak_tflops": FP32_VALU_PEAK_TFLOPS,
                "frac": round(main_r["sweep_tflops"] / FP32_VALU_PEAK_TFLOPS, 4)},
    }
    line = {
        "metric": METRIC, "value": round(main_r["amplitudes_per_s"], 3), "unit": "amplitudes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": main_r["workload"], "batch_amplitudes": 1 << main_r["k"],
                   "boundary_bits": main_r["h"], "passes": main_r["n_passes"], "updates": main_r["n_ops"],
                   "log2_cost": round(main_r["log2_cost"], 3), "tile_options": main_r["tile_options"],
                   "autotune_candidates": MAIN_CANDIDATES, "autotune_ms_per_batch": main_r["autotune_ms"]},
        "hbm_gbs": round(main_r["pass_gbs"], 1), "hbm_frac": roofline["frac"],
        "latency_ms_p50": main_r["latency_ms_p50"], "latency_ms_p99": main_r["latency_ms_p99"],
        "kernel_ms": {"pass": round(main_r["pass_ms"], 2), "late": round(main_r["late_ms"], 2),
                      "init": round(main_r["init_ms"], 2)},
        "roofline": roofline,
        "pass_classes": main_r["pass_classes"],
    }
    if secondary is not None:
        line["secondary"] = {k2: (round(v, 4) if isinstance(v, float) else v) for k2, v in secondary.items()
                             if k2 in ("workload", "amplitudes_per_s", "pass_gbs", "latency_ms_p50",
                                       "latency_ms_p99", "ms_per_step", "steps", "pass_avg_ms", "tile_options",
                                       "pass_classes")}
        line["secondary"]["hbm_frac"] = round(secondary["pass_gbs"] / HBM_PEAK_GBS, 4)
    if storage is not None:
        line["storage_modes"] = storage
    if sampling is not None:
        line["sampling"] = sampling
    if ring is not None:
        line["ring"] = ring
    if storage33 is not None:
        line["storage_full_width"] = storage33
    if width35 is not None:
        line["width35"] = width35
    if bond4 is not None:
        line["bond4"] = bond4
    if accuracy is not None:
        line["accuracy"] = accuracy
    if serving is not None:
        line["serving"] = serving
    if not args.no_cpu_baseline:
        try:
            log("cpu baseline (oracle)")
            line["cpu_baseline"] = cpu_baseline(W, torch, Plan)
        except Exception as e:  # noqa: BLE001
            line["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}"}
    log("done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
