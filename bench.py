#!/usr/bin/env python3
"""Benchmark of the PivCo-Huffman hot path on one MI355X.

Workload (N=1): 256 MiB of uint8 symbols drawn i.i.d. from Zipf(1.1) over 256
ranks with a seeded permutation of symbol ids, coded in 64 KiB blocks, each
block with its own length-limited (11-bit) canonical tree, no entropy-coded
nodes.  The stream is produced by the GPU encoder and checked against the
input; a "step" is one batched decode of the whole stream (one persistent,
HIP-graph-captured launch).  The JSON line reports decoded GB/s (10^9 B/s),
the HBM roofline fraction of the merge kernel, the same decode as one launch
per block ("plain"), the encode rate, and the CPU oracle timed on a sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

`--workload skew256m|mix4096|geo1m` times the other synthetic workloads the
same way (batched decode and merge-kernel roofline only; the plain, serving
and CPU legs belong to the default line).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded GB/s per MI355X (% HBM roofline), batched vs plain; p99 latency"
HBM_PEAK_GBPS = 8000.0
# one element merge (a byte chosen by a bitmap bit) needs at least one VALU
# lane operation: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS_PEAK_G = 256 * 4 * 16 * 2.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2606_05765_amd", "csrc", "decode.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, variant):
    """HBM bytes per merge launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_k_merge_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("decode_hip_sha256_16") != kernel_source_hash() or t.get("variant") != variant:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(stream_np, n_blocks, block_size, budget_s=12.0):
    import oracle
    t0 = time.perf_counter()
    done = 0
    step = 16
    while done < n_blocks and time.perf_counter() - t0 < budget_s:
        b1 = min(n_blocks, done + step)
        oracle.decode_blocks(stream_np, done, b1)
        done = b1
    dt = time.perf_counter() - t0
    nbytes = done * block_size
    return {"value": round(nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {n_blocks} blocks ({nbytes / 2**20:.0f} MiB) of the same "
                      f"stream, single-threaded C oracle (tree walk per symbol), {dt:.1f} s"}


def element_merges(x, block_size):
    """Sum over blocks of the symbols passing every internal node (n * mean
    code length): the element merges a decode performs.  Per-block trees
    from the library's own tree builder (the encoder's default)."""
    from paper_2606_05765_amd import pivco as P
    total = 0
    for b0 in range(0, x.size, block_size):
        blk = x[b0:b0 + block_size]
        counts = np.bincount(blk, minlength=256).astype(np.uint64)
        if np.count_nonzero(counts) < 2:
            continue
        lens = P.pivco_build_tree(counts, 11)
        total += int(np.dot(counts, np.asarray(lens, dtype=np.uint64)))
    return total


def serving_leg(torch, dev, seconds=1.0, rate_hz=2000.0, n_pool=48, seed=11,
                budget=32 * 10**9):
    """Poisson request trace against the continuous-batching server: decode
    requests of resident streams (sizes log-uniform 16 KiB - 64 MiB, mixed
    families, 1 MiB blocks), output space recycled under the byte budget."""
    import workloads as W
    from paper_2606_05765_amd import pivco as P
    w = W.serve_requests(seed=seed, n_req=n_pool)
    streams = [P.pivco_encode(torch.from_numpy(x).to(dev), w.block_size, ans_mode=w.ans_mode)
               for x in w.jobs]
    torch.cuda.synchronize()
    pool = torch.empty(budget, dtype=torch.uint8, device=dev)
    sv = P.Server(mem_budget=budget, slots=4, max_batch=64, keep_outputs=False)
    ids = [sv.register(st) for st in streams]
    n = int(rate_hz * seconds)
    rng = np.random.default_rng(seed)
    order = rng.integers(0, n_pool, size=n)
    arrivals = W.poisson_arrivals(seed, rate_hz, n)
    res, stats = sv.run(arrivals, [ids[k] for k in order], pool)
    torch.cuda.synchronize()
    sv.close()
    bad = [r["status"] for r in res if r["status"] != 0]
    assert not bad, f"serving statuses {bad[:5]}"
    lat = np.array([r["t_done"] - r["arrival"] for r in res]) * 1e3
    sizes = np.array([w.jobs[k].size for k in order], dtype=np.float64)
    return {"requests": n, "rate_hz": rate_hz, "resident_requests": n_pool,
            "mean_request_MB": round(float(sizes.mean()) / 1e6, 2),
            "offered_GBps": round(float(sizes.sum()) / float(arrivals[-1]) / 1e9, 2),
            "sustained_GBps": round(stats["bytes_decoded"] / stats["wall_s"] / 1e9, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "batches": stats["batches"], "max_batch": stats["max_batch"],
            "budget_GB": round(budget / 1e9, 1), "slots": 4}


WORKLOAD_TEXT = {
    "skew256m": "skew256m: 256 MiB uint8, p(0)=0.9 and 0.1 spread as 0.7^s over 1..255, 128 KiB blocks, "
                "selective binary rANS (one-bit fraction < 0.1 or > 0.9)",
    "mix4096": "mix4096: 4096 independent single-block streams, sizes log-uniform 4 KiB-4 MiB, "
               "geometric / Zipf / uniform families, selective binary rANS",
    "geo1m": "geo1m: 1 MiB uint8, p(s) ~ 0.8^s, one block, no ANS",
}


def other_workload(args, torch, dev):
    """Batched decode of a non-default workload: GB/s and the merge kernel's
    roofline on the same JSON shape (no plain, serving or CPU legs)."""
    import workloads as W
    from paper_2606_05765_amd import pivco as P
    log(f"generating workload {args.workload} ...")
    w = getattr(W, args.workload)(seed=args.seed)
    xs = [np.ascontiguousarray(j) for j in w.jobs]
    d_xs = [torch.from_numpy(x).to(dev) for x in xs]
    bss = [w.block_size or max(x.size, 1) for x in xs]
    streams = [P.pivco_encode(d, bs, max_len=11, ans_mode=w.ans_mode) for d, bs in zip(d_xs, bss)]
    torch.cuda.synchronize()
    n = sum(x.size for x in xs)
    comp = sum(s.numel() for s in streams)
    outs = [torch.empty(x.size, dtype=torch.uint8, device=dev) for x in xs]
    if args.variant is not None:
        tune = P.Tune()
        tune.merge_variant = args.variant
        tune.merge_grid = args.grid or 256
        tune.rans_grid = 512
    else:
        tune = P.pivco_autotune(streams, outs)
    plan = P.BatchPlan(streams, outs, tune=tune)
    variant = P.pivco_merge_variants()[plan.tune.merge_variant]
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert (plan.statuses() == 0).all()
    for o, d in zip(outs, d_xs):
        assert torch.equal(o, d), "decoded bytes differ from the input"
    ms_per_step = dt * 1e3 / args.steps
    value = n / (dt / args.steps) / 1e9
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(); ev1.record()        # torch marks them recorded; the plan re-records them
    torch.cuda.synchronize()
    merge_ms = []
    for _ in range(args.steps):
        plan.launch_timed(ev0, ev1)
        ev1.synchronize()
        merge_ms.append(ev0.elapsed_time(ev1))
    merge_avg = float(np.mean(merge_ms))
    algo_bytes = comp + n
    achieved = algo_bytes / (merge_avg * 1e-3) / 1e9
    merges = sum(element_merges(x, bs) for x, bs in zip(xs, bss))
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "decode": "batched: one persistent HIP-graph launch over all blocks",
                   "variant": variant, "tune": plan.tune.as_dict()},
        "pct_hbm_roofline": round(achieved / HBM_PEAK_GBPS * 100, 2),
        "compression_ratio": round(n / comp, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(w.name, variant), "kernel": f"k_merge<{variant}>",
                     "merge_ms_avg": round(merge_avg, 4), "algorithmic_bytes_per_launch": algo_bytes},
        "alu_view": {"unit": "G element merges/s", "element_merges_per_launch": merges,
                     "mean_code_len": round(merges / n, 4),
                     "achieved": round(merges / (merge_avg * 1e-3) / 1e9, 1),
                     "peak": round(VALU_LANE_OPS_PEAK_G, 1),
                     "frac": round(merges / (merge_avg * 1e-3) / 1e9 / VALU_LANE_OPS_PEAK_G, 4)},
    }
    plan.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant", type=int, default=None, help="fixed merge variant (skips autotune)")
    ap.add_argument("--grid", type=int, default=None, help="fixed merge grid (with --variant)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (latency) leg")
    ap.add_argument("--workload", default="zipf256m",
                    choices=["zipf256m", "skew256m", "mix4096", "geo1m"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (counter scale reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(blocks are independent, so N GPUs would each decode their own share)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2606_05765_amd import pivco as P

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.workload != "zipf256m":
        other_workload(args, torch, dev)
        return
    log("generating workload zipf256m ...")
    w = W.zipf256m(seed=args.seed)
    x = w.jobs[0]
    n = x.size
    bs = w.block_size
    d_x = torch.from_numpy(x).to(dev)

    # encode on the GPU (timed, reported as extra)
    enc_times = []
    stream = None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stream = P.pivco_encode(d_x, bs, max_len=11, ans_mode=w.ans_mode)
        torch.cuda.synchronize()
        enc_times.append(time.perf_counter() - t0)
    comp = stream.numel()
    info = P.pivco_stream_info(stream)
    log(f"encoded {n} -> {comp} bytes ({comp / n:.4f}), {info['n_blocks']} blocks, "
        f"best encode {min(enc_times) * 1e3:.1f} ms")

    out = torch.empty(n, dtype=torch.uint8, device=dev)
    tune = None
    if args.variant is not None:
        tune = P.Tune()
        tune.merge_variant = args.variant
        tune.merge_grid = args.grid or 256
        tune.rans_grid = 256
    elif not args.no_autotune:
        tune = P.pivco_autotune([stream], [out])
        log("autotune:", tune.as_dict(), P.pivco_merge_variants()[tune.merge_variant])
    plan = P.BatchPlan([stream], [out], tune=tune)
    variant = P.pivco_merge_variants()[plan.tune.merge_variant] if plan.tune is not None else \
        P.pivco_merge_variants()[0]

    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = n / (dt / args.steps) / 1e9

    st = plan.statuses()
    assert (st == 0).all(), f"decode status {st}"
    got = out.cpu().numpy()
    assert np.array_equal(got, x), "decoded bytes differ from the input"
    log(f"batched graph decode: {ms_per_step:.3f} ms/step, {value:.1f} GB/s, output verified")

    # roofline of the dominant kernel: HIP events around the merge kernel on
    # the stream it runs on, same number of launches as the timed region
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(); ev1.record()
    torch.cuda.synchronize()
    merge_ms = []
    for _ in range(args.steps):
        plan.launch_timed(ev0, ev1)
        ev1.synchronize()
        merge_ms.append(ev0.elapsed_time(ev1))
    merge_avg = float(np.mean(merge_ms))
    algo_bytes = comp + n             # stream read once + output written once
    achieved = algo_bytes / (merge_avg * 1e-3) / 1e9
    traffic = measured_traffic(w.name, variant)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": traffic, "kernel": f"k_merge<{variant}>",
                "merge_ms_avg": round(merge_avg, 4),
                "algorithmic_bytes_per_launch": algo_bytes}
    log(f"merge kernel: {merge_avg:.3f} ms avg, {achieved:.1f} GB/s algorithmic "
        f"({achieved / HBM_PEAK_GBPS * 100:.1f}% of HBM peak)")
    merges = element_merges(x, bs)
    alu_view = {"unit": "G element merges/s", "element_merges_per_launch": merges,
                "mean_code_len": round(merges / n, 4),
                "achieved": round(merges / (merge_avg * 1e-3) / 1e9, 1),
                "peak": round(VALU_LANE_OPS_PEAK_G, 1),
                "frac": round(merges / (merge_avg * 1e-3) / 1e9 / VALU_LANE_OPS_PEAK_G, 4)}
    log("element merges:", alu_view)

    plain = None
    if not args.no_plain:
        out2 = torch.empty(n, dtype=torch.uint8, device=dev)
        ws = P.Workspace(P.pivco_decode_workspace([stream], [out2]))
        best = 1e30
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, pst = P.pivco_decode_plain([stream], [out2], ws=ws)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            assert (pst == 0).all()
        assert torch.equal(out2, out)
        plain = round(n / best / 1e9, 2)
        log(f"plain per-block launches: {best * 1e3:.2f} ms, {plain} GB/s")

    if args.copy_probe:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    serving = None
    if not args.no_serve:
        log("serving leg (Poisson trace) ...")
        serving = serving_leg(torch, dev)
        log("serving:", serving)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(stream.cpu().numpy(), info["n_blocks"], bs)
        log("cpu baseline:", cpu)

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "zipf256m: 256 MiB uint8, Zipf(1.1) over 256 permuted ids, "
                               "64 KiB blocks, one L=11 canonical tree per block, no ANS",
                   "decode": "batched: one persistent HIP-graph launch over all blocks",
                   "variant": variant,
                   "tune": plan.tune.as_dict() if plan.tune is not None else None},
        "pct_hbm_roofline": round(achieved / HBM_PEAK_GBPS * 100, 2),
        "plain_per_block_GBps": plain,
        "encode_GBps": round(n / min(enc_times) / 1e9, 2),
        "compression_ratio": round(n / comp, 4),
        "roofline": roofline,
        "alu_view": alu_view,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
