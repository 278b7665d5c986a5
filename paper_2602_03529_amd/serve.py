"""Streaming load generator for the tokenizer server (tok_server_*).

Clips arrive by a Poisson process and are submitted at their wall-clock
arrival times; the native server admits them as stream slots and arena
memory free up (batching queued clips of equal shape), runs encode -> FSQ ->
per-clip token drop -> decode, and keeps results on the device until
released.  Reports p50 / p99 latency (submit to completion) and frames/s.

    python -m paper_2602_03529_amd.serve --clips 256 --rate 40 --budget-gb 8
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(clips=256, rate=40.0, T=17, budget_gb=8.0, slots=4, max_batch=4, precision="bf16", seed=3,
        pixel_seeds=2, resolutions=None, max_drop=0.5, drop_mode=1, log=None):
    import torch

    import synth
    from paper_2602_03529_amd import tok

    resolutions = resolutions or synth.SERVE_RESOLUTIONS
    reqs = synth.make_requests(clips, rate, T, seed=seed, resolutions=resolutions, max_drop=max_drop)
    # Pinned host pixels: `pixel_seeds` distinct clips per resolution, reused
    # round-robin (generating 256 full-HD clips on the host would dominate).
    pool = {}
    for (H, W) in resolutions:
        pool[(H, W)] = [torch.from_numpy(synth.make_clip(s, T, H, W)).pin_memory() for s in range(pixel_seeds)]
        if log:
            log("pixels ready for %dx%d" % (W, H))
    model = tok.TokModel(synth.flatten_weights(synth.make_weights(1)), precision)
    budget = int(budget_gb * (1 << 30))
    sv = tok.TokServer(model, budget, slots=slots, max_batch=max_batch)
    def wait(t, what):
        r = sv.wait(t, timeout_ms=120000)
        if r is None:
            raise RuntimeError("server made no progress for 120 s on %s: %s" % (what, sv.stats()))
        return r

    # warm-up: one clip per resolution, outside the measurement
    for (H, W) in resolutions:
        t = sv.submit(pool[(H, W)][0])
        wait(t, "warm-up %dx%d" % (W, H))
        sv.release(t)
        if log:
            log("warm-up %dx%d done" % (W, H))
    torch.cuda.synchronize()

    tickets = [None] * len(reqs)
    results = [None] * len(reqs)
    submitted = threading.Event()

    def submitter():
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            delay = r.arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            px = pool[(r.H, r.W)][r.pixel_seed % pixel_seeds]
            d = tok.Drop(mode=drop_mode, rate=r.drop_rate, seed=seed, clip_id0=r.clip_id)
            tickets[i] = sv.submit(px, d)
        submitted.set()

    start = time.perf_counter()
    th = threading.Thread(target=submitter)
    th.start()
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0005)
        res = wait(tickets[i], "clip %d" % i)
        results[i] = res
        sv.release(tickets[i])
        if log and (i + 1) % 16 == 0:
            log("%d / %d clips done" % (i + 1, len(reqs)))
    th.join()
    makespan = time.perf_counter() - start
    st = sv.stats()
    sv.close()

    lat = np.array([r["total_ms"] for r in results])
    qms = np.array([r["queue_ms"] for r in results])
    frames = sum(r.T for r in reqs)
    by_res = {}
    for r, res in zip(reqs, results):
        by_res.setdefault("%dx%d" % (r.W, r.H), []).append(res["total_ms"])
    batches = np.bincount([r["batch_size"] for r in results])
    return dict(
        clips=len(reqs), frames=frames, rate_per_s=rate, budget_gb=budget_gb, slots=slots, max_batch=max_batch,
        precision=precision, drop_mode=drop_mode, failed=int(sum(r["status"] != 0 for r in results)),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
        mean_queue_ms=float(qms.mean()), makespan_s=makespan, frames_per_s=frames / makespan,
        arrival_span_s=reqs[-1].arrival_s, peak_arena_gb=st["bytes_peak"] / (1 << 30),
        batch_size_hist={str(k): int(v) for k, v in enumerate(batches) if v},
        p50_ms_by_resolution={k: float(np.percentile(v, 50)) for k, v in sorted(by_res.items())})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--clips", type=int, default=256)
    ap.add_argument("--rate", type=float, default=40.0)
    ap.add_argument("--frames", type=int, default=17)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=4)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--pixel-seeds", type=int, default=2)
    ap.add_argument("--drop", choices=["bernoulli", "rows", "similarity"], default="bernoulli",
                    help="per-clip token drop: seeded Bernoulli tokens, lost rows, or similarity-based selection")
    args = ap.parse_args()
    mode = {"bernoulli": 1, "rows": 2, "similarity": 4}[args.drop]
    out = run(args.clips, args.rate, args.frames, args.budget_gb, args.slots, args.max_batch, args.precision,
              pixel_seeds=args.pixel_seeds, drop_mode=mode,
              log=lambda m: print("serve: " + m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
