"""Workload driver for hardware-counter runs (rocprofv3 --pmc): the benchmark's BF16 varlen batches
(64 events each, the same seeded batches bench.py times), with tile shapes chosen by the autotuner
as bench.py does; one warm-up pass, then one forward pass per batch, then a plain device copy of
known size whose FETCH_SIZE / WRITE_SIZE readings calibrate the counters.

    python profile_run.py [--precision bf16] [--batches 4] [--copy-mib 256]
        [--tiles '{"attention": 7, ...}']

With --one-event it instead runs the one-event-per-launch workload of bench.py's plain legs: the
event of median element count among its 40 events, tiles autotuned for it, 20 graph replays.
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--tiles", default="", help="JSON {op: tile} to pin (default: autotune)")
    ap.add_argument("--one-event", action="store_true", help="one median full-size event per launch")
    args = ap.parse_args()
    root = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, root)
    import torch

    import bench
    import synth
    from paper_2601_17554_amd import autotune
    from paper_2601_17554_amd import binding as B

    cfg = synth.FULL
    model = B.Model(cfg, synth.make_weights(cfg, 1), args.precision)
    if args.one_event:
        one_event(model, args, B, autotune, synth, torch)
        return
    batches = bench.make_batches(args.batches)
    dev = []
    for pk in batches:
        dev.append((torch.from_numpy(pk.x).cuda(), B.Batch.from_host(pk.row_start, pk.n_valid)))
    rows = max(pk.total_rows for pk in batches)
    ws = model.workspace(rows, bench.EVENTS_PER_BATCH)
    out = model.outputs(rows)
    if args.tiles:
        tiles = json.loads(args.tiles)
        for op, t in tiles.items():
            model.tune_set(op, int(t))
    else:
        tiles = autotune.tune(model, dev[0][0], dev[0][1], ws=ws, use_cache=False)
    torch.cuda.synchronize()
    print("profile_run: tiles " + json.dumps(tiles), flush=True)
    model.reconstruct(dev[0][0], dev[0][1], ws=ws, out=out)
    torch.cuda.synchronize()
    print("profile_run: measured passes begin", flush=True)
    for x, b in dev:
        model.reconstruct(x, b, ws=ws, out=out)
    torch.cuda.synchronize()
    n = args.copy_mib << 18  # float32 elements
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    for i, pk in enumerate(batches):
        n2 = float((pk.n_valid.astype("float64") ** 2).sum())
        print(f"profile_run: batch {i} rows {pk.total_rows} sum n^2 {n2:.6e}", flush=True)
    print(f"profile_run: copy {args.copy_mib} MiB", flush=True)


def one_event(model, args, B, autotune, synth, torch) -> None:
    """The median event of bench.py's one-event legs (40 events, seed 200, at least 500 elements),
    padded to a multiple of 64, graph-replayed 20 times after the autotuner's choice."""
    import numpy as np
    evs = synth.event_set(200, 40, lo=500)
    ev = evs[int(np.argsort([e.n for e in evs])[len(evs) // 2])]
    pk = synth.pack([ev], pad_to=64)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        x = torch.from_numpy(pk.x).cuda()
        batch = B.Batch.from_host(pk.row_start, pk.n_valid)
        ws = model.workspace(pk.total_rows, 1)
        out = model.outputs(pk.total_rows)
        stream.synchronize()
        if args.tiles:
            for op, t in json.loads(args.tiles).items():
                model.tune_set(op, int(t))
            tiles = json.loads(args.tiles)
        else:
            tiles = autotune.tune(model, x, batch, ws=ws, use_cache=False)
        print(f"profile_run: one event of {ev.n} elements, tiles " + json.dumps(tiles), flush=True)
        graph = B.Graph(model, x, batch, out, ws, stream)
        for _ in range(5):
            graph.launch()
        stream.synchronize()
        print("profile_run: measured replays begin", flush=True)
        for _ in range(20):
            graph.launch()
        stream.synchronize()
    print("profile_run: done", flush=True)


if __name__ == "__main__":
    main()
