"""Workload driver for hardware-counter runs (rocprofv3 --pmc): the benchmark's BF16 varlen batches
(64 events each, the same seeded batches bench.py times), with tile shapes chosen by the autotuner
as bench.py does; one warm-up pass, then one forward pass per batch, then a plain device copy of
known size whose FETCH_SIZE / WRITE_SIZE readings calibrate the counters.

    python profile_run.py [--precision bf16] [--batches 4] [--copy-mib 256]
        [--tiles '{"attention": 7, ...}']
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


if __name__ == "__main__":
    main()
