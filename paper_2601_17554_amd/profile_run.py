"""Workload driver for hardware-counter runs (rocprofv3 --pmc): one warm-up and one profiled forward
pass of the benchmark's BF16 varlen batch (64 events), then a plain device copy of known size
whose FETCH_SIZE / WRITE_SIZE readings calibrate the counters.

    python -m paper_2601_17554_amd.profile_run [--precision bf16] [--copy-mib 256]
"""
from __future__ import annotations

import argparse
import os
import sys


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--batches", type=int, default=1)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch

    import bench
    import synth
    from paper_2601_17554_amd import binding as B

    cfg = synth.FULL
    model = B.Model(cfg, synth.make_weights(cfg, 1), args.precision)
    pk = bench.make_batches(args.batches)[0]
    x = torch.from_numpy(pk.x).cuda()
    batch = B.Batch.from_host(pk.row_start, pk.n_valid)
    ws = model.workspace(pk.total_rows, pk.n_events)
    out = model.outputs(pk.total_rows)
    model.reconstruct(x, batch, ws=ws, out=out)
    torch.cuda.synchronize()
    model.reconstruct(x, batch, ws=ws, out=out)
    torch.cuda.synchronize()
    n = args.copy_mib << 18  # float32 elements
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    n2 = (pk.n_valid.astype("float64") ** 2).sum()
    print(f"profile_run: rows {pk.total_rows}, events {pk.n_events}, sum n^2 {n2:.6e}, "
          f"copy {args.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
