"""Per-output error of the GPU forward pass against the FP64 oracle on the benchmark workloads.

Workloads (full model d256 h8 ffn1024 L6, weights seed 1):
  single : a stratified 50-event subset of the 1,000-event single-event set (SeedSequence(200),
           element counts log-normal median 3000 in [500, 8192]): the events at the 50 quantiles
           (i + 0.5) / 50 of the element count; one event per launch, padded to a multiple of 64,
           in FP32 (the plain path) and in BF16;
  varlen : the first 64-event batch of the varlen set (SeedSequence(300), counts in [200, 8192]),
           packed without padding, in BF16 and in BF16 with the FFN products in FP8-E4M3 (activation
           scales calibrated on the FP32 model over 16 events of SeedSequence(500), disjoint from
           the evaluated events).
For each (workload, precision) the report holds, per output, the max / p99 / median over all
elements of the per-element error in the form its tolerance applies to (see parity_util.errors),
and the class agreement (raw, on clear elements, near-tie fraction).

  python tests/error_report.py oracle [--cache DIR]   # CPU: oracle outputs of every event, cached
  python tests/error_report.py gpu [--cache DIR] [--json OUT]   # GPU: the library, then the report

The oracle step only calls oracle/ on the seeded inputs; the GPU step computes any oracle output
the cache lacks itself.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import synth  # noqa: E402
from parity_util import TOL, error_stats  # noqa: E402

CFG = synth.FULL
WEIGHT_SEED = 1
N_SINGLE = 50


def single_indices():
    counts = synth.event_set_counts(200, 1000, lo=500)
    order = np.argsort(counts, kind="stable")
    return [int(order[int((i + 0.5) / N_SINGLE * len(counts))]) for i in range(N_SINGLE)]


def single_events():
    return [(i, synth.event_of_set(200, 1000, i, lo=500)) for i in single_indices()]


def varlen_events():
    return list(enumerate(synth.event_set(300, 64, lo=200)))


def event_of(seed_set: str, idx: int):
    if seed_set == "single":
        return synth.event_of_set(200, 1000, idx, lo=500)
    return synth.event_of_set(300, 64, idx, lo=200)


def _cache_path(cache: str, name: str, idx: int) -> str:
    return os.path.join(cache, f"{name}_{idx}.npz")


def oracle_out(cache: str, name: str, idx: int, ev, w):
    from oracle import mlpf_oracle as O
    path = _cache_path(cache, name, idx)
    if os.path.exists(path):
        z = np.load(path)
        return {"logits": z["logits"], "reg": z["reg"], "cls": z["cls"]}
    ref = O.forward(ev.x, w, CFG)
    out = {"logits": ref["logits"], "reg": ref["reg"], "cls": ref["cls"]}
    os.makedirs(cache, exist_ok=True)
    np.savez(path, **out)
    return out


def _oracle_job(job):
    cache, name, idx, seed_set = job
    w = synth.make_weights(CFG, WEIGHT_SEED)
    ev = event_of(seed_set, idx)
    t = time.perf_counter()
    oracle_out(cache, name, idx, ev, w)
    return name, idx, ev.n, time.perf_counter() - t


def run_oracle(cache: str, procs: int) -> None:
    import multiprocessing as mp
    jobs = [(cache, "single", i, "single") for i in single_indices()]
    jobs += [(cache, "varlen", i, "varlen") for i in range(64)]
    jobs = [j for j in jobs if not os.path.exists(_cache_path(cache, j[1], j[2]))]
    print(f"{len(jobs)} oracle events to compute", flush=True)
    with mp.get_context("spawn").Pool(procs) as pool:
        for name, idx, n, dt in pool.imap_unordered(_oracle_job, jobs):
            print(f"oracle {name} {idx} n={n}: {dt:.1f} s", flush=True)


def run_gpu(cache: str) -> dict:
    import torch
    from paper_2601_17554_amd import binding as B

    torch.cuda.set_device(0)
    w = synth.make_weights(CFG, WEIGHT_SEED)
    report = {"model": "d256 h8 ffn1024 L6, weights seed 1", "tolerance": TOL}
    single = single_events()
    for prec in ("fp32", "bf16"):
        m = B.Model(CFG, w, prec)
        pairs = []
        for i, ev in single:
            pk = synth.pack([ev], pad_to=64)
            out = m.reconstruct(torch.from_numpy(pk.x).cuda(), B.Batch.from_host(pk.row_start, pk.n_valid))
            torch.cuda.synchronize()
            got = {k: v[: ev.n].cpu().numpy() for k, v in out.items()}
            pairs.append((got, oracle_out(cache, "single", i, ev, w)))
        report[f"single_{prec}"] = {
            "events": len(pairs), "elements": int(sum(ev.n for _, ev in single)),
            "element_counts": [int(min(ev.n for _, ev in single)), int(max(ev.n for _, ev in single))],
            **error_stats(pairs, TOL[prec])}
        print(f"single {prec}: {json.dumps(report[f'single_{prec}'])}", flush=True)
        del m
    var = varlen_events()
    pk = synth.pack([ev for _, ev in var])
    calib = synth.event_set(500, 16, lo=200)
    models = {"bf16": B.Model(CFG, w, "bf16"),
              "bf16_fp8ffn": B.build_fp8_model(CFG, w, [(e.x, np.array([0, e.n], np.int32), None)
                                                        for e in calib])}
    for name, m in models.items():
        out = m.reconstruct(torch.from_numpy(pk.x).cuda(), B.Batch.from_host(pk.row_start, pk.n_valid))
        torch.cuda.synchronize()
        outs = {k: v.cpu().numpy() for k, v in out.items()}
        pairs = []
        for e, ev in var:
            r = pk.event_rows(e)
            pairs.append(({k: v[r] for k, v in outs.items()}, oracle_out(cache, "varlen", e, ev, w)))
        report[f"varlen_{name}"] = {"events": len(pairs), "elements": int(pk.n_valid.sum()),
                                    **error_stats(pairs, TOL["bf16"])}
        print(f"varlen {name}: {json.dumps(report[f'varlen_{name}'])}", flush=True)
    return report


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["oracle", "gpu"])
    ap.add_argument("--cache", default=os.path.join(ROOT, ".oracle_cache"))
    ap.add_argument("--procs", type=int, default=2)
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    if args.mode == "oracle":
        run_oracle(args.cache, args.procs)
        return
    report = run_gpu(args.cache)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(report, f, indent=1)
    print(json.dumps(report))


if __name__ == "__main__":
    main()
