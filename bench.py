"""Benchmark of the MLPF forward pass on one MI355X.

A step is one mlpf_reconstruct_events call (embedding, all encoder blocks, heads) over one batch of
64 synthetic events packed varlen (element counts log-normal, median 3000, 200..8192) in BF16,
inputs already resident in HBM. Beside it: the plain path runs one full-size event per launch in FP32
and in BF16 (the same log-normal counts, 500..8192, padded to a multiple of 64); the small model runs
one 256-element event per launch in FP32 (latency over many reps, kernels only and with the PCIe
copies); and the FP64 oracle is timed on the host's cores on a bounded sample of the varlen events.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "events/sec + p50/p99 ms/event, BF16 varlen vs FP32 plain, 1 MI355X"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
# exp2 ceiling of the BF16 attention: transcendentals issue at a quarter of the FP32 vector rate
# (157.3 TFLOP/s = 32 FMA lanes per SIMD x 1024 SIMDs x 2.4 GHz), i.e. 8 lanes per cycle per SIMD.
PEAK_EXP_T_PER_S = 1024 * 8 * 2.4e9 / 1e12
EVENTS_PER_BATCH = 64

# HBM bytes per launch of the BF16 attention kernel on these batches, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) of profile_run.py scaled by a 256 MiB copy
# (profiles/attention_bf16_varlen64_hbm_traffic.md). Valid only for the kernel source it was
# measured on: reported as null once that source changes (attention.hip, common.h, and the
# attention declarations of kernels.h: AttnArgs, AttnTile and the launchers).
ATTN_TRAFFIC = {"sha256": "ce919856719c313bf501cd4171f28d8612aa806aaa38196baea70f32ce0549c5",
                "bytes_per_launch": 458213662.2}


def attention_source_hash() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_2601_17554_amd", "csrc")
    h = hashlib.sha256()
    for f in ("attention.hip", "common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "kernels.h"), "r") as fh:
        k = fh.read()
    a = k.index("// Attention over a device work list")
    b = k.index("\n", k.index("hipError_t launch_keynorm("))
    h.update(k[a:b].encode())
    return h.hexdigest()


def attention_traffic():
    return ATTN_TRAFFIC["bytes_per_launch"] if attention_source_hash() == ATTN_TRAFFIC["sha256"] else None


def attention_flops(n: np.ndarray, cfg) -> float:
    """Algorithmic FLOPs of one attention launch (one layer): 4 d sum_e n_e^2."""
    n = n.astype(np.float64)
    return float(4.0 * cfg.d_model * (n * n).sum())


def forward_flops(n: np.ndarray, cfg) -> float:
    d, f, dff, L = cfg.d_model, cfg.n_features, cfg.d_ff, cfg.n_layers
    n = n.astype(np.float64)
    lin = 2 * n * (f * d + d * d + L * (4 * d * d + 2 * d * dff) + 5 * d * d + 11 * d)
    return float((lin + L * 4 * d * n * n).sum())


def make_batches(count: int, root_seed: int = 300):
    evs = synth.event_set(root_seed, count * EVENTS_PER_BATCH, lo=200)
    return [synth.pack(evs[i * EVENTS_PER_BATCH:(i + 1) * EVENTS_PER_BATCH]) for i in range(count)]


def _timed_steps(stream, steps, fn):
    """Runs fn(i) for i < steps between per-step events; returns (wall seconds, per-step ms)."""
    import torch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn(i)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])


def bench_varlen(args, cfg, w, model=None, partition_target=None):
    """Graph-replayed varlen batches (timed region), then the same steps eagerly with the
    per-kernel HIP-event profiler (kernel durations for the roofline). ``partition_target``: the
    attention runs within (eta, phi) cells of about that many elements of each event."""
    import torch
    from paper_2601_17554_amd import autotune
    from paper_2601_17554_amd import binding as B
    from paper_2601_17554_amd import partition

    if model is None:
        model = B.Model(cfg, w, args.precision)
    batches = make_batches(args.batches)
    stream = torch.cuda.Stream()
    res = {}

    def device_batch(pk):
        if partition_target is None:
            return torch.from_numpy(pk.x).cuda(), B.Batch.from_host(pk.row_start, pk.n_valid)
        perm, prs, pnv = partition.partition_batch(pk.x, pk.row_start, pk.n_valid, partition_target)
        b = B.Batch.from_host(pk.row_start, pk.n_valid).with_parts(B.Batch.from_host(prs, pnv))
        res["partitions"] = res.get("partitions", 0) + len(pnv)
        res.setdefault("part_n", []).append(pnv)
        return torch.from_numpy(np.ascontiguousarray(pk.x[perm])).cuda(), b
    with torch.cuda.stream(stream):
        dev = [device_batch(pk) for pk in batches]
        wss = [model.workspace(pk.total_rows, b.work_events) for pk, (_, b) in zip(batches, dev)]
        outs = [model.outputs(pk.total_rows) for pk in batches]
        stream.synchronize()
        res["tiles"] = autotune.tune(model, dev[0][0], dev[0][1], ws=wss[0], use_cache=False)
        print(f"bench: tiles {res['tiles']}", file=sys.stderr, flush=True)
        # Before the timed passes: the eager pass stays the last run of the attention kernel.
        res["candidates"] = bench_candidates(model, batches[0], dev[0], wss[0], stream)
        graphs = [B.Graph(model, x, b, o, ws, stream) for (x, b), o, ws in zip(dev, outs, wss)]
        for i in range(args.warmup):
            graphs[i % len(graphs)].launch()
        res["wall_s"], res["batch_ms"] = _timed_steps(stream, args.steps,
                                                     lambda i: graphs[i % len(graphs)].launch())
        # Eager pass of the same steps with the profiler on (kernel durations on this stream).
        model.profiler_enable(True)
        eager_wall, _ = _timed_steps(stream, args.steps, lambda i: model.reconstruct(
            dev[i % len(dev)][0], dev[i % len(dev)][1], ws=wss[i % len(dev)], out=outs[i % len(dev)],
            stream=stream))
        res["prof"] = model.profiler_read()
        model.profiler_enable(False)
        # The outputs of the first batch (its last run), for the error statistics.
        res["out0"] = model.reconstruct(dev[0][0], dev[0][1], ws=wss[0], out=outs[0], stream=stream)
        stream.synchronize()
        res["out0"] = {k: v.cpu().numpy() for k, v in res["out0"].items()}
    res["eager_ms_per_step"] = eager_wall * 1e3 / args.steps
    n_timed = np.concatenate([batches[i % len(batches)].n_valid for i in range(args.steps)])
    res["events"] = len(n_timed)
    res["flops"] = forward_flops(n_timed, cfg)
    res["attn_ms"], res["attn_launches"] = res["prof"]["attention"]
    # Attention FLOPs of what runs: sum over events (or attention partitions) of 4 d n^2.
    units = res["part_n"] if partition_target is not None else [pk.n_valid for pk in batches]
    res["attn_flops"] = sum(attention_flops(units[i % len(batches)], cfg) * cfg.n_layers
                            for i in range(args.steps))
    res["mean_n"] = float(n_timed.mean())
    del graphs
    return res


def bench_candidates(model, pk, dev, ws, stream, reps: int = 50):
    """Candidate construction (mlpf_candidates: per-event counts, scan, ordered writes) on the
    outputs of one 64-event batch with the Eq. 2 decode; HIP events on the launch stream."""
    import torch
    from paper_2601_17554_amd import binding as B
    x, batch = dev
    prim = torch.from_numpy(pk.prim).cuda()
    out = model.outputs(pk.total_rows, decode=True)
    model.reconstruct(x, batch, prim=prim, ws=ws, out=out, stream=stream)
    cands = B.candidates(batch, out["cls"], out["decoded"], stream=stream)
    _, ms = _timed_steps(stream, reps, lambda i: B.mlpf_candidates(
        batch, out["cls"], out["decoded"], cands["offsets"], cands["rows"], cands["cls"],
        cands["kin"], pk.total_rows, stream))
    total = int(cands["offsets"][-1].item())
    valid = int(pk.n_valid.sum())
    # Algorithmic bytes: the classes of the valid rows read twice (count, write), 16 B of decoded
    # kinematics read and 24 B written per candidate, the offsets written twice and read once.
    nbytes = 8 * valid + 40 * total + 12 * (pk.n_events + 1)
    avg = float(ms.mean())
    return {"ms_per_batch": round(avg, 4), "p99_ms": round(float(np.percentile(ms, 99)), 4),
            "candidates_per_batch": total, "elements_per_batch": valid,
            "algorithmic_bytes": nbytes, "gb_per_s": round(nbytes / (avg * 1e-3) / 1e9, 1),
            "launches": 3}


def bench_plain(args, cfg, w, precision):
    """One full-size event per launch (the same events for FP32 and BF16): eager (profiled) and
    graph-replayed latency."""
    import torch
    from paper_2601_17554_amd import autotune
    from paper_2601_17554_amd import binding as B

    model = B.Model(cfg, w, precision)
    evs = synth.event_set(200, args.plain_events, lo=500)
    pks = [synth.pack([e], pad_to=64) for e in evs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dev = [(torch.from_numpy(p.x).cuda(), B.Batch.from_host(p.row_start, p.n_valid)) for p in pks]
        ws = model.workspace(max(p.total_rows for p in pks), 1)
        outs = [model.outputs(p.total_rows) for p in pks]
        med = int(np.argsort([e.n for e in evs])[len(evs) // 2])
        stream.synchronize()
        tiles = autotune.tune(model, dev[med][0], dev[med][1], ws=ws, use_cache=False)
        for i in range(min(3, len(dev))):
            model.reconstruct(dev[i][0], dev[i][1], ws=ws, out=outs[i], stream=stream)
        model.profiler_enable(True)
        wall, lat = _timed_steps(stream, len(dev), lambda i: model.reconstruct(
            dev[i][0], dev[i][1], ws=ws, out=outs[i], stream=stream))
        prof = model.profiler_read()
        model.profiler_enable(False)
        graphs = [B.Graph(model, x, b, o, ws, stream) for (x, b), o in zip(dev, outs)]
        graphs[0].launch()
        gwall, glat = _timed_steps(stream, len(dev), lambda i: graphs[i].launch())
        del graphs
    n = np.array([e.n for e in evs])
    attn_flops = sum(attention_flops(np.array([k]), cfg) * cfg.n_layers for k in n)
    pl_attn_ms, pl_attn_n = prof["attention"]
    achieved = (attn_flops / max(pl_attn_n, 1)) / (pl_attn_ms / max(pl_attn_n, 1) * 1e-3) / 1e12
    return {
        "value": round(len(n) / gwall, 2), "unit": "events/s",
        "p50_ms_per_event": round(float(np.percentile(glat, 50)), 3),
        "p99_ms_per_event": round(float(np.percentile(glat, 99)), 3),
        "eager_value": round(len(n) / wall, 2),
        "eager_p50_ms_per_event": round(float(np.percentile(lat, 50)), 3),
        "eager_p99_ms_per_event": round(float(np.percentile(lat, 99)), 3),
        "events": int(len(n)), "median_elements": int(np.median(n)),
        "attention_tflops": round(achieved, 1),
        f"attention_frac_{precision}_peak": round(achieved / PEAK_TFLOPS[precision], 4),
        "tiles": tiles,
    }


def bench_small(args):
    """The small model (d64 h4 ffn256 L3, weights seed 0) on one event of exactly 256 elements
    (seed 100) in FP32, one event per launch. Latency per rep: kernels only (eager launches, then
    the captured graph, input resident), and end to end (pinned H2D of the features, the graph,
    D2H of the outputs, host wait)."""
    import torch
    from paper_2601_17554_amd import binding as B

    cfg = synth.SMALL
    model = B.Model(cfg, synth.make_weights(cfg, 0), "fp32")
    pk = synth.pack([synth.make_event(100, 256)])
    reps, warm = args.small_reps, 50
    stream = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(stream):
        x_host = torch.from_numpy(pk.x).pin_memory()
        x = x_host.cuda()
        batch = B.Batch.from_host(pk.row_start, pk.n_valid)
        ws = model.workspace(pk.total_rows, 1)
        out = model.outputs(pk.total_rows)
        host_out = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True) for k, v in out.items()}
        stream.synchronize()
        for _ in range(warm):
            model.reconstruct(x, batch, ws=ws, out=out, stream=stream)
        _, res["eager"] = _timed_steps(stream, reps, lambda i: model.reconstruct(
            x, batch, ws=ws, out=out, stream=stream))
        graph = B.Graph(model, x, batch, out, ws, stream)
        for _ in range(warm):
            graph.launch()
        _, res["graph"] = _timed_steps(stream, reps, lambda i: graph.launch())
        e2e = np.empty(reps)
        for i in range(warm + reps):
            t0 = time.perf_counter()
            x.copy_(x_host, non_blocking=True)
            graph.launch()
            for k, v in out.items():
                host_out[k].copy_(v, non_blocking=True)
            stream.synchronize()
            if i >= warm:
                e2e[i - warm] = (time.perf_counter() - t0) * 1e3
        res["e2e"] = e2e
        del graph

    def summary(ms):
        return {"p50_ms": round(float(np.percentile(ms, 50)), 4),
                "p99_ms": round(float(np.percentile(ms, 99)), 4),
                "events_per_s": round(1e3 / float(ms.mean()), 1)}
    return {"model": "d64 h4 ffn256 L3", "elements": 256, "reps": reps, "warmup": warm,
            "eager_kernels": summary(res["eager"]), "graph_kernels": summary(res["graph"]),
            "graph_with_h2d_d2h": summary(res["e2e"])}


def bench_serving(args, cfg, w):
    """Poisson arrivals at several rates through the continuous-batching server (BF16, up to 64
    events per batch, admission bounded by a 64 GB activation budget, the Eq. 2 decode on); latency
    = arrival to result on the host, including host packing and both PCIe copies. Per rate: the
    latency percentiles, how they split into queue wait (arrival to admission) and batch service
    (launch to result), the batch sizes and the budget's use."""
    from paper_2601_17554_amd import binding as B
    from paper_2601_17554_amd import serve

    model = B.Model(cfg, w, args.precision)
    budget = 64 << 30
    # Row-capacity buckets 262144 / 2^k down to 4096: a lone event replays a graph captured for
    # at most 4096 rows, where the key split and the split FFN apply.
    ex = serve.GpuExecutor(model, max_rows=262144, max_events=EVENTS_PER_BATCH, slots=3,
                           hbm_budget=budget, buckets=7, decode=True)

    def pct(a, q):
        return round(float(np.percentile(a, q)), 3) if len(a) else None
    # A discarded warm-up stream (100 events at 1000/s) before the measured rates: the host threads,
    # allocator caches and every graph bucket have then run once.
    warm = synth.event_set(399, 100, lo=200)
    srv = serve.Server(ex)
    arr = synth.poisson_arrivals(1000.0, 100, seed=1399)
    serve.run_poisson(srv, [e.x for e in warm], arr - arr[0], prims=[e.prim for e in warm])
    srv.close()
    out = {}
    for rate in args.serve_rates:
        count = max(50, int(rate * args.serve_seconds))
        evs = synth.event_set(400 + int(rate), count, lo=200)
        arrivals = synth.poisson_arrivals(float(rate), count, seed=1400 + int(rate))
        srv = serve.Server(ex)
        late = []
        # Python's cyclic garbage collector is paused while the requests stream in (its full
        # collections stop both the submitting and the scheduling thread for milliseconds).
        gc.collect()
        gc.disable()
        try:
            wall = serve.run_poisson(srv, [e.x for e in evs], arrivals - arrivals[0],
                                     prims=[e.prim for e in evs], late=late)
            srv.close()
        finally:
            gc.enable()
        lat = srv.latencies_ms()
        wait = srv.queue_waits_ms()
        log = np.array(srv.batch_log, dtype=np.float64).reshape(-1, 4)
        sizes = log[:, 0].astype(int)
        out[str(rate)] = {
            "offered_events_per_s": rate, "events": count, "events_per_s": round(count / wall, 1),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "queue_wait_ms": {"p50": pct(wait, 50), "p99": pct(wait, 99)},
            "submit_late_ms": {"p50": pct(np.array(late) * 1e3, 50), "p99": pct(np.array(late) * 1e3, 99)},
            "batch_service_ms": {"p50": pct(log[:, 3] * 1e3, 50), "p99": pct(log[:, 3] * 1e3, 99)},
            "batches": srv.stats["batches"],
            "batch_events": {"mean": round(float(sizes.mean()), 2), "max": int(sizes.max()),
                             "histogram": {str(k): int(v) for k, v in
                                           zip(*np.unique(np.minimum(sizes, 16), return_counts=True))}},
            "max_slots_in_flight": srv.stats["max_inflight_slots"],
            "max_inflight_gb": round(srv.stats["max_inflight_bytes"] / 2**30, 3),
            "admission_blocked": srv.stats["admission_blocked"]}
        print(f"serving {rate}/s: {out[str(rate)]}", file=sys.stderr, flush=True)
    return {"slots": ex.slots(), "slot_gb": round(ex.slot_bytes / 2**30, 3),
            "budget_gb": budget / 2**30, "rates": out}


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use (the job's CPU share: the
    OMP_NUM_THREADS limit where one is set, else the affinity mask)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0))
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return {"model": model, "affinity_cores": affinity, "cores": min(env, affinity) if env else affinity}


def cpu_baseline(cfg, w, budget_s: float):
    """The FP64 oracle on the host's cores, twice: with all the job's cores, then with one thread,
    each on the first events of the varlen workload (its first 64-event batch) until its time budget
    is spent (at least one event). Returns the record and the oracle outputs of the all-core run
    (event index -> outputs), which the error statistics compare the GPU's outputs with."""
    from threadpoolctl import threadpool_limits

    from oracle import mlpf_oracle as O
    cpu = host_cpu()
    evs = synth.event_set(300, EVENTS_PER_BATCH, lo=200)

    def run(threads):
        refs = {}
        with threadpool_limits(threads):
            t0 = time.perf_counter()
            for i, e in enumerate(evs):
                refs[i] = O.forward(e.x, w, cfg)
                if time.perf_counter() - t0 > budget_s:
                    break
            dt = time.perf_counter() - t0
        n = [evs[i].n for i in refs]
        return {"value": round(len(refs) / dt, 4), "unit": "events/s", "cores": threads,
                "kind": "oracle", "seconds": round(dt, 2),
                "sample": f"first {len(refs)} events of the varlen workload (seed 300; elements "
                          f"{', '.join(map(str, n))}), FP64 NumPy, {threads} thread(s)"}, refs

    rec, refs = run(cpu["cores"])
    one, _ = run(1)
    rec["one_thread"] = one
    rec["host"] = cpu
    return rec, refs


def output_errors(refs, outs: dict, pk) -> dict:
    """Per-output error statistics (tests/parity_util.error_stats) of each precision's outputs on
    the events the oracle ran."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_util import TOL, error_stats
    res = {"events": sorted(refs), "elements": int(sum(pk.n_valid[i] for i in refs))}
    for name, out in outs.items():
        if out is None:
            continue
        tol = TOL["fp32" if name == "fp32" else "bf16"]
        pairs = [({k: v[pk.event_rows(i)] for k, v in out.items()}, ref) for i, ref in refs.items()]
        st = error_stats(pairs, tol)
        res[name] = {k: ({q: (x if isinstance(x, int) else float(f"{x:.3g}")) for q, x in v.items()}
                         if isinstance(v, dict) else v) for k, v in st.items()}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--plain-events", type=int, default=40)
    ap.add_argument("--small-reps", type=int, default=2000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-layout", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-partitioned", action="store_true")
    ap.add_argument("--serve-rates", type=int, nargs="*", default=[200, 500, 1000, 2000])
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(events are independent: the multi-GPU form is data parallel over events)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)

    cfg = synth.FULL
    w = synth.make_weights(cfg, 1)
    # The one-event legs first: the varlen leg's eager pass is then the last run of the BF16
    # attention kernel before the serving leg (a kernel trace reads its dispatches there).
    sm = bench_small(args)
    print("bench: small fp32 done", file=sys.stderr, flush=True)
    pl = bench_plain(args, cfg, w, "fp32")
    print("bench: fp32 plain done", file=sys.stderr, flush=True)
    pb = bench_plain(args, cfg, w, "bf16")
    print("bench: bf16 plain done", file=sys.stderr, flush=True)
    pl_layout = None
    if not args.no_paper_layout:
        # The paper's own network (two parallel 3-block encoders, 16 heads of width 16, ReLU,
        # separate track embeddings, binary-score rule) on the same batches: twice the exponentials
        # per score FLOP of the d_head 32 model.
        pargs = argparse.Namespace(**vars(args))
        pargs.steps, pargs.warmup = min(args.steps, 10), 1
        pc = synth.PAPER_MODEL
        pr = bench_varlen(pargs, pc, synth.make_weights(pc, 1))
        a_ms = pr["attn_ms"] / max(pr["attn_launches"], 1)
        a_fl = pr["attn_flops"] / max(pr["attn_launches"], 1)
        pl_layout = {
            "model": "d256 h16 (d_head 16) ffn1024, two parallel stacks of 3 blocks, ReLU, "
                     "track/other embeddings, binary-score class rule",
            "value": round(pr["events"] / pr["wall_s"], 2), "unit": "events/s",
            "ms_per_step": round(pr["wall_s"] * 1e3 / pargs.steps, 3), "steps": pargs.steps,
            "attention_avg_launch_ms": round(a_ms, 4),
            "attention_frac_bf16_peak": round(a_fl / (a_ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"], 4),
            "attention_exp_frac": round(a_fl * pc.n_heads / (4.0 * pc.d_model) / (a_ms * 1e-3) / 1e12
                                        / PEAK_EXP_T_PER_S, 4),
            "tiles": pr["tiles"]}
        print(f"bench: paper layout {pl_layout['value']} events/s", file=sys.stderr, flush=True)
    part = None
    if not args.no_partitioned:
        # Partitioned attention (events cut into (eta, phi) cells of about 512 elements; attention
        # within a cell only): an approximation of the model, timed on the same batches.
        pargs = argparse.Namespace(**vars(args))
        pargs.steps, pargs.warmup = min(args.steps, 10), 1
        pr = bench_varlen(pargs, cfg, w, partition_target=512)
        a_ms = pr["attn_ms"] / max(pr["attn_launches"], 1)
        part = {"value": round(pr["events"] / pr["wall_s"], 2), "unit": "events/s",
                "ms_per_step": round(pr["wall_s"] * 1e3 / pargs.steps, 3), "steps": pargs.steps,
                "cell_target": 512, "partitions_per_batch": round(pr["partitions"] / args.batches, 1),
                "attention_avg_launch_ms": round(a_ms, 4),
                "attention_frac_bf16_peak": round(pr["attn_flops"] / max(pr["attn_launches"], 1)
                                                  / (a_ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"], 4),
                "tiles": pr["tiles"]}
        print(f"bench: partitioned {part['value']} events/s", file=sys.stderr, flush=True)
    fp8 = None
    fp8_out0 = None
    if not args.no_fp8:
        # BF16 with the FFN products in FP8-E4M3 (activation scales calibrated on the FP32 model
        # over the first batch), on the same batches.
        from paper_2601_17554_amd import binding as B
        pk0 = make_batches(1)[0]
        m8 = B.build_fp8_model(cfg, w, [(pk0.x, pk0.row_start, pk0.n_valid)])
        fargs = argparse.Namespace(**vars(args))
        fargs.steps, fargs.warmup = min(args.steps, 10), 1
        fr = bench_varlen(fargs, cfg, w, model=m8)
        fp8_out0 = fr["out0"]
        fp8 = {"value": round(fr["events"] / fr["wall_s"], 2), "unit": "events/s",
               "ms_per_step": round(fr["wall_s"] * 1e3 / fargs.steps, 3), "steps": fargs.steps,
               "ffn_ms_per_step": round((fr["prof"]["ffn1"][0] + fr["prof"]["ffn2"][0]) / fargs.steps, 4),
               "tiles": fr["tiles"]}
        del m8
        print(f"bench: fp8 ffn {fp8['value']} events/s", file=sys.stderr, flush=True)
    vr = bench_varlen(args, cfg, w)
    print(f"bench: varlen {vr['events'] / vr['wall_s']:.1f} events/s", file=sys.stderr, flush=True)

    ms_per_step = vr["wall_s"] * 1e3 / args.steps
    value = vr["events"] / vr["wall_s"]
    per_event = vr["batch_ms"] / EVENTS_PER_BATCH
    attn_avg_ms = vr["attn_ms"] / max(vr["attn_launches"], 1)
    attn_flops_per_launch = vr["attn_flops"] / max(vr["attn_launches"], 1)
    achieved = attn_flops_per_launch / (attn_avg_ms * 1e-3) / 1e12
    exp_rate = attn_flops_per_launch * cfg.n_heads / (4.0 * cfg.d_model) / (attn_avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = attention_traffic() if args.precision == "bf16" else None
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"varlen_{args.precision}_64_events_per_launch_hipgraph",
                   "events_per_step": EVENTS_PER_BATCH,
                   "element_count": "lognormal median 3000 sigma 0.5 in [200, 8192]",
                   "mean_elements": round(vr["mean_n"], 1),
                   "model": "d256 h8 ffn1024 L6 (5.14M params)", "tiles": vr["tiles"]},
        "p50_ms_per_batch": round(float(np.percentile(vr["batch_ms"], 50)), 3),
        "p99_ms_per_batch": round(float(np.percentile(vr["batch_ms"], 99)), 3),
        "p50_ms_per_event_amortised": round(float(np.percentile(per_event, 50)), 4),
        "p99_ms_per_event_amortised": round(float(np.percentile(per_event, 99)), 4),
        "eager_ms_per_step": round(vr["eager_ms_per_step"], 3),
        "forward_tflops": round(vr["flops"] / vr["wall_s"] / 1e12, 1),
        "fp32_plain": pl,
        "bf16_plain": pb,
        "small_fp32_one_event": sm,
        "roofline": {"bound": "mfma", "kernel": "attention", "achieved": round(achieved, 1),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic, "traffic_unit": "bytes per launch (HBM)",
                     "traffic_gb_per_s": (round(traffic / (attn_avg_ms * 1e-3) / 1e9, 1)
                                          if traffic is not None else None),
                     "avg_launch_ms": round(attn_avg_ms, 4),
                     # One exp2 per score: h * sum N^2 per launch, against the transcendental rate.
                     "exp_ceiling": {"achieved": round(exp_rate, 2), "peak": round(PEAK_EXP_T_PER_S, 2),
                                     "unit": "Texp/s", "frac": round(exp_rate / PEAK_EXP_T_PER_S, 4)}},
        "kernel_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in vr["prof"].items()},
        "candidates": vr["candidates"],
        "paper_layout_bf16": pl_layout,
        "bf16_fp8ffn": fp8,
        "partitioned_bf16": part,
    }
    if args.serve_rates:
        line["serving"] = bench_serving(args, cfg, w)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], refs = cpu_baseline(cfg, w, args.cpu_budget)
        # Error per output against the oracle on the events it ran, for each precision's outputs of
        # the first varlen batch (BF16 and FP8 from their benchmark legs, FP32 from one launch).
        from paper_2601_17554_amd import binding as B
        import torch
        pk0 = make_batches(1)[0]
        m32 = B.Model(cfg, w, "fp32")
        o32 = m32.reconstruct(torch.from_numpy(pk0.x).cuda(), B.Batch.from_host(pk0.row_start, pk0.n_valid))
        torch.cuda.synchronize()
        o32 = {k: v.cpu().numpy() for k, v in o32.items()}
        line["errors"] = output_errors(refs, {"bf16": vr["out0"], "bf16_fp8ffn": fp8_out0,
                                              "fp32": o32}, pk0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
