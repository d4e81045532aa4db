"""Tile-shape autotuner for libmlpf.

For one workload (model, device batch), every op's tile shapes (mlpf_tune_count) are timed with the
library's HIP-event profiler while the other ops keep their current choice; the fastest shape that
passes the correctness guard is pinned with mlpf_tune_set. The guard compares the final outputs of
each candidate with a reference run under the choices made so far (with the op's product unfused,
and the two-product FFN for the FFN's shapes): GEMM tiles and the fused FFN shapes must give
bitwise identical outputs where the library guarantees it (BF16 and FP8 always; FP32 for equal
k-tile lengths), and otherwise agree to the rounding level of the precision (relative to the
output scale: 1e-4 in FP32, 2e-2 in BF16 and FP8), as attention tiles and key splits must (they
change only the order and offsets of the softmax sums), the split FFN shapes (the order of the
partial sums) and the fused heads (the order of the second-layer sums). Choices are cached in a JSON file
(``MLPF_AUTOTUNE_CACHE``, default ``~/.cache/mlpf_autotune.json``) keyed by GPU architecture,
precision, model sizes and the batch's size bucket.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

import torch

from . import binding as B

# Profiler class that times each op (ops sharing a class are compared with the others fixed).
_CLASS = {"embed1": ("embed",), "embed2": ("embed",), "qkv": ("qkv",), "outproj": ("outproj",),
          "ffn1": ("ffn1",), "ffn2": ("ffn2",), "heads1": ("heads",), "attention": ("attention",),
          # the FFN's shapes also decide whether LN2 and the next LN1 run as kernels of their own
          # (timed with the output projection and the Q/K/V projection) or inside the FFN
          "ffn": ("ffn1", "ffn2", "outproj", "qkv"), "heads": ("heads",), "attn_split": ("attention",)}

# Products that a fused kernel replaces by default: (product -> op whose tile 0 runs them unfused).
# The ops are tuned in B.OPS order, so each fused op is decided after its products' tiles.
_UNFUSED = {"ffn1": "ffn", "ffn2": "ffn", "heads1": "heads"}


def cache_path() -> str:
    return os.environ.get("MLPF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mlpf_autotune.json"))


def cache_key(model: B.Model, batch: B.Batch) -> str:
    c = model.cfg
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    rows = 1 << max(0, math.ceil(math.log2(max(batch.total_rows, 1))))
    return (f"{arch}|{model.precision}|d{c.d_model}h{c.n_heads}ff{c.d_ff}L{c.n_layers}{c.topology}"
            f"|rows{rows}|ev{batch.n_events}")


def _run(model, x, batch, ws, out, reps: int) -> Dict[str, float]:
    model.reconstruct(x, batch, ws=ws, out=out)
    torch.cuda.synchronize()
    model.profiler_enable(True)
    for _ in range(reps):
        model.reconstruct(x, batch, ws=ws, out=out)
    torch.cuda.synchronize()
    prof = model.profiler_read()
    model.profiler_enable(False)
    return {k: v[0] / reps for k, v in prof.items()}


def _same(a: Dict[str, torch.Tensor], b: Dict[str, torch.Tensor], exact: bool, tol: float) -> bool:
    if exact:
        return all(torch.equal(a[k], b[k]) for k in ("logits", "reg", "cls"))
    scale = max(float(a["logits"].abs().max()), 1e-6)
    return float((a["logits"] - b["logits"]).abs().max()) <= tol * scale and \
        float((a["reg"] - b["reg"]).abs().max()) <= tol * max(float(a["reg"].abs().max()), 1e-6)


def tune(model: B.Model, x: torch.Tensor, batch: B.Batch, ws: Optional[torch.Tensor] = None,
         reps: int = 3, use_cache: bool = True, verbose: bool = False) -> Dict[str, int]:
    """Chooses and pins a tile shape per op for this workload; returns {op: tile}."""
    key = cache_key(model, batch)
    path = cache_path()
    if use_cache and os.path.exists(path):
        try:
            cached = json.load(open(path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached:
            for op, t in cached.items():
                model.tune_set(op, int(t))
            return {op: int(t) for op, t in cached.items()}
    if ws is None:
        ws = model.workspace(batch.total_rows, batch.n_events)
    out = model.outputs(batch.total_rows)
    for op in B.OPS:
        model.tune_set(op, -1)
    ref_bkb = B.Model.tune_shape("qkv", 0)["bkb"]  # FP32: the size-based rule picks among tiles 0..2
    choice: Dict[str, int] = {}
    for op in B.OPS:
        best, best_t = None, float("inf")
        parent = _UNFUSED.get(op)
        if parent:  # time the product's tiles with the fused kernel that replaces it switched off
            model.tune_set(parent, 0)
        if op == "ffn":  # the fused FFN shapes are bitwise equal to the two-product FFN (tile 0)
            model.tune_set(op, 0)
        # The guard's reference: the outputs of the choices made so far, with this op's product
        # unfused (a choice that changes the rounding, such as an attention tile, moves the bits).
        model.reconstruct(x, batch, ws=ws, out=out)
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in out.items()}
        for tile in range(B.Model.tune_count(op)):
            try:
                model.tune_set(op, tile)
            except B.MlpfError:  # a shape this model cannot run (e.g. the fused FFN outside BF16)
                continue
            prof = _run(model, x, batch, ws, out, reps)
            t = sum(prof[c] for c in _CLASS[op])
            # (the reference ran the fused heads, whose sums the unfused heads1 tiles reorder)
            # (the FFN's split tiles add partial products: rounding, not bits)
            exact = (op == "ffn" and B.Model.tune_shape(op, tile)["fused"] <= 1) or (
                op not in ("ffn", "attention", "attn_split", "heads", "heads1") and (
                model.precision != "fp32" or B.Model.tune_shape(op, tile)["bkb"] == ref_bkb))
            ok = _same(out, ref, exact, 1e-4 if model.precision == "fp32" else 2e-2)
            if verbose:
                print(f"autotune {op} tile {tile}: {t:.4f} ms {'ok' if ok else 'REJECTED'}", flush=True)
            if ok and t < best_t:
                best, best_t = tile, t
        model.tune_set(op, best if best is not None else -1)
        choice[op] = best if best is not None else -1
        if parent:
            model.tune_set(parent, -1)
    if use_cache:
        try:
            data = json.load(open(path)) if os.path.exists(path) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = choice
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return choice
