"""ctypes binding of libmlpf (include/mlpf.h). Argument marshalling only: every step of the forward
pass runs in the library's HIP kernels; torch provides device memory and the stream.

The raw entry points keep the C names (``mlpf_embed``, ``mlpf_encoder_forward``, ``mlpf_heads``,
``mlpf_reconstruct_events``) and take torch tensors. ``Model`` owns the device weight buffer and
a workspace and is what tests and the benchmark use.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Mapping, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlpf.so")

MLPF_FP32, MLPF_BF16, MLPF_BF16_FP8FFN = 0, 1, 2
PRECISIONS = {"fp32": MLPF_FP32, "bf16": MLPF_BF16, "bf16_fp8ffn": MLPF_BF16_FP8FFN}
TOPOLOGIES = {"serial": 0, "parallel2": 1}
HEAD_WIDTHS = (("cls", 6), ("pt", 1), ("eta", 1), ("phi", 2), ("e", 1))
# With the paper's separate binary and particle-type heads (config binary_head).
HEAD_WIDTHS_BINARY = (("binary", 1), ("pid", 5), ("pt", 1), ("eta", 1), ("phi", 2), ("e", 1))
MAX_SEQLEN = 8192


class MlpfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("n_features", ctypes.c_int32), ("d_model", ctypes.c_int32),
                ("n_heads", ctypes.c_int32), ("d_ff", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("topology", ctypes.c_int32),
                ("ln_eps", ctypes.c_float), ("activation", ctypes.c_int32),
                ("decision", ctypes.c_int32), ("embed_per_type", ctypes.c_int32),
                ("binary_head", ctypes.c_int32)]


class _Batch(ctypes.Structure):
    pass


_Batch._fields_ = [("row_start", ctypes.c_void_p), ("n_valid", ctypes.c_void_p),
                   ("row_start_host", ctypes.c_void_p), ("n_valid_host", ctypes.c_void_p),
                   ("n_events", ctypes.c_int32), ("total_rows", ctypes.c_int32),
                   ("max_seqlen", ctypes.c_int32), ("attn_parts", ctypes.POINTER(_Batch))]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libmlpf.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2601_17554_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int
    cfgp, bp = ctypes.POINTER(_Config), ctypes.POINTER(_Batch)
    sig = {
        "mlpf_weights_bytes": (sz, [cfgp, st]),
        "mlpf_weights_count": (sz, [cfgp]),
        "mlpf_model_create": (st, [cfgp, st, vp, sz, vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "mlpf_model_destroy": (st, [vp]),
        "mlpf_workspace_bytes": (sz, [vp, i32, i32, i32]),
        "mlpf_embed": (st, [vp, vp, bp, vp, vp, sz, vp]),
        "mlpf_encoder_forward": (st, [vp, vp, bp, vp, sz, vp]),
        "mlpf_heads": (st, [vp, vp, bp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "mlpf_reconstruct_events": (st, [vp, vp, bp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "mlpf_reconstruct_events_noalloc": (st, [vp, vp, bp, vp, vp, vp, vp, vp, vp]),
        "mlpf_profiler_enable": (st, [vp, st]),
        "mlpf_profiler_read": (st, [vp, st, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]),
        "mlpf_attention_forward": (st, [vp, vp, vp, vp, vp, bp, vp, sz, vp]),
        "mlpf_calibrate_fp8": (st, [vp, vp, bp, vp, vp, sz, vp]),
        "mlpf_graph_create": (st, [vp, vp, bp, vp, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]),
        "mlpf_graph_launch": (st, [vp, vp]),
        "mlpf_graph_destroy": (st, [vp]),
        "mlpf_tune_count": (i32, [i32]),
        "mlpf_tune_set": (st, [vp, i32, i32]),
        "mlpf_tune_get": (i32, [vp, i32]),
        "mlpf_tune_shape": (st, [i32, i32, ctypes.POINTER(ctypes.c_int32)]),
        "mlpf_candidates": (st, [bp, vp, vp, vp, vp, vp, vp, i32, vp]),
        "mlpf_status_string": (ctypes.c_char_p, [st]),
        "mlpf_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    _lib = lib
    return lib


def exported_symbols() -> Sequence[str]:
    return ("mlpf_weights_bytes", "mlpf_weights_count", "mlpf_model_create", "mlpf_model_destroy",
            "mlpf_workspace_bytes", "mlpf_embed", "mlpf_encoder_forward", "mlpf_heads",
            "mlpf_reconstruct_events", "mlpf_reconstruct_events_noalloc", "mlpf_profiler_enable", "mlpf_profiler_read",
            "mlpf_attention_forward", "mlpf_calibrate_fp8", "mlpf_graph_create", "mlpf_graph_launch",
            "mlpf_graph_destroy", "mlpf_tune_count", "mlpf_tune_set", "mlpf_tune_get",
            "mlpf_tune_shape", "mlpf_candidates", "mlpf_status_string", "mlpf_last_error")


ACTIVATIONS = {"gelu": 0, "relu": 1}
DECISIONS = {"argmax": 0, "binary": 1}
PROF_CLASSES = ("embed", "qkv", "attention", "outproj", "ffn1", "ffn2", "heads", "worklist")
OPS = ("embed1", "embed2", "qkv", "outproj", "ffn1", "ffn2", "heads1", "attention", "ffn",
       "heads", "attn_split")


def _status_name(s: int) -> str:
    try:
        return load().mlpf_status_string(s).decode()
    except Exception:  # pragma: no cover - only while formatting another error
        return f"status {s}"


def _check(status: int) -> None:
    if status != 0:
        raise MlpfError(status, load().mlpf_last_error().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libmlpf must be contiguous")
    return t.data_ptr()


def _stream(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_config(cfg) -> _Config:
    """From any object with the config attributes (n_features, d_model, ...)."""
    return _Config(cfg.n_features, cfg.d_model, cfg.n_heads, cfg.d_ff, cfg.n_layers,
                   TOPOLOGIES[cfg.topology], cfg.ln_eps,
                   ACTIVATIONS[getattr(cfg, "activation", "gelu")],
                   DECISIONS[getattr(cfg, "decision", "argmax")],
                   1 if getattr(cfg, "embed_per_type", False) else 0,
                   1 if getattr(cfg, "binary_head", False) else 0)


def flatten_weights(weights: Mapping[str, np.ndarray], cfg) -> np.ndarray:
    """The master FP32 blob in the library's documented order (include/mlpf.h)."""
    names = ["embed.W1", "embed.b1", "embed.W2", "embed.b2"]
    if getattr(cfg, "embed_per_type", False):
        names += ["embed_cl.W1", "embed_cl.b1", "embed_cl.W2", "embed_cl.b2"]
    for layer in range(cfg.n_layers):
        names += [f"layers.{layer}.{s}" for s in
                  ("ln1.gamma", "ln1.beta", "W_qkv", "b_qkv", "W_o", "b_o",
                   "ln2.gamma", "ln2.beta", "W_1", "b_1", "W_2", "b_2")]
    heads = HEAD_WIDTHS_BINARY if getattr(cfg, "binary_head", False) else HEAD_WIDTHS
    for name, _ in heads:
        names += [f"heads.{name}.{s}" for s in ("W1", "b1", "W2", "b2")]
    return np.concatenate([np.ascontiguousarray(weights[n], dtype=np.float32).ravel() for n in names])


class Batch:
    """Device-side batch description: rows of event e are row_start[e]..row_start[e+1]-1, the first
    n_valid[e] of them valid. ``row_start_host`` / ``n_valid_host`` (int32 numpy arrays holding the
    same values) are the optional host mirrors the library validates before launching."""

    def __init__(self, row_start: torch.Tensor, n_valid: Optional[torch.Tensor], n_events: int,
                 total_rows: int, max_seqlen: int, row_start_host: Optional[np.ndarray] = None,
                 n_valid_host: Optional[np.ndarray] = None, parts: Optional["Batch"] = None):
        self.row_start, self.n_valid = row_start, n_valid
        self.n_events, self.total_rows, self.max_seqlen = n_events, total_rows, max_seqlen
        self.parts = parts  # attention partitions (mlpf_batch_t.attn_parts), a Batch, or None
        self.set_host_mirrors(row_start_host, n_valid_host)

    def set_host_mirrors(self, row_start_host: Optional[np.ndarray],
                         n_valid_host: Optional[np.ndarray]) -> None:
        def host(a):
            return None if a is None else np.ascontiguousarray(a, dtype=np.int32)
        self.row_start_host, self.n_valid_host = host(row_start_host), host(n_valid_host)
        hp = lambda a: None if a is None else a.ctypes.data
        parts = ctypes.pointer(self.parts._c) if self.parts is not None else None
        self._c = _Batch(_ptr(self.row_start), _ptr(self.n_valid), hp(self.row_start_host),
                         hp(self.n_valid_host), self.n_events, self.total_rows, self.max_seqlen,
                         parts)

    def with_parts(self, parts: Optional["Batch"]) -> "Batch":
        """Sets the attention partitions (a Batch over the same rows, or None); returns self."""
        self.parts = parts
        self.set_host_mirrors(self.row_start_host, self.n_valid_host)
        return self

    @property
    def work_events(self) -> int:
        """The event count that sizes workspaces: the larger of events and attention partitions."""
        return max(self.n_events, self.parts.n_events if self.parts is not None else 0)

    @classmethod
    def from_host(cls, row_start: np.ndarray, n_valid: Optional[np.ndarray], device="cuda",
                  max_seqlen: Optional[int] = None, mirrors: bool = True) -> "Batch":
        """Uploads the description; with ``mirrors`` the host arrays are kept as the validated
        host mirrors."""
        rs_h = np.ascontiguousarray(row_start, dtype=np.int32)
        nv_h = None if n_valid is None else np.ascontiguousarray(n_valid, dtype=np.int32)
        rs = torch.as_tensor(rs_h).to(device)
        nv = None if nv_h is None else torch.as_tensor(nv_h).to(device)
        n_events = len(rs_h) - 1
        total = int(rs_h[-1]) if n_events >= 0 and len(rs_h) else 0
        if max_seqlen is None:
            spans = np.diff(rs_h) if nv_h is None else nv_h
            max_seqlen = int(spans.max()) if len(spans) else 0
        return cls(rs, nv, n_events, total, max_seqlen, rs_h if mirrors else None,
                   nv_h if mirrors else None)

    @property
    def c(self):
        return ctypes.byref(self._c)


# ------------------------------------------------------------------ raw entry points (C names)

def mlpf_embed(model: "Model", x, batch: Batch, h, ws, stream=None) -> None:
    _check(load().mlpf_embed(model.handle, _ptr(x), batch.c, _ptr(h), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(stream)))


def mlpf_encoder_forward(model: "Model", h, batch: Batch, ws, stream=None) -> None:
    _check(load().mlpf_encoder_forward(model.handle, _ptr(h), batch.c, _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream)))


def mlpf_heads(model: "Model", h, batch: Batch, logits, reg, cls, prim, decoded, ws,
               stream=None) -> None:
    _check(load().mlpf_heads(model.handle, _ptr(h), batch.c, _ptr(logits), _ptr(reg), _ptr(cls),
                             _ptr(prim), _ptr(decoded), _ptr(ws), ws.numel() * ws.element_size(),
                             _stream(stream)))


def mlpf_reconstruct_events(model: "Model", x, batch: Batch, logits, reg, cls, prim, decoded, ws,
                            stream=None) -> None:
    _check(load().mlpf_reconstruct_events(model.handle, _ptr(x), batch.c, _ptr(logits), _ptr(reg),
                                          _ptr(cls), _ptr(prim), _ptr(decoded), _ptr(ws),
                                          ws.numel() * ws.element_size(), _stream(stream)))


def mlpf_reconstruct_events_noalloc(model: "Model", x, batch: Batch, logits, reg, cls, prim,
                                    decoded, stream=None) -> None:
    _check(load().mlpf_reconstruct_events_noalloc(model.handle, _ptr(x), batch.c, _ptr(logits),
                                                  _ptr(reg), _ptr(cls), _ptr(prim), _ptr(decoded),
                                                  _stream(stream)))


def mlpf_attention_forward(model: "Model", q, k, v, o, batch: Batch, ws, stream=None) -> None:
    _check(load().mlpf_attention_forward(model.handle, _ptr(q), _ptr(k), _ptr(v), _ptr(o), batch.c,
                                         _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def mlpf_candidates(batch: Batch, cls, decoded, event_offsets, cand_row, cand_cls, cand_kin,
                    cap: int, stream=None) -> None:
    _check(load().mlpf_candidates(batch.c, _ptr(cls), _ptr(decoded), _ptr(event_offsets),
                                  _ptr(cand_row), _ptr(cand_cls), _ptr(cand_kin), int(cap),
                                  _stream(stream)))


def candidates(batch: Batch, cls: torch.Tensor, decoded: Optional[torch.Tensor] = None,
               cap: Optional[int] = None, stream=None) -> Dict[str, torch.Tensor]:
    """Device candidate lists (mlpf_candidates) with cap = total_rows by default (nothing can be
    cut): {"offsets" [n_events + 1], "rows" [cap], "cls" [cap], "kin" [cap][4] if decoded}."""
    dev = cls.device
    cap = batch.total_rows if cap is None else cap
    out = {"offsets": torch.empty(batch.n_events + 1, dtype=torch.int32, device=dev),
           "rows": torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
           "cls": torch.empty(max(cap, 1), dtype=torch.int32, device=dev)}
    if decoded is not None:
        out["kin"] = torch.empty(max(cap, 1), 4, dtype=torch.float32, device=dev)
    mlpf_candidates(batch, cls, decoded, out["offsets"], out["rows"], out["cls"], out.get("kin"),
                    cap, stream)
    return out


def candidates_to_host(cands: Dict[str, torch.Tensor], stream=None) -> Dict[str, np.ndarray]:
    """Variable-length download: the offsets first, then only the first total entries."""
    s = stream if stream is not None else torch.cuda.current_stream()
    s.synchronize()
    offsets = cands["offsets"].cpu().numpy()
    total = min(int(offsets[-1]), cands["rows"].numel())
    out = {"offsets": offsets, "total": int(offsets[-1])}
    for k in ("rows", "cls", "kin"):
        if k in cands:
            out[k] = cands[k][:total].cpu().numpy()
    return out


def build_fp8_model(cfg, weights: Mapping[str, np.ndarray], calib: Sequence, device: str = "cuda",
                    calib_precision: str = "fp32") -> "Model":
    """An MLPF_BF16_FP8FFN model whose activation scales are calibrated on ``calib`` (a sequence of
    (x [T][F] float32 array, row_start, n_valid) host batches without padding rows): per-tensor
    amax of each block's FFN inputs on the calibration model (the library sets each scale from
    it)."""
    ref = Model(cfg, weights, calib_precision, device=device)
    amax = torch.zeros(2 * cfg.n_layers, dtype=torch.float32, device=device)
    for x, row_start, n_valid in calib:
        batch = Batch.from_host(row_start, n_valid, device=device)
        ref.calibrate_fp8(torch.from_numpy(np.ascontiguousarray(x)).to(device), batch, amax)
    torch.cuda.synchronize()
    return Model(cfg, weights, "bf16_fp8ffn", act_amax=amax.cpu().numpy(), device=device)


class Graph:
    """A captured mlpf_reconstruct_events call (see mlpf_graph_create). Holds references to every
    buffer it borrows. Capacity = the host sizes of ``batch``; rewrite x / row_start / n_valid /
    prim in place (same tensors) and call ``launch``."""

    def __init__(self, model: "Model", x, batch: "Batch", out: Dict[str, torch.Tensor], ws,
                 stream: torch.cuda.Stream, prim=None):
        self.model, self.x, self.batch, self.out, self.ws, self.prim = model, x, batch, out, ws, prim
        self.stream = stream
        handle = ctypes.c_void_p()
        _check(load().mlpf_graph_create(model.handle, _ptr(x), batch.c, _ptr(out["logits"]),
                                        _ptr(out["reg"]), _ptr(out["cls"]), _ptr(prim),
                                        _ptr(out.get("decoded")), _ptr(ws),
                                        ws.numel() * ws.element_size(), stream.cuda_stream,
                                        ctypes.byref(handle)))
        self.handle = handle

    def launch(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        s = stream if stream is not None else self.stream
        _check(load().mlpf_graph_launch(self.handle, s.cuda_stream))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mlpf_graph_destroy(h)
            self.handle = None


class Model:
    """A libmlpf model handle with its device weight buffer (allocated by torch)."""

    def __init__(self, cfg, weights: Mapping[str, np.ndarray], precision: str = "fp32",
                 act_amax: Optional[np.ndarray] = None, device: str = "cuda"):
        lib = load()
        self.cfg, self.precision, self.device = cfg, precision, device
        self._ccfg = make_config(cfg)
        prec = PRECISIONS[precision]
        blob = flatten_weights(weights, cfg)
        if blob.size != lib.mlpf_weights_count(ctypes.byref(self._ccfg)):
            raise ValueError("weight blob size does not match the configuration")
        nbytes = lib.mlpf_weights_bytes(ctypes.byref(self._ccfg), prec)
        if nbytes == 0:
            raise MlpfError(2, f"unsupported configuration/precision {cfg} {precision}")
        self.wbuf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        amax = None
        if act_amax is not None:
            self._amax = np.ascontiguousarray(act_amax, dtype=np.float32)
            amax = self._amax.ctypes.data
        handle = ctypes.c_void_p()
        _check(lib.mlpf_model_create(ctypes.byref(self._ccfg), prec, blob.ctypes.data, blob.size,
                                     amax, self.wbuf.data_ptr(), nbytes,
                                     _stream(None), ctypes.byref(handle)))
        self.handle = handle
        self.stacks = 2 if cfg.topology == "parallel2" else 1

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.mlpf_model_destroy(h)
            self.handle = None

    def profiler_enable(self, on: bool = True) -> None:
        _check(load().mlpf_profiler_enable(self.handle, 1 if on else 0))

    def profiler_read(self) -> Dict[str, tuple]:
        """{class: (total_ms, launches)}; the streams used must have been synchronised."""
        out = {}
        for i, name in enumerate(PROF_CLASSES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(load().mlpf_profiler_read(self.handle, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def tune_set(self, op: str, tile: int) -> None:
        _check(load().mlpf_tune_set(self.handle, OPS.index(op), tile))

    def tune_get(self, op: str) -> int:
        return int(load().mlpf_tune_get(self.handle, OPS.index(op)))

    @staticmethod
    def tune_count(op: str) -> int:
        return int(load().mlpf_tune_count(OPS.index(op)))

    @staticmethod
    def tune_shape(op: str, tile: int) -> Dict[str, int]:
        """Shape of one tile: GEMM ops {bm, bn, wm, wn, bkb, persist}; attention {waves, kt, qb,
        kind}; ffn {fused, rows, waves, double_buffered}; heads {fused, bm, bn}; attn_split
        {splits}."""
        v = (ctypes.c_int32 * 6)()
        _check(load().mlpf_tune_shape(OPS.index(op), tile, v))
        keys = (("waves", "kt", "qb", "kind") if op == "attention" else
                ("fused", "rows", "waves", "double_buffered", "persistent", "pipelined") if op == "ffn" else
                ("fused", "bm", "bn") if op == "heads" else
                ("splits",) if op == "attn_split"
                else ("bm", "bn", "wm", "wn", "bkb", "persist"))
        return {k: int(v[i]) for i, k in enumerate(keys)}

    def workspace_bytes(self, total_rows: int, n_events: int, max_seqlen: int = MAX_SEQLEN) -> int:
        return int(load().mlpf_workspace_bytes(self.handle, total_rows, max_seqlen, n_events))

    def workspace(self, total_rows: int, n_events: int, max_seqlen: int = MAX_SEQLEN) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(total_rows, n_events, max_seqlen), 1),
                           dtype=torch.uint8, device=self.device)

    def outputs(self, total_rows: int, decode: bool = False) -> Dict[str, torch.Tensor]:
        t = total_rows
        out = {"logits": torch.empty(t, 6, dtype=torch.float32, device=self.device),
               "reg": torch.empty(t, 5, dtype=torch.float32, device=self.device),
               "cls": torch.empty(t, dtype=torch.int32, device=self.device)}
        if decode:
            out["decoded"] = torch.empty(t, 4, dtype=torch.float32, device=self.device)
        return out

    def reconstruct(self, x: torch.Tensor, batch: Batch, prim: Optional[torch.Tensor] = None,
                    ws: Optional[torch.Tensor] = None, out: Optional[Dict[str, torch.Tensor]] = None,
                    stream=None) -> Dict[str, torch.Tensor]:
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        if out is None:
            out = self.outputs(batch.total_rows, decode=prim is not None)
        mlpf_reconstruct_events(self, x, batch, out["logits"], out["reg"], out["cls"], prim,
                                out.get("decoded"), ws, stream)
        return out

    def attention(self, q, k, v, batch: Batch, ws=None) -> torch.Tensor:
        """q, k, v: [n_heads][total_rows][d_head] tensors of the operand dtype (float32 or
        bfloat16); returns o [total_rows][d_model] (rows beyond an event's count untouched: 0)."""
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        o = torch.zeros(batch.total_rows, self.cfg.d_model, dtype=q.dtype, device=self.device)
        mlpf_attention_forward(self, q, k, v, o, batch, ws)
        return o

    def calibrate_fp8(self, x, batch: Batch, amax: torch.Tensor, ws=None) -> torch.Tensor:
        """Raises amax ([2 n_layers] float32, device) to the FFN input maxima on this batch."""
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        _check(load().mlpf_calibrate_fp8(self.handle, _ptr(x), batch.c, _ptr(amax), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(None)))
        return amax

    def embed(self, x, batch: Batch, ws=None) -> torch.Tensor:
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        h = torch.empty(self.stacks, batch.total_rows, self.cfg.d_model, dtype=self.residual_dtype,
                        device=self.device)
        mlpf_embed(self, x, batch, h, ws)
        return h

    @property
    def residual_dtype(self) -> torch.dtype:
        """Element type of the residual stream h: float32 for fp32 models, bfloat16 otherwise."""
        return torch.float32 if self.precision == "fp32" else torch.bfloat16

    def encoder(self, h: torch.Tensor, batch: Batch, ws=None) -> torch.Tensor:
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        mlpf_encoder_forward(self, h, batch, ws)
        return h

    def heads(self, h: torch.Tensor, batch: Batch, prim=None, ws=None) -> Dict[str, torch.Tensor]:
        if ws is None:
            ws = self.workspace(batch.total_rows, batch.work_events)
        out = self.outputs(batch.total_rows, decode=prim is not None)
        mlpf_heads(self, h, batch, out["logits"], out["reg"], out["cls"], prim, out.get("decoded"), ws)
        return out
