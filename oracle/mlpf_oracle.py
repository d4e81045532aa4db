"""FP64 CPU oracle of the MLPF forward pass. TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module. It
is a plain, slow, obviously correct NumPy implementation of what the paper's model computes; it
shares no code with the GPU library and is never on the product path.

What it follows (arxiv 2601.17554):
  * Sec. 5.3, "The MLPF algorithm": the input is the set X of N element feature vectors of one
    event; every element gets a particle-type prediction and a four-momentum
    (p_T, eta, sin phi, cos phi, E). The pipeline is an embedding feed-forward network, transformer
    encoder blocks with LayerNorm before each block, and two-layer feed-forward output heads;
    at inference the particle type is the class with the largest score.
  * Eq. 4: scaled dot-product attention A = softmax(Q K^T / sqrt(d_k)), each row of A is positive
    and sums to one. FlashAttention gives exactly these values, so the oracle uses the plain
    materialised form (the fallback the paper names for hardware without a fused kernel).
  * Eq. 2: the regression targets for p_T and E are log-ratios to the primary element; ``decode``
    inverts them.
  * Sec. 5.3 (inference rule) and Sec. 8 (the reconstruction module turns the model outputs into a
    list of particle candidates per event): ``candidates`` keeps, event by event and in element
    order, the elements whose predicted class is a particle, with their class and decoded
    four-momentum.
  * Sec. 5.3 (closing remark: partitioning the event before the correlation-building layers) and
    Sec. 9 (sparse or block attention): with ``parts`` (a partition label per element) every
    attention layer takes as keys of an element only the elements of its own partition (a
    block-diagonal attention mask); everything else in the network acts on each element alone and
    is unchanged. This is an approximation of the full-event model, not the same function.

Readings where the paper is silent (each is listed with its reason in the design notes):
  * serial topology by default (one stack of L blocks read by all heads); 'parallel2' is the
    paper's two-encoder form: stack A = first L/2 blocks -> classification head, stack B = last
    L/2 blocks -> regression heads, both fed by the same embedding;
  * activation: exact-erf GELU after every hidden linear layer, none after output layers; the
    paper's own network uses ReLU there (Sec. 5.3), available as cfg.activation = 'relu';
  * pre-LN blocks: H += MHA(LN1(H)); H += FFN(LN2(H)); no final LayerNorm; eps 1e-5; biased
    variance; affine gamma/beta;
  * attention: Q/K/V/O biases, contiguous head split (head j owns columns j*d_h..(j+1)*d_h-1),
    bidirectional, only the event's own valid elements are keys, no dropout;
  * embedding: Linear(F, d) -> GELU -> Linear(d, d), one network for all element types; with
    cfg.embed_per_type, type-0 elements (tracks) and the others use separate networks (Sec. 5.3);
  * heads (cls 6, p_T' 1, eta 1, phi 2, E' 1): Linear(d, d) -> GELU -> Linear(d, width);
    with cfg.binary_head the classification outputs come from the paper's two separate heads
    instead (Sec. 5.3 and the caption of its model figure: a binary output and multi-class
    particle-type outputs): a binary head of width 1 and a particle-type head of width 5, both
    two-layer, both reading the classification encoder; the six logits are then
    (binary, type 1..5);
  * class 0 means "no particle"; argmax ties go to the lowest index. With cfg.decision = 'binary'
    output 0 is read as the paper's binary score and 1..5 as its particle-type scores (Sec. 5.3):
    kept when the sigmoid of output 0 exceeds 0.5, typed by the largest of 1..5.

Every function works in float64 on one event at a time; events never interact.
"""
from __future__ import annotations

import math
from typing import Dict, Mapping

import numpy as np
from scipy.special import erf

HEAD_WIDTHS = (("cls", 6), ("pt", 1), ("eta", 1), ("phi", 2), ("e", 1))
# The paper's classification heads (Sec. 5.3), used instead of "cls" when cfg.binary_head is set.
CLS_HEADS_BINARY = (("binary", 1), ("pid", 5))


def gelu(z: np.ndarray) -> np.ndarray:
    """GELU(z) = z * Phi(z) = z/2 * (1 + erf(z / sqrt 2)), the exact (erf) form."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def relu(z: np.ndarray) -> np.ndarray:
    """ReLU(z) = max(z, 0), the activation of the paper's network (Sec. 5.3)."""
    return np.maximum(np.asarray(z, dtype=np.float64), 0.0)


ACTIVATIONS = {"gelu": gelu, "relu": relu}


def layer_norm(z: np.ndarray, gamma: np.ndarray, beta: np.ndarray, eps: float) -> np.ndarray:
    """Per row: (z - mean) / sqrt(var + eps) * gamma + beta, with the biased variance."""
    mu = z.mean(axis=-1, keepdims=True)
    var = ((z - mu) ** 2).mean(axis=-1, keepdims=True)
    return (z - mu) / np.sqrt(var + eps) * gamma + beta


def softmax_rows(s: np.ndarray) -> np.ndarray:
    """Row-wise softmax, shifted by the row maximum (the shift cancels exactly)."""
    e = np.exp(s - s.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def sdpa(q: np.ndarray, k: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Eq. 4 for one head: softmax(Q K^T / sqrt(d_k)) V with the attention matrix materialised.
    q: [Nq, d_k], k: [Nk, d_k], v: [Nk, d_v]."""
    a = softmax_rows(q @ k.T / math.sqrt(q.shape[-1]))
    return a @ v


def attention_matrix(q: np.ndarray, k: np.ndarray) -> np.ndarray:
    """The matrix A of Eq. 4 (for the row-sum and positivity checks)."""
    return softmax_rows(q @ k.T / math.sqrt(q.shape[-1]))


def mha(y: np.ndarray, w_qkv, b_qkv, w_o, b_o, n_heads: int, parts=None) -> np.ndarray:
    """Multi-head self-attention over the rows of y ([N, d]); returns [N, d] (before residual).
    With ``parts`` ([N] labels) each row attends only to the rows of its own label."""
    d = y.shape[-1]
    dh = d // n_heads
    qkv = y @ w_qkv + b_qkv
    q, k, v = qkv[:, :d], qkv[:, d:2 * d], qkv[:, 2 * d:]
    if parts is None:
        groups = [np.arange(y.shape[0])]
    else:
        parts = np.asarray(parts)
        groups = [np.flatnonzero(parts == lab) for lab in np.unique(parts)]
    o = np.zeros((y.shape[0], d))
    for idx in groups:
        if idx.size == 0:
            continue
        for j in range(n_heads):
            c = slice(j * dh, (j + 1) * dh)
            o[idx, c] = sdpa(q[idx, c], k[idx, c], v[idx, c])
    return o @ w_o + b_o


def encoder_block(h: np.ndarray, p: Mapping[str, np.ndarray], n_heads: int, eps: float,
                  act=gelu, parts=None) -> np.ndarray:
    """One pre-LN transformer block: LayerNorm before attention and before the FFN."""
    y = layer_norm(h, p["ln1.gamma"], p["ln1.beta"], eps)
    h = h + mha(y, p["W_qkv"], p["b_qkv"], p["W_o"], p["b_o"], n_heads, parts)
    y = layer_norm(h, p["ln2.gamma"], p["ln2.beta"], eps)
    return h + act(y @ p["W_1"] + p["b_1"]) @ p["W_2"] + p["b_2"]


def embed(x: np.ndarray, w: Mapping[str, np.ndarray], act=gelu) -> np.ndarray:
    """Element embedding FFN: Linear(F, d) -> activation -> Linear(d, d)."""
    return act(x @ w["embed.W1"] + w["embed.b1"]) @ w["embed.W2"] + w["embed.b2"]


def embed_per_type(x: np.ndarray, w: Mapping[str, np.ndarray], act=gelu) -> np.ndarray:
    """Separate embeddings for tracks and the other elements (Sec. 5.3): a row whose element type
    is 0 (feature 0, the one-hot of type 0, is set) goes through the 'embed' network, any other row
    through the 'embed_cl' network of the same shape."""
    track = np.asarray(x)[:, 0] > 0.5
    h_t = act(x @ w["embed.W1"] + w["embed.b1"]) @ w["embed.W2"] + w["embed.b2"]
    h_c = act(x @ w["embed_cl.W1"] + w["embed_cl.b1"]) @ w["embed_cl.W2"] + w["embed_cl.b2"]
    return np.where(track[:, None], h_t, h_c)


def head(h: np.ndarray, w: Mapping[str, np.ndarray], name: str, act=gelu) -> np.ndarray:
    """Two-layer FFN head: Linear(d, d) -> activation -> Linear(d, width)."""
    p = f"heads.{name}."
    return act(h @ w[p + "W1"] + w[p + "b1"]) @ w[p + "W2"] + w[p + "b2"]


def argmax_lowest(logits: np.ndarray) -> np.ndarray:
    """Index of the largest logit per row; on exact ties the lowest index wins."""
    return np.argmax(logits, axis=-1).astype(np.int32)


def decide_binary(logits: np.ndarray) -> np.ndarray:
    """The paper's inference rule (Sec. 5.3) with output 0 a binary "is a particle" logit and
    outputs 1..5 the particle-type logits: keep the element when sigmoid(logit_0) > 0.5, and give it
    the type of the largest probability (softmax is monotone, so the largest logit); 0 otherwise."""
    logits = np.asarray(logits, dtype=np.float64)
    keep = 1.0 / (1.0 + np.exp(-logits[:, 0])) > 0.5
    return np.where(keep, 1 + argmax_lowest(logits[:, 1:]), 0).astype(np.int32)


def _as64(w: Mapping[str, np.ndarray]) -> Dict[str, np.ndarray]:
    return {k: np.asarray(v, dtype=np.float64) for k, v in w.items()}


def _layer_params(w: Mapping[str, np.ndarray], layer: int) -> Dict[str, np.ndarray]:
    pre = f"layers.{layer}."
    return {k[len(pre):]: v for k, v in w.items() if k.startswith(pre)}


def forward(x: np.ndarray, weights: Mapping[str, np.ndarray], cfg, parts=None) -> Dict[str, np.ndarray]:
    """The forward pass for ONE event's valid elements x ([N, F]); ``parts`` ([N] labels, or None)
    restricts every attention layer to the elements of the same label.

    Returns float64 'logits' [N, 6], 'reg' [N, 5] = (p_T', eta, sin phi, cos phi, E'),
    int32 'cls' [N] and the encoder outputs 'h_cls', 'h_reg' (identical for 'serial')."""
    w = _as64(weights)
    x = np.asarray(x, dtype=np.float64)
    n_layers, n_heads, eps = cfg.n_layers, cfg.n_heads, cfg.ln_eps
    act = ACTIVATIONS[getattr(cfg, "activation", "gelu")]
    h0 = embed_per_type(x, w, act) if getattr(cfg, "embed_per_type", False) else embed(x, w, act)
    if cfg.topology == "serial":
        h = h0
        for layer in range(n_layers):
            h = encoder_block(h, _layer_params(w, layer), n_heads, eps, act, parts)
        h_cls = h_reg = h
    elif cfg.topology == "parallel2":
        half = n_layers // 2
        h_cls = h0
        for layer in range(half):
            h_cls = encoder_block(h_cls, _layer_params(w, layer), n_heads, eps, act, parts)
        h_reg = h0
        for layer in range(half, n_layers):
            h_reg = encoder_block(h_reg, _layer_params(w, layer), n_heads, eps, act, parts)
    else:
        raise ValueError(f"unknown topology {cfg.topology!r}")
    if getattr(cfg, "binary_head", False):
        logits = np.concatenate([head(h_cls, w, name, act) for name, _ in CLS_HEADS_BINARY],
                                axis=-1)
    else:
        logits = head(h_cls, w, "cls", act)
    reg = np.concatenate([head(h_reg, w, name, act) for name, _ in HEAD_WIDTHS[1:]], axis=-1)
    rule = getattr(cfg, "decision", "argmax")
    cls = decide_binary(logits) if rule == "binary" else argmax_lowest(logits)
    return {"logits": logits, "reg": reg, "cls": cls, "h_cls": h_cls, "h_reg": h_reg}


def forward_packed(packed, weights, cfg) -> Dict[str, np.ndarray]:
    """Run ``forward`` on every event of a packed batch separately; padding rows get NaN."""
    t = packed.total_rows
    logits = np.full((t, 6), np.nan)
    reg = np.full((t, 5), np.nan)
    cls = np.full((t,), -1, dtype=np.int32)
    for e in range(packed.n_events):
        rows = packed.event_rows(e)
        if rows.stop > rows.start:
            out = forward(packed.x[rows], weights, cfg)
            logits[rows], reg[rows], cls[rows] = out["logits"], out["reg"], out["cls"]
    return {"logits": logits, "reg": reg, "cls": cls}


def decode(reg: np.ndarray, prim: np.ndarray) -> Dict[str, np.ndarray]:
    """Invert Eq. 2: p_T = p_T^prim * exp(p_T'), E = E^prim * exp(E'); phi = atan2(sin, cos)."""
    reg = np.asarray(reg, dtype=np.float64)
    prim = np.asarray(prim, dtype=np.float64)
    return {"pt": prim[:, 0] * np.exp(reg[:, 0]), "eta": reg[:, 1],
            "phi": np.arctan2(reg[:, 2], reg[:, 3]), "e": prim[:, 1] * np.exp(reg[:, 4])}


def candidates(cls, kin, row_start, n_valid=None):
    """Particle candidates per event (Sec. 5.3 inference rule, Sec. 8 module output).

    cls: [T] predicted class per row (0 = no particle); kin: [T][k] per-row kinematics (the decoded
    p_T, eta, phi, E) or None; row_start: [n_events + 1]; n_valid: [n_events] or None (every row of
    an event is an element). Event e's elements are rows row_start[e] .. row_start[e] + n_valid[e] - 1.
    Returns (offsets [n_events + 1], rows [C], classes [C], kin [C][k] or None): event e's
    candidates are entries offsets[e] .. offsets[e+1] - 1, in element order; each entry names its
    row, its class and that row's kinematics.
    """
    cls = np.asarray(cls)
    row_start = np.asarray(row_start, dtype=np.int64)
    n_events = len(row_start) - 1
    offsets = [0]
    rows = []
    for e in range(n_events):
        n = row_start[e + 1] - row_start[e] if n_valid is None else n_valid[e]
        for i in range(int(n)):
            r = int(row_start[e]) + i
            if cls[r] != 0:
                rows.append(r)
        offsets.append(len(rows))
    rows = np.asarray(rows, dtype=np.int64)
    out_kin = None if kin is None else np.asarray(kin)[rows]
    return np.asarray(offsets, dtype=np.int64), rows, cls[rows], out_kin


def encode(pt_target, e_target, prim) -> np.ndarray:
    """Eq. 2 forward: (log(p_T^target / p_T^prim), log(E^target / E^prim))."""
    prim = np.asarray(prim, dtype=np.float64)
    return np.stack([np.log(np.asarray(pt_target, np.float64) / prim[:, 0]),
                     np.log(np.asarray(e_target, np.float64) / prim[:, 1])], axis=-1)


def flops_per_event(n: int, cfg) -> int:
    """Algorithmic FLOPs (2 per multiply-add, unpadded N) of one forward pass."""
    d, f, dff, L = cfg.d_model, cfg.n_features, cfg.d_ff, cfg.n_layers
    embed_f = 2 * n * (f * d + d * d)
    layer_f = 2 * n * (3 * d * d + d * d + 2 * d * dff) + 4 * n * n * d
    n_heads = 6 if getattr(cfg, "binary_head", False) else 5
    heads_f = 2 * n * (n_heads * d * d) + 2 * n * d * 11
    return embed_f + L * layer_f + heads_f
