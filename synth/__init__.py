"""Seeded synthetic inputs for the MLPF forward pass: model configurations, weights, events.

This module draws random numbers and lays them out; it computes none of the method's arithmetic.
Both the FP64 oracle and the GPU path take their inputs from here, and nothing else is shared
between them.

Workload recipe (the paper's CMS Run-3 samples are not available, so these stand in for them):
  * an event is a set of N PF elements (tracks and calorimeter clusters), each a feature vector
    (paper Sec. 5.3); here every element has 17 float features: columns 0-5 are the one-hot of an
    element-type id t ~ Uniform{1..6} (column t-1), columns 6-16 are iid N(0, 1);
  * N is log-normal with median 3000 and sigma 0.5, rounded and clipped to [lo, 8192]
    (lo = 500 for single events, 200 for varlen batches); the paper quotes about 5,000 elements
    per event with pileup (Sec. 5.3);
  * weights ~ N(0, 0.02) for every Linear weight and bias, LayerNorm gamma = 1 + 0.02 z,
    beta = 0.02 z, drawn from PCG64(seed) in the canonical order listed by ``param_names``;
  * primary-element p_T and E for the optional decode (Eq. 2 inverse) are log-normal(0, 1).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Output heads in canonical order: (name, width). The classification head gives 6 logits
# (class 0 = no particle, 1..5 = particle types); the regression heads give
# p_T' (log-ratio, Eq. 2), eta, (sin phi, cos phi) and E' (log-ratio, Eq. 2).
HEADS: Tuple[Tuple[str, int], ...] = (("cls", 6), ("pt", 1), ("eta", 1), ("phi", 2), ("e", 1))
# With a separate binary head (the paper's six heads, Sec. 5.3): the classification outputs come
# from a binary "is a particle" head (width 1) and a particle-type head (width 5), both two-layer.
HEADS_BINARY: Tuple[Tuple[str, int], ...] = (("binary", 1), ("pid", 5), ("pt", 1), ("eta", 1),
                                             ("phi", 2), ("e", 1))
N_FEATURES = 17
N_TYPES = 6
MAX_SEQLEN = 8192


@dataclasses.dataclass(frozen=True)
class Config:
    """Model sizes. ``topology`` is 'serial' (one stack of n_layers, all heads read it) or
    'parallel2' (two stacks of n_layers/2 fed by the same embedding: the first feeds the
    classification head, the second the regression heads, as in paper Sec. 5.3)."""

    n_features: int = N_FEATURES
    d_model: int = 256
    n_heads: int = 8
    d_ff: int = 1024
    n_layers: int = 6
    topology: str = "serial"
    ln_eps: float = 1e-5
    activation: str = "gelu"  # or "relu" (the paper's network, Sec. 5.3)
    decision: str = "argmax"  # or "binary": output 0 a binary score, 1..5 particle types (Sec. 5.3)
    embed_per_type: bool = False  # tracks (type 0) and other elements embedded separately (Sec. 5.3)
    binary_head: bool = False  # separate two-layer binary and particle-type heads (Sec. 5.3)

    @property
    def d_head(self) -> int:
        return self.d_model // self.n_heads


SMALL = Config(d_model=64, n_heads=4, d_ff=256, n_layers=3)
FULL = Config(d_model=256, n_heads=8, d_ff=1024, n_layers=6)
# The paper's own layout (Sec. 5.3): 2 parallel encoders of 3 blocks, 16 heads of width 16.
PAPER = Config(d_model=256, n_heads=16, d_ff=1024, n_layers=6, topology="parallel2")
# The paper's network in full (Sec. 5.3): that layout with ReLU activations, separate track and
# other-element embeddings, six two-layer heads (binary and particle type on the classification
# encoder, p_T, eta, phi and E on the regression encoder) and the binary-score class rule.
PAPER_MODEL = Config(d_model=256, n_heads=16, d_ff=1024, n_layers=6, topology="parallel2",
                     activation="relu", decision="binary", embed_per_type=True, binary_head=True)


def heads_of(cfg: Config) -> Tuple[Tuple[str, int], ...]:
    """The output heads of a configuration, in canonical order: (name, width)."""
    return HEADS_BINARY if getattr(cfg, "binary_head", False) else HEADS


def param_shapes(cfg: Config) -> List[Tuple[str, Tuple[int, ...]]]:
    """Canonical parameter order and shapes. Linear weights are stored [in, out] (y = x W + b)."""
    d, f, dff = cfg.d_model, cfg.n_features, cfg.d_ff
    out: List[Tuple[str, Tuple[int, ...]]] = [
        ("embed.W1", (f, d)), ("embed.b1", (d,)), ("embed.W2", (d, d)), ("embed.b2", (d,)),
    ]
    if cfg.embed_per_type:
        out += [("embed_cl.W1", (f, d)), ("embed_cl.b1", (d,)), ("embed_cl.W2", (d, d)),
                ("embed_cl.b2", (d,))]
    for layer in range(cfg.n_layers):
        p = f"layers.{layer}."
        out += [
            (p + "ln1.gamma", (d,)), (p + "ln1.beta", (d,)),
            (p + "W_qkv", (d, 3 * d)), (p + "b_qkv", (3 * d,)),
            (p + "W_o", (d, d)), (p + "b_o", (d,)),
            (p + "ln2.gamma", (d,)), (p + "ln2.beta", (d,)),
            (p + "W_1", (d, dff)), (p + "b_1", (dff,)),
            (p + "W_2", (dff, d)), (p + "b_2", (d,)),
        ]
    for name, width in heads_of(cfg):
        p = f"heads.{name}."
        out += [(p + "W1", (d, d)), (p + "b1", (d,)), (p + "W2", (d, width)), (p + "b2", (width,))]
    return out


def param_count(cfg: Config) -> int:
    return int(sum(int(np.prod(s)) for _, s in param_shapes(cfg)))


def make_weights(cfg: Config, seed: int, sharpen: float = 1.0, head_gain: float = 1.0,
                 embed_gain: float = 1.0) -> Dict[str, np.ndarray]:
    """FP32 master weights, drawn in canonical order from PCG64(seed).

    ``sharpen`` multiplies the query and key column blocks of every W_qkv, which spreads the
    attention logits so that the softmax is far from uniform (used by parity tests only).
    ``embed_gain`` multiplies the weight matrices (not the biases) of the embedding network(s) and
    ``head_gain`` the second-layer weight W2 of every output head. With N(0, 0.02) weights every
    element of an event ends up with nearly the same outputs (the biases along the residual path
    dominate the per-element part by ~20x, and every output column is a small difference of
    similar terms); larger embedding weights make the per-element part dominate, and the head gain
    sets the output scale. ``WIDE`` is the "wide-output" set of the parity tests: every logit and
    regression column then varies by O(0.1-1) from element to element, each column is
    well-conditioned, and a zeroed, swapped or mis-scaled output column is far outside any
    tolerance. The random draws are the same for every gain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w: Dict[str, np.ndarray] = {}
    for name, shape in param_shapes(cfg):
        z = rng.standard_normal(shape)
        if name.endswith(".gamma"):
            v = 1.0 + 0.02 * z
        else:
            v = 0.02 * z
        if name.endswith("W_qkv") and sharpen != 1.0:
            v = v.copy()
            v[:, : 2 * cfg.d_model] *= sharpen
        if name.startswith("heads.") and name.endswith(".W2") and head_gain != 1.0:
            v = v * head_gain
        if name.startswith("embed") and ".W" in name and embed_gain != 1.0:
            v = v * embed_gain
        w[name] = v.astype(np.float32)
    return w


# The "wide-output" weight set of the parity tests (make_weights(cfg, seed, **WIDE)).
WIDE = {"embed_gain": 6.0, "head_gain": 10.0}


def make_features(rng: np.random.Generator, n: int, n_features: int = N_FEATURES) -> np.ndarray:
    """[n, n_features] float32: one-hot element type in columns 0-5, N(0,1) elsewhere."""
    x = np.zeros((n, n_features), dtype=np.float32)
    if n:
        t = rng.integers(1, N_TYPES + 1, size=n)
        x[np.arange(n), t - 1] = 1.0
        x[:, N_TYPES:] = rng.standard_normal((n, n_features - N_TYPES)).astype(np.float32)
    return x


def sample_count(rng: np.random.Generator, lo: int, hi: int = MAX_SEQLEN,
                 median: float = 3000.0, sigma: float = 0.5) -> int:
    z = rng.standard_normal()
    return int(np.clip(np.rint(median * np.exp(sigma * z)), lo, hi))


@dataclasses.dataclass
class Event:
    x: np.ndarray            # [n, F] float32
    prim: np.ndarray         # [n, 2] float32: primary-element (p_T, E), both > 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def make_event(seed, n: Optional[int] = None, lo: int = 500, n_features: int = N_FEATURES) -> Event:
    """One event from a seed (int or SeedSequence). If n is None it is drawn log-normally."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n is None:
        n = sample_count(rng, lo)
    x = make_features(rng, n, n_features)
    prim = np.exp(rng.standard_normal((n, 2))).astype(np.float32)
    return Event(x=x, prim=prim)


def event_set(root_seed: int, count: int, lo: int = 500) -> List[Event]:
    """``count`` events from SeedSequence(root_seed).spawn(count)."""
    return [make_event(s, None, lo) for s in np.random.SeedSequence(root_seed).spawn(count)]


def event_of_set(root_seed: int, count: int, index: int, lo: int = 500) -> Event:
    """Event ``index`` of event_set(root_seed, count, lo), without drawing the others."""
    return make_event(np.random.SeedSequence(root_seed).spawn(count)[index], None, lo)


def event_set_counts(root_seed: int, count: int, lo: int = 500) -> np.ndarray:
    """The element counts of event_set(root_seed, count, lo) (the first draw of each event)."""
    return np.array([sample_count(np.random.Generator(np.random.PCG64(s)), lo)
                     for s in np.random.SeedSequence(root_seed).spawn(count)], dtype=np.int64)


@dataclasses.dataclass
class Packed:
    """Events packed row-wise. Rows of event e are row_start[e] .. row_start[e+1]-1, of which the
    first n_valid[e] are elements and the rest padding."""

    x: np.ndarray            # [total_rows, F] float32
    prim: np.ndarray         # [total_rows, 2] float32
    row_start: np.ndarray    # [n_events + 1] int32
    n_valid: np.ndarray      # [n_events] int32

    @property
    def total_rows(self) -> int:
        return int(self.row_start[-1])

    @property
    def n_events(self) -> int:
        return int(self.n_valid.shape[0])

    @property
    def max_seqlen(self) -> int:
        return int(self.n_valid.max()) if self.n_valid.size else 0

    def event_rows(self, e: int) -> slice:
        s = int(self.row_start[e])
        return slice(s, s + int(self.n_valid[e]))


def pack(events: Sequence[Event], pad_to: int = 1, pad_fill: float = 0.0,
         seed: int = 0) -> Packed:
    """Pack events row-wise; each event's span is rounded up to a multiple of ``pad_to``.

    Padding rows hold ``pad_fill`` if it is finite and zero, or uniform garbage in
    [-|pad_fill|, |pad_fill|] otherwise (drawn from ``seed``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spans = [((e.n + pad_to - 1) // pad_to) * pad_to for e in events]
    row_start = np.zeros(len(events) + 1, dtype=np.int32)
    row_start[1:] = np.cumsum(spans)
    total = int(row_start[-1])
    f = events[0].x.shape[1] if events else N_FEATURES
    x = np.zeros((total, f), dtype=np.float32)
    prim = np.ones((total, 2), dtype=np.float32)
    for i, e in enumerate(events):
        s = int(row_start[i])
        x[s:s + e.n] = e.x
        prim[s:s + e.n] = e.prim
        pad = spans[i] - e.n
        if pad and pad_fill != 0.0:
            x[s + e.n:s + spans[i]] = rng.uniform(-abs(pad_fill), abs(pad_fill),
                                                  (pad, f)).astype(np.float32)
    n_valid = np.array([e.n for e in events], dtype=np.int32)
    return Packed(x=x, prim=prim, row_start=row_start, n_valid=n_valid)


def poisson_arrivals(rate_hz: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds, ascending) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
