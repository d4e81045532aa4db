"""GPU parity of the fused masked varlen attention kernel alone (mlpf_attention_forward) against the
oracle's materialised SDPA (Eq. 4) on the same operands, element by element."""
import math

import numpy as np
import pytest

import synth
from oracle import mlpf_oracle as O

pytestmark = pytest.mark.gpu

# Normwise tolerance on O per (event, head): FP32 path vs FP64; BF16 path: P and O are rounded to
# bf16 (relative 2^-9 each), so a few 2^-9 on well-conditioned scores.
TOL = {"fp32": 1e-5, "bf16": 1.5e-2}


def _bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_17554_amd import binding
    binding.load()
    return binding


def _operands(kind, H, T, dh, spread, rng):
    """q, k, v of one of the input families: "random" (i.i.d. normal times spread), "low" (every
    score near -200 in log2 units), "shifted" (every
    query has a large component along a direction no key shares, and one key per event a large
    norm: the score bound |q| max|k| lies about 70 log2 units above the true maxima), "loose" (the
    same with the bound more than 96 above, which the BF16 kernel answers with an exact-maximum
    pass)."""
    q = rng.standard_normal((H, T, dh)).astype(np.float32) * spread
    k = rng.standard_normal((H, T, dh)).astype(np.float32) * spread
    v = rng.standard_normal((H, T, dh)).astype(np.float32)
    if kind == "low":
        # Every score of every query lies near -200 (log2 units, after the log2(e)/sqrt(dh)
        # prescale): the rows' maxima are far below 0, where an offset that starts at 0 instead
        # of at the first tile's maximum would overflow exp2.
        a = math.sqrt(200.0 * math.sqrt(dh) / 1.4426950408889634)
        q[:, :, 0] = -a
        k[:, :, 0] = a
        return q, k, v
    if kind != "random":
        big_q, big_k = (20.0, 14.0) if kind == "shifted" else (30.0, 16.0)
        q[:, :, 0] = big_q
        k[:, :, 0] = 0.0
        k[:, ::7, 1] = big_k
    return q, k, v


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("cfg", [synth.FULL, synth.SMALL], ids=["dh32", "dh16"])
@pytest.mark.parametrize("kind,spread", [("random", 1.0), ("random", 3.0), ("shifted", 0.5),
                                         ("loose", 0.5)], ids=["flat", "sharp", "shifted", "loose"])
def test_attention_alone(B, prec, cfg, kind, spread):
    # The rule splits this small launch's keys (BF16); split tile 0 runs it unsplit.
    _attention_case(B, prec, cfg, kind, spread, tile=-1)
    if prec == "bf16":
        _attention_case(B, prec, cfg, kind, spread, tile=-1, split=0)


SIZES = [1, 2, 5, 31, 33, 64, 65, 100, 130, 300]


def _attention_case(B, prec, cfg, kind, spread, tile, split=-1, sizes=SIZES):
    import torch
    rs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    T, H, dh = int(rs[-1]), cfg.n_heads, cfg.d_head
    rng = np.random.default_rng(7)
    q, k, v = _operands(kind, H, T, dh, spread, rng)
    if prec == "bf16":
        q, k, v = _bf16(q), _bf16(k), _bf16(v)
    m = B.Model(cfg, synth.make_weights(cfg, 0), prec)
    m.tune_set("attention", tile)
    m.tune_set("attn_split", split)
    tdt = torch.float32 if prec == "fp32" else torch.bfloat16
    dq, dk, dv = (torch.from_numpy(a).to(tdt).cuda() for a in (q, k, v))
    batch = B.Batch.from_host(rs, None)
    o = m.attention(dq, dk, dv, batch).float().cpu().numpy()
    # The kernel scores in log2 units with q pre-scaled by log2(e)/sqrt(dh) in the operand type.
    scale = np.float32(1.4426950408889634 / math.sqrt(dh))
    qs = (q * scale).astype(np.float32)
    if prec == "bf16":
        qs = _bf16(qs)
    worst = 0.0
    for e in range(len(sizes)):
        r = slice(int(rs[e]), int(rs[e + 1]))
        for j in range(H):
            ref = O.sdpa(qs[j, r].astype(np.float64) * math.log(2) * math.sqrt(dh),
                         k[j, r].astype(np.float64), v[j, r].astype(np.float64))
            got = o[r, j * dh:(j + 1) * dh]
            err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-6)
            worst = max(worst, err)
            tol = TOL[prec]
            if prec == "fp32":
                # FP32 scores of magnitude |s| (log2 units) carry an absolute rounding error of a
                # few |s| 2^-24, i.e. a relative error of that times ln 2 on every softmax weight,
                # which O passes on relative to max |v| (not to max |O|, which cancellation can make
                # much smaller): negligible but for the "low" family's |s| ~ 200.
                sv = np.abs(qs[j, r].astype(np.float64) @ k[j, r].astype(np.float64).T).max()
                tol += 4 * 2.0 ** -24 * sv * math.log(2) * np.abs(v[j, r]).max() / max(np.abs(ref).max(), 1e-6)
            assert err <= tol, (f"tile {tile} split {split} event {e} (n={sizes[e]}) head {j}: "
                                f"{err:.3e} > {tol:.3e}")
    print(f"{prec} dh={dh} {kind} spread={spread} tile {tile} split {split}: worst normwise error "
          f"{worst:.2e}")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kind,spread", [("random", 3.0), ("loose", 0.5), ("low", 0.3)],
                         ids=["sharp", "loose", "low"])
def test_attention_every_tile(B, prec, kind, spread):
    """Every attention kernel shape the tuner may pick, on the head size of the full model."""
    from paper_2601_17554_amd import binding
    for tile in range(binding.Model.tune_count("attention")):
        _attention_case(B, prec, synth.FULL, kind, spread, tile, split=0)
        if prec == "bf16" and binding.Model.tune_shape("attention", tile)["kind"] >= 1:
            for split in (1, 3):  # 2 and 8 key splits
                _attention_case(B, prec, synth.FULL, kind, spread, tile, split=split)


@pytest.mark.parametrize("cfg", [synth.FULL, synth.SMALL], ids=["dh32", "dh16"])
@pytest.mark.parametrize("kind,spread", [("random", 3.0), ("loose", 0.5), ("low", 0.3)],
                         ids=["sharp", "loose", "low"])
def test_attention_key_split_long_events(B, cfg, kind, spread):
    """Key splits over events of several LDS stages per split (2, 4 and 8 splits of 2000, 1500
    and 17 keys, the last event leaving most splits empty), on the default tile and the
    look-ahead tile, against the oracle."""
    for tile in (-1, 8):
        for split in (1, 2, 3):
            _attention_case(B, "bf16", cfg, kind, spread, tile, split=split, sizes=[2000, 1500, 17])
