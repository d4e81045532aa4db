"""GPU parity of the candidate construction (mlpf_candidates) against the oracle's ``candidates``:
bit-exact on the same per-row classes and kinematics (integer selection and copies), on synthetic
class maps and on a full forward pass, with empty, ragged, malformed and maximum-size batches."""
import numpy as np
import pytest

import synth
from oracle import mlpf_oracle as O
from parity_util import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2601_17554_amd import binding
    binding.load()
    return binding


def _run(B, row_start, n_valid, cls, kin, cap=None, total_rows=None, max_seqlen=8192):
    import torch
    rs = torch.as_tensor(np.asarray(row_start, dtype=np.int32)).cuda()
    nv = None if n_valid is None else torch.as_tensor(np.asarray(n_valid, dtype=np.int32)).cuda()
    T = int(len(cls)) if total_rows is None else total_rows
    batch = B.Batch(rs, nv, len(row_start) - 1, T, max_seqlen)
    c = torch.as_tensor(np.asarray(cls, dtype=np.int32)).cuda()
    k = None if kin is None else torch.as_tensor(np.asarray(kin, dtype=np.float32)).cuda()
    dev = B.candidates(batch, c, k, cap=cap)
    return B.candidates_to_host(dev)


def _compare(got, want, cap=None):
    offsets, rows, classes, kin = want
    np.testing.assert_array_equal(got["offsets"], offsets)
    n = len(rows) if cap is None else min(cap, len(rows))
    np.testing.assert_array_equal(got["rows"][:n], rows[:n])
    np.testing.assert_array_equal(got["cls"][:n], classes[:n])
    if kin is not None:
        np.testing.assert_array_equal(got["kin"][:n], kin[:n])


def _clamped(row_start, n_valid, T, max_seqlen):
    """The batch description as the library reads it (header rule: ranges clamped into [0, T],
    valid counts to the range and to max_seqlen)."""
    rs, nv = [], []
    for e in range(len(row_start) - 1):
        s = min(max(row_start[e], 0), T)
        en = min(max(row_start[e + 1], s), T)
        n = en - s if n_valid is None else min(max(n_valid[e], 0), en - s)
        rs.append(s)
        nv.append(min(n, max_seqlen))
    return rs, nv


def _oracle_clamped(row_start, n_valid, cls, kin, T, max_seqlen):
    rs, nv = _clamped(row_start, n_valid, T, max_seqlen)
    offsets, rows = [0], []
    for s, n in zip(rs, nv):
        rows += [s + i for i in range(n) if cls[s + i] != 0]
        offsets.append(len(rows))
    rows = np.asarray(rows, dtype=np.int64)
    return (np.asarray(offsets), rows, np.asarray(cls)[rows],
            None if kin is None else np.asarray(kin, dtype=np.float32)[rows])


@pytest.mark.parametrize("p_zero", [0.0, 0.5, 0.97, 1.0])
def test_candidates_random_ragged(B, p_zero):
    rng = np.random.default_rng(int(p_zero * 100) + 3)
    lens = rng.integers(0, 700, 40)
    lens[[3, 17]] = 0
    nval = np.array([rng.integers(0, l + 1) for l in lens])
    rs = np.concatenate([[0], np.cumsum(lens)])
    T = int(rs[-1])
    cls = np.where(rng.random(T) < p_zero, 0, rng.integers(1, 6, T)).astype(np.int32)
    kin = rng.standard_normal((T, 4)).astype(np.float32)
    got = _run(B, rs, nval, cls, kin)
    _compare(got, O.candidates(cls, kin, rs, nval))
    got = _run(B, rs, None, cls, None)
    _compare(got, O.candidates(cls, None, rs, None))


def test_candidates_edges(B):
    # no events
    got = _run(B, [0], None, np.zeros(5, np.int32), None)
    np.testing.assert_array_equal(got["offsets"], [0])
    # one event of the maximum size, every element a particle
    cls = np.full(8192, 4, np.int32)
    kin = np.arange(8192 * 4, dtype=np.float32).reshape(8192, 4)
    _compare(_run(B, [0, 8192], None, cls, kin), O.candidates(cls, kin, [0, 8192]))
    # more events than one scan round (3000), many empty
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 4, 3000)
    rs = np.concatenate([[0], np.cumsum(lens)])
    cls = rng.integers(0, 3, int(rs[-1])).astype(np.int32)
    _compare(_run(B, rs, None, cls, None), O.candidates(cls, None, rs))
    # a cap below the total: the first cap entries, offsets complete
    rs = [0, 300, 900, 1000]
    cls = np.ones(1000, np.int32)
    got = _run(B, rs, None, cls, None, cap=450)
    _compare(got, O.candidates(cls, None, rs), cap=450)
    assert got["total"] == 1000


def test_candidates_malformed_batch(B):
    """Offsets past the rows, decreasing offsets, negative and oversized valid counts and a
    max_seqlen below some counts are clamped as the header states (no access outside the buffers)."""
    rng = np.random.default_rng(8)
    T = 500
    cls = rng.integers(0, 6, T).astype(np.int32)
    kin = rng.standard_normal((T, 4)).astype(np.float32)
    row_start = [0, 120, 90, 300, 10_000, 10_000, 450]
    n_valid = [100, 50, -3, 9999, 4, 40]
    got = _run(B, row_start, n_valid, cls, kin, total_rows=T, max_seqlen=64)
    _compare(got, _oracle_clamped(row_start, n_valid, cls, kin, T, 64))


def test_candidates_from_forward(B):
    """The full model (BF16) with the Eq. 2 decode on a ragged batch with garbage padding, the
    classification bias of class 0 raised so that about half of the elements are "no particle"
    (the shift is taken from the oracle's logits). The library's candidate lists are checked
    against (1) the selection rule applied to the library's own per-row outputs (exact), and
    (2) the oracle's candidates from its FP64 forward pass: the same candidates except at
    near-tie elements, the same class, and kinematics within the BF16 tolerance."""
    from parity_util import TOL
    cfg = synth.FULL
    w = synth.make_weights(cfg, 30, sharpen=8.0)
    evs = [synth.make_event(7000 + i, n) for i, n in enumerate([150, 1, 0, 257, 90])]
    pk = synth.pack(evs, pad_to=64, pad_fill=1e4, seed=4)
    base = [O.forward(e.x, w, cfg)["logits"] for e in evs if e.n]
    lg = np.concatenate(base)
    w["heads.cls.b2"] = w["heads.cls.b2"].copy()
    w["heads.cls.b2"][0] += np.float32(np.median(lg[:, 1:].max(axis=1) - lg[:, 0]))
    m = B.Model(cfg, w, "bf16")
    out = run_gpu(m, pk, prim=True)
    got = _run(B, pk.row_start, pk.n_valid, out["cls"], out["decoded"])
    # (1) the rule on the library's own outputs
    valid = np.zeros(pk.total_rows, dtype=bool)
    for e in range(pk.n_events):
        r = pk.event_rows(e)
        valid[r.start:r.start + pk.n_valid[e]] = True
    sel = np.nonzero(valid & (out["cls"] != 0))[0]
    np.testing.assert_array_equal(got["rows"], sel)
    np.testing.assert_array_equal(got["cls"], out["cls"][sel])
    np.testing.assert_array_equal(got["kin"], out["decoded"][sel])
    # (2) against the oracle
    tol = TOL["bf16"]
    ref_rows, ref_cls, ref_kin, clear = [], [], [], []
    for e, ev in enumerate(evs):
        if ev.n == 0:
            continue
        ref = O.forward(ev.x, w, cfg)
        dec = O.decode(ref["reg"], ev.prim)
        kin = np.stack([dec["pt"], dec["eta"], dec["phi"], dec["e"]], axis=1)
        srt = np.sort(ref["logits"], axis=1)
        ok = srt[:, -1] - srt[:, -2] > 2 * tol * np.abs(ref["logits"]).max()
        r0 = pk.event_rows(e).start
        scale = np.abs(ref["reg"]).max()  # the angles' tolerance is relative to this (errors())
        for i in range(ev.n):
            clear.append(ok[i])
            if ref["cls"][i] != 0:
                ref_rows.append(r0 + i)
                ref_cls.append(ref["cls"][i])
                # phi = atan2(sin, cos): an error d in each of sin, cos moves phi by at most
                # sqrt(2) d / |(sin, cos)|
                ref_kin.append((kin[i], scale, np.hypot(ref["reg"][i, 2], ref["reg"][i, 3])))
    clear = np.asarray(clear)
    n_present = len(ref_rows)
    print(f"oracle: {n_present} candidates of {len(clear)} elements, {int((~clear).sum())} near-ties; "
          f"library: {len(sel)}")
    assert 0.2 * len(clear) < n_present < 0.8 * len(clear)
    live = np.concatenate([np.arange(pk.event_rows(e).start, pk.event_rows(e).start + pk.n_valid[e])
                           for e in range(pk.n_events)])
    clear_row = dict(zip(live.tolist(), clear.tolist()))
    got_set, ref_set = set(got["rows"].tolist()), set(ref_rows)
    differ = got_set ^ ref_set
    assert all(not clear_row[r] for r in differ), "a candidate differs away from a near-tie"
    ref_map = dict(zip(ref_rows, zip(ref_cls, ref_kin)))
    checked = 0
    for k, r in enumerate(got["rows"].tolist()):
        if r not in ref_map or not clear_row[r]:
            continue
        c, (kin, scale, hyp) = ref_map[r]
        assert got["cls"][k] == c
        g = got["kin"][k].astype(np.float64)
        assert abs(g[0] / kin[0] - 1) <= tol and abs(g[3] / kin[3] - 1) <= tol, (r, g, kin)
        assert abs(g[1] - kin[1]) <= tol * scale, (r, g, kin)
        dphi = (g[2] - kin[2] + np.pi) % (2 * np.pi) - np.pi
        assert abs(dphi) <= np.sqrt(2) * tol * scale / hyp, (r, g, kin, hyp)
        checked += 1
    assert checked > 50


def test_candidates_graph_capture(B):
    """mlpf_candidates captured in a HIP graph (through torch's graph API) and replayed after the
    classes are rewritten in place: every replay equals the oracle on the current classes."""
    import torch
    rng = np.random.default_rng(12)
    lens = rng.integers(0, 300, 20)
    rs = np.concatenate([[0], np.cumsum(lens)])
    T = int(rs[-1])
    batch = B.Batch.from_host(rs, None, max_seqlen=8192)
    cls = torch.zeros(T, dtype=torch.int32, device="cuda")
    kin = torch.as_tensor(rng.standard_normal((T, 4)).astype(np.float32)).cuda()
    out = {"offsets": torch.empty(len(rs), dtype=torch.int32, device="cuda"),
           "rows": torch.empty(T, dtype=torch.int32, device="cuda"),
           "cls": torch.empty(T, dtype=torch.int32, device="cuda"),
           "kin": torch.empty(T, 4, dtype=torch.float32, device="cuda")}
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        B.mlpf_candidates(batch, cls, kin, out["offsets"], out["rows"], out["cls"], out["kin"], T, s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            B.mlpf_candidates(batch, cls, kin, out["offsets"], out["rows"], out["cls"], out["kin"], T, s)
    for rep, p_zero in enumerate([0.5, 0.0, 0.9, 1.0]):
        c = np.where(rng.random(T) < p_zero, 0, rng.integers(1, 6, T)).astype(np.int32)
        cls.copy_(torch.as_tensor(c))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = B.candidates_to_host(out)
        _compare(got, O.candidates(c, kin.cpu().numpy(), rs))
