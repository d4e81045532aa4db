"""The C ABI library on the CPU: it loads, exports every entry point its header declares, and
rejects bad configurations before touching a GPU."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2601_17554_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libmlpf.so is not built (run __graft_entry__.build())")
    return B, B.load()


def test_exports_every_declared_symbol():
    B, lib = _lib()
    header = open(os.path.join(ROOT, "include", "mlpf.h")).read()
    declared = set(re.findall(r"\b(mlpf_[a-z0-9_]+)\s*\(", header))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), f"{name} not exported"
    assert declared == set(B.exported_symbols())


def test_sizes_and_validation_without_gpu():
    B, lib = _lib()
    cfg = B.make_config(synth.FULL)
    assert lib.mlpf_weights_count(ctypes.byref(cfg)) == synth.param_count(synth.FULL)
    fp32 = lib.mlpf_weights_bytes(ctypes.byref(cfg), 0)
    bf16 = lib.mlpf_weights_bytes(ctypes.byref(cfg), 1)
    assert fp32 >= 4 * synth.param_count(synth.FULL) and bf16 < fp32
    import dataclasses
    act = B.make_config(dataclasses.replace(synth.FULL, activation="relu"))
    assert act.activation == 1
    act.activation = 7
    h0 = ctypes.c_void_p()
    st = lib.mlpf_model_create(ctypes.byref(act), 0, None, 0, None, None, 0, None, ctypes.byref(h0))
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG" and b"activation" in lib.mlpf_last_error()
    dec = B.make_config(dataclasses.replace(synth.FULL, decision="binary"))
    assert dec.decision == 1
    dec.decision = -2
    st = lib.mlpf_model_create(ctypes.byref(dec), 0, None, 0, None, None, 0, None, ctypes.byref(h0))
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG" and b"decision" in lib.mlpf_last_error()
    pt = B.make_config(dataclasses.replace(synth.FULL, embed_per_type=True))
    assert lib.mlpf_weights_count(ctypes.byref(pt)) == synth.param_count(dataclasses.replace(synth.FULL, embed_per_type=True))
    assert lib.mlpf_weights_count(ctypes.byref(pt)) > synth.param_count(synth.FULL)
    bad = B.make_config(synth.Config(d_model=96, n_heads=3))
    assert lib.mlpf_weights_bytes(ctypes.byref(bad), 0) == 0
    h = ctypes.c_void_p()
    st = lib.mlpf_model_create(ctypes.byref(bad), 0, None, 0, None, None, 0, None, ctypes.byref(h))
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_UNSUPPORTED"
    assert b"d_model" in lib.mlpf_last_error()
    st = lib.mlpf_model_create(ctypes.byref(cfg), 0, None, 0, None, None, 0, None, None)
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG"
    st = lib.mlpf_model_create(ctypes.byref(cfg), 0, None, 0, None, None, 0, None, ctypes.byref(h))
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG"  # host_weights NULL


def test_candidates_validation_without_gpu():
    """mlpf_candidates rejects bad arguments before anything is enqueued (fake non-NULL device
    addresses are never dereferenced on these paths)."""
    B, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    odd = ctypes.c_void_p(0x1008)

    def status(batch, cls, dec, offs, rows, clss, kin, cap):
        return lib.mlpf_status_string(lib.mlpf_candidates(batch, cls, dec, offs, rows, clss, kin, cap, None))

    good = B._Batch(fake, None, None, None, 2, 10, 10)
    neg = B._Batch(fake, None, None, None, -1, 10, 10)
    big = B._Batch(fake, None, None, None, 2, 10, 100_000)
    assert status(None, fake, None, fake, fake, fake, None, 4) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(neg), fake, None, fake, fake, fake, None, 4) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(big), fake, None, fake, fake, fake, None, 4) == b"MLPF_ERR_UNSUPPORTED"
    assert status(ctypes.byref(good), None, None, fake, fake, fake, None, 4) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(good), fake, None, None, fake, fake, None, 4) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(good), fake, None, fake, fake, fake, None, -1) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(good), fake, None, fake, None, fake, None, 4) == b"MLPF_ERR_INVALID_ARG"
    assert status(ctypes.byref(good), fake, None, fake, fake, fake, fake, 4) == b"MLPF_ERR_INVALID_ARG"
    assert b"decoded" in lib.mlpf_last_error()
    assert status(ctypes.byref(good), fake, odd, fake, fake, fake, fake, 4) == b"MLPF_ERR_INVALID_ARG"
    assert b"aligned" in lib.mlpf_last_error()


def _mirror_batch(B, row_start, n_valid, total_rows, max_seqlen, device_n_valid=True):
    """A batch whose device pointers are fake (never dereferenced on a rejected call) and whose
    host mirrors hold the given values."""
    rs = (ctypes.c_int32 * len(row_start))(*row_start)
    nv = None if n_valid is None else (ctypes.c_int32 * len(n_valid))(*n_valid)
    dev_nv = ctypes.c_void_p(0x2000) if (n_valid is not None and device_n_valid) else None
    b = B._Batch(ctypes.c_void_p(0x1000), dev_nv, ctypes.cast(rs, ctypes.c_void_p),
                 None if nv is None else ctypes.cast(nv, ctypes.c_void_p), len(row_start) - 1,
                 total_rows, max_seqlen)
    b._keep = (rs, nv)
    return b


@pytest.mark.parametrize("row_start,n_valid,total,maxlen,what", [
    ([0, 5, 3], None, 10, 10, b"decreases"),          # non-monotone row_start
    ([-1, 5], None, 10, 10, b"negative"),              # negative first offset
    ([0, 5, 12], None, 10, 10, b"total_rows"),         # last offset beyond total_rows
    ([0, 5, 9], [5, 6], 10, 10, b"outside"),           # n_valid > its span
    ([0, 5, 9], [5, -1], 10, 10, b"outside"),          # negative n_valid
    ([0, 5, 9], [5, 4], 10, 4, b"max_seqlen"),         # valid count above max_seqlen
    ([0, 8, 9], None, 10, 4, b"max_seqlen"),           # packed span above max_seqlen
])
def test_host_mirror_rejections_without_gpu(row_start, n_valid, total, maxlen, what):
    """With host mirrors of row_start / n_valid, a malformed batch is rejected with
    MLPF_ERR_INVALID_ARG before anything is enqueued (so no GPU is needed to see it)."""
    B, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    b = _mirror_batch(B, row_start, n_valid, total, maxlen)
    st = lib.mlpf_candidates(ctypes.byref(b), fake, None, fake, fake, fake, None, 4, None)
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG", lib.mlpf_last_error()
    assert what in lib.mlpf_last_error(), lib.mlpf_last_error()


def test_host_mirror_needs_n_valid_mirror_without_gpu():
    B, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    b = _mirror_batch(B, [0, 5, 9], [5, 4], 10, 10)
    b.n_valid_host = None
    st = lib.mlpf_candidates(ctypes.byref(b), fake, None, fake, fake, fake, None, 4, None)
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG"
    assert b"n_valid_host" in lib.mlpf_last_error()


def test_six_head_config_sizes_without_gpu():
    """The paper's six heads (separate binary and particle-type heads) add one d x d + d hidden
    layer and keep the 11 outputs: the master blob grows by exactly that."""
    import dataclasses
    B, lib = _lib()
    six = dataclasses.replace(synth.FULL, binary_head=True)
    c6, c5 = B.make_config(six), B.make_config(synth.FULL)
    assert c6.binary_head == 1
    d = synth.FULL.d_model
    n6, n5 = lib.mlpf_weights_count(ctypes.byref(c6)), lib.mlpf_weights_count(ctypes.byref(c5))
    assert n6 == synth.param_count(six) and n6 - n5 == d * d + d
    assert lib.mlpf_weights_bytes(ctypes.byref(c6), 1) > lib.mlpf_weights_bytes(ctypes.byref(c5), 1)
    c6.binary_head = 2
    h = ctypes.c_void_p()
    st = lib.mlpf_model_create(ctypes.byref(c6), 0, None, 0, None, None, 0, None, ctypes.byref(h))
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG" and b"binary_head" in lib.mlpf_last_error()
    # The paper's full network: ~5.1 M parameters in the paper (Sec. 5.3).
    print("PAPER_MODEL parameters:", synth.param_count(synth.PAPER_MODEL))


def test_workspace_bytes_rejects_bad_sizes_without_gpu():
    B, lib = _lib()
    assert lib.mlpf_workspace_bytes(None, 100, 100, 1) == 0


def test_no_cpu_fallback_when_library_missing(monkeypatch):
    from paper_2601_17554_amd import binding as B
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libmlpf.so")
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        B.load()


def _parts_batch(B, events, ev_valid, parts, part_valid, total, maxlen=100, parts_mirrors=True):
    b = _mirror_batch(B, events, ev_valid, total, maxlen)
    q = _mirror_batch(B, parts, part_valid, total, maxlen)
    if not parts_mirrors:
        q.row_start_host = None
        q.n_valid_host = None
    b.attn_parts = ctypes.pointer(q)
    b._keep = (b._keep, q)
    return b


@pytest.mark.parametrize("events,ev_valid,parts,part_valid,total,what", [
    ([0, 10, 20], [8, 10], [0, 4, 10, 15, 20], [3, 4, 5, 5], 20, b"does not continue"),  # gap
    ([0, 10, 20], [8, 10], [0, 10, 20], [8, 0], 20, b"in no attention partition"),  # event uncovered
    ([0, 10, 20], [10, 10], [0, 6, 14, 20], None, 20, b"does not continue"),        # crosses events
    ([0, 10, 20], [10, 10], [0, 5, 10, 15, 20], [5, 5, 5, 4], 20, b"no attention partition"),  # short
    ([0, 10, 20], [10, 10], [0, 5, 10, 15, 20], None, 24, b"span"),                  # row totals differ
    ([0, 10, 20], [10, 10], [0, 10, 5, 20], None, 20, b"decreases"),                 # bad layout
])
def test_attention_partition_rejections_without_gpu(events, ev_valid, parts, part_valid, total, what):
    """Attention partitions must tile every event's valid rows in order inside the event; with host
    mirrors the library checks it before anything is enqueued."""
    B, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    b = _parts_batch(B, events, ev_valid, parts, part_valid, 20)
    b.attn_parts.contents.total_rows = total
    st = lib.mlpf_candidates(ctypes.byref(b), fake, None, fake, fake, fake, None, 4, None)
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG", lib.mlpf_last_error()
    assert what in lib.mlpf_last_error(), lib.mlpf_last_error()


def test_attention_partitions_need_mirrors_without_gpu():
    B, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    b = _parts_batch(B, [0, 10], [10], [0, 5, 10], None, 10, parts_mirrors=False)
    st = lib.mlpf_candidates(ctypes.byref(b), fake, None, fake, fake, fake, None, 4, None)
    assert lib.mlpf_status_string(st) == b"MLPF_ERR_INVALID_ARG"
    assert b"mirrors" in lib.mlpf_last_error()


def test_partition_helper_tiles_events():
    """The host partitioner (cells of about `target` elements in (eta, phi)) returns a row
    permutation inside each event's valid rows and partitions that tile them."""
    import numpy as np
    from paper_2601_17554_amd import partition as P
    evs = [synth.make_event(60 + i, n) for i, n in enumerate([1300, 5, 0, 700, 1])]
    pk = synth.pack(evs, pad_to=64)
    perm, prs, pnv = P.partition_batch(pk.x, pk.row_start, pk.n_valid, target=256)
    assert sorted(perm.tolist()) == list(range(pk.total_rows))
    for e in range(pk.n_events):
        r = pk.event_rows(e)
        assert set(perm[r].tolist()) == set(range(r.start, r.stop))
    assert prs[-1] == pk.total_rows and (np.diff(prs) >= pnv).all() and (pnv > 0).all()
    assert pnv.sum() == pk.n_valid.sum() and pnv.max() <= 256


def test_attention_split_tiles_without_gpu():
    """The key-split op: four settings (1, 2, 4 and 8 splits), nothing beyond."""
    B, lib = _lib()
    assert B.Model.tune_count("attn_split") == 4
    assert [B.Model.tune_shape("attn_split", t)["splits"] for t in range(4)] == [1, 2, 4, 8]
    with pytest.raises(B.MlpfError, match="INVALID_ARG"):
        B.Model.tune_shape("attn_split", 4)
