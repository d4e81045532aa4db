"""mlpf_reconstruct_events_noalloc (the entry point for callers that cannot allocate device
memory: its scratch is the library's fixed per-GPU array) against mlpf_reconstruct_events with a
caller workspace: the same kernels on the same inputs, so the same bits, on two calls in a row
(the second with a smaller batch, which reuses the scratch the first one left), plus the capacity
rejection of a batch whose workspace exceeds the scratch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _run_both(B, m, pk, prim):
    import torch
    x = torch.from_numpy(pk.x).cuda()
    batch = B.Batch.from_host(pk.row_start, pk.n_valid)
    p = torch.from_numpy(pk.prim).cuda() if prim else None
    ref = m.reconstruct(x, batch, prim=p)
    got = m.outputs(pk.total_rows, decode=prim)
    for v in got.values():
        v.fill_(-7)
    B.mlpf_reconstruct_events_noalloc(m, x, batch, got["logits"], got["reg"], got["cls"], p,
                                      got.get("decoded"))
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in got.items()}, {k: v.cpu().numpy() for k, v in ref.items()})


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_noalloc_matches_workspace_entry_point(prec):
    import torch
    from paper_2601_17554_amd import binding as B
    cfg = synth.FULL
    w = synth.make_weights(cfg, 3, sharpen=2.0, **synth.WIDE)
    m = B.Model(cfg, w, prec)
    big = synth.pack([synth.make_event(7100 + i, n) for i, n in enumerate([3000, 1, 777, 4100])],
                     pad_to=64, pad_fill=1e4, seed=21)
    small = synth.pack([synth.make_event(7200 + i, n) for i, n in enumerate([130, 65])])
    assert m.workspace_bytes(big.total_rows, big.n_events) <= 128 << 20
    for pk, prim in ((big, True), (small, False)):
        got, ref = _run_both(B, m, pk, prim)
        live = np.concatenate([np.arange(pk.event_rows(e).start, pk.event_rows(e).stop)
                               for e in range(pk.n_events)])
        for k in ref:
            np.testing.assert_array_equal(got[k][live], ref[k][live], err_msg=f"{prec} {k} rows {pk.total_rows}")
    # A batch whose workspace exceeds the 128 MiB scratch is refused before anything runs.
    n = 40000 if prec == "bf16" else 20000
    rs = np.array([0, n], np.int32)
    batch = B.Batch(torch.zeros(2, dtype=torch.int32, device="cuda"), None, 1, n, 8192,
                    row_start_host=None)
    assert m.workspace_bytes(n, 1) > 128 << 20
    out = m.outputs(1)
    with pytest.raises(B.MlpfError, match="CAPACITY"):
        B.mlpf_reconstruct_events_noalloc(m, torch.zeros(1, 17, device="cuda"), batch, out["logits"],
                                          out["reg"], out["cls"], None, None)
    del rs
