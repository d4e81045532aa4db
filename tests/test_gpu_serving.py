"""Serving on the GPU: events arriving as a Poisson stream are batched continuously over several
slots; each event's result is the same as when it is run alone (bitwise here; the requirement is
the BF16 tolerance), and the HBM budget bounds the slots."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_serving_alone_vs_mix():
    import torch
    from paper_2601_17554_amd import binding as B
    from paper_2601_17554_amd import serve

    cfg = synth.FULL
    m = B.Model(cfg, synth.make_weights(cfg, 1), "bf16")
    ex = serve.GpuExecutor(m, max_rows=16384, max_events=16, slots=3, buckets=3, decode=True)
    srv = serve.Server(ex)
    rng = np.random.default_rng(9)
    evs = [synth.make_event(700 + i, int(rng.integers(50, 1500))) for i in range(30)]
    arrivals = synth.poisson_arrivals(800.0, len(evs), seed=1200)
    serve.run_poisson(srv, [e.x for e in evs], arrivals - arrivals[0], prims=[e.prim for e in evs])
    srv.close()
    assert srv.stats["events"] == len(evs)
    assert srv.stats["batches"] < len(evs)          # some events shared a batch
    futs = {id(r.x): r.future.result() for r in srv.completed}
    bitwise = 0
    for e in evs:
        pk = synth.pack([e])
        alone = m.reconstruct(torch.from_numpy(pk.x).cuda(), B.Batch.from_host(pk.row_start, pk.n_valid),
                              prim=torch.from_numpy(pk.prim).cuda())
        torch.cuda.synchronize()
        got = next(r.future.result() for r in srv.completed if r.x.shape == e.x.shape and np.array_equal(r.x, e.x))
        for k in ("logits", "reg", "decoded"):
            ref = alone[k].cpu().numpy()
            scale = max(np.abs(ref).max(), 1e-6)
            assert np.abs(got[k] - ref).max() <= 2e-2 * scale
        bitwise += int(np.array_equal(got["logits"], alone["logits"].cpu().numpy()))
    lat = srv.latencies_ms()
    print(f"served {len(evs)} events in {srv.stats['batches']} batches, max slots in flight "
          f"{srv.stats['max_inflight_slots']}, p50 {np.percentile(lat, 50):.2f} ms, "
          f"p99 {np.percentile(lat, 99):.2f} ms, bitwise equal to alone: {bitwise}/{len(evs)}")


def test_budget_bounds_slots():
    from paper_2601_17554_amd import binding as B
    from paper_2601_17554_amd import serve
    cfg = synth.SMALL
    m = B.Model(cfg, synth.make_weights(cfg, 0), "bf16")
    one = serve.GpuExecutor(m, max_rows=4096, max_events=8, slots=4, buckets=1)
    budget = int(one.slot_bytes * 2.5)
    ex = serve.GpuExecutor(m, max_rows=4096, max_events=8, slots=4, hbm_budget=budget, buckets=1)
    assert ex.slots() == 2 and ex.slots() * ex.slot_bytes <= budget
