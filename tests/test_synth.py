"""The seeded input generators: reproducible, well-formed, with the workload's distributions."""
import numpy as np

import synth


def test_weights_reproducible_and_shaped():
    a, b = synth.make_weights(synth.SMALL, 3), synth.make_weights(synth.SMALL, 3)
    assert list(a) == [n for n, _ in synth.param_shapes(synth.SMALL)]
    for k in a:
        assert a[k].dtype == np.float32 and a[k].shape == dict(synth.param_shapes(synth.SMALL))[k]
        np.testing.assert_array_equal(a[k], b[k])
    assert abs(a["layers.0.W_1"].std() - 0.02) < 2e-3
    assert abs(a["layers.0.ln1.gamma"].mean() - 1.0) < 1e-2
    s = synth.make_weights(synth.SMALL, 3, sharpen=8.0)
    d = synth.SMALL.d_model
    np.testing.assert_array_equal(s["layers.0.W_qkv"][:, :2 * d], a["layers.0.W_qkv"][:, :2 * d] * 8)
    np.testing.assert_array_equal(s["layers.0.W_qkv"][:, 2 * d:], a["layers.0.W_qkv"][:, 2 * d:])


def test_features_one_hot():
    x = synth.make_features(np.random.default_rng(0), 500)
    assert x.shape == (500, 17) and x.dtype == np.float32
    np.testing.assert_array_equal(x[:, :6].sum(1), 1.0)
    assert set(np.unique(x[:, :6])) == {0.0, 1.0}
    assert abs(x[:, 6:].std() - 1) < 0.05


def test_event_counts_lognormal():
    evs = synth.event_set(200, 400, lo=500)
    n = np.array([e.n for e in evs])
    assert n.min() >= 500 and n.max() <= 8192
    assert 2700 < np.median(n) < 3300
    again = synth.event_set(200, 3, lo=500)
    np.testing.assert_array_equal(again[1].x, evs[1].x)


def test_pack_layout():
    evs = [synth.make_event(s, n) for s, n in ((1, 3), (2, 64), (3, 65), (4, 0))]
    pk = synth.pack(evs, pad_to=64, pad_fill=1e4)
    np.testing.assert_array_equal(pk.row_start, [0, 64, 128, 256, 256])
    np.testing.assert_array_equal(pk.n_valid, [3, 64, 65, 0])
    np.testing.assert_array_equal(pk.x[64:128], evs[1].x)
    assert np.abs(pk.x[3:64]).max() > 100  # garbage in padding rows
    assert pk.max_seqlen == 65
    un = synth.pack(evs)
    np.testing.assert_array_equal(un.row_start, [0, 3, 67, 132, 132])


def test_poisson_arrivals():
    t = synth.poisson_arrivals(1000.0, 20000, seed=1400)
    assert np.all(np.diff(t) > 0)
    assert abs(20000 / t[-1] - 1000) < 30
