"""Host checks of the input generators: the numpy streams and kept-column
choice equal the torch ones bit for bit (the device feature kernel is checked
against them on the GPU)."""
import numpy as np

from paper_2512_12036_amd import gen


def test_numpy_streams_match_torch():
    for seed in (0, 1, 77, 4095, 123456):
        for tag in (1, 3, 4):
            s = gen._stream_np(seed, tag, 1000)
            t = gen._stream(seed, tag, 1000, "cpu").numpy()
            assert np.array_equal(s, t)


def test_kept_columns_match_reference_generator():
    for seed in range(0, 4096, 257):
        n, f, nk = gen.gnn_features_shape(seed, n=20)
        x = gen.gnn_features_t(seed, "cpu", n=n)
        assert np.array_equal(gen.gnn_kept_columns(seed, f, nk), x.col[:nk].numpy())



def test_feature_values_from_the_stream():
    """X's values, restated from the stream definition with numpy: entry e
    (row-major over the n x nk block) is (bits 63..40 of hash e of stream 4,
    plus one) / 2^24, and the row pointers step by nk."""
    for seed, n in ((5, 7), (77, 20), (4095, 33)):
        _, f, nk = gen.gnn_features_shape(seed, n=n)
        x = gen.gnn_features_t(seed, "cpu", n=n)
        h = gen._stream_np(seed, 4, n * nk).view(np.uint64)
        k = (h >> np.uint64(40)) + np.uint64(1)
        want = (k.astype(np.float64) / float(1 << 24)).astype(np.float32)
        assert np.array_equal(x.val.numpy(), want)
        assert x.val.numpy().min() > 0 and x.val.numpy().max() <= 1
        assert np.array_equal(x.rpt.numpy(), np.arange(n + 1) * nk)
