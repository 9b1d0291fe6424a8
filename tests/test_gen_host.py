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
