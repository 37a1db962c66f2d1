"""Checkpoint files (host side): the gauge field, counter and random-generator state
survive a save / load round trip, and the restored generator continues the original
stream."""
import numpy as np

import synth
from paper_0710_0066_amd import checkpoint


def test_checkpoint_roundtrip(tmp_path):
    U = synth.gauge_field((4, 4, 2, 2), 0.5, 11)
    rng = np.random.default_rng(123)
    rng.standard_normal(17)                     # advance the stream
    path = tmp_path / "ck.npz"
    checkpoint.save(path, U, 5, rng, {"beta": 5.6})
    expected = rng.standard_normal(9)
    U2, n, rng2, extra = checkpoint.load(path)
    assert np.array_equal(U2, U) and U2.dtype == np.complex128
    assert n == 5 and extra == {"beta": 5.6}
    assert np.array_equal(rng2.standard_normal(9), expected)
    assert not (tmp_path / "ck.npz.tmp").exists()
