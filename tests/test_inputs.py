"""CPU checks of the seeded input generators (no device, no oracle arithmetic)."""
import numpy as np

from paper_1012_2273_amd import inputs


def test_splitmix64_published_first_output():
    # SplitMix64 from state 0: the first output is 0xE220A8397B1DCDAF
    z = inputs._splitmix64(np.array([0], dtype=np.uint64))
    assert int(z[0]) == 0xE220A8397B1DCDAF


def test_hashed_integers_addressable_and_deterministic():
    full = inputs.hashed_integers(np.arange(300), 257, salt=3)
    rows = np.array([299, 0, 17, 17, 150])
    cols = np.array([256, 0, 5])
    sub = inputs.hashed_integers(rows, cols, salt=3)
    assert np.array_equal(sub, full[rows][:, cols])
    assert np.array_equal(full, inputs.hashed_integers(np.arange(300), 257, salt=3))
    assert not np.array_equal(full, inputs.hashed_integers(np.arange(300), 257, salt=4))
    # rows far past 2^32 / 8 elements address distinct, valid entries
    far = inputs.hashed_integers([2 ** 31 + 5], 64, salt=3)
    assert far.shape == (1, 64) and not np.array_equal(far[0], full[5, :64])


def test_hashed_integers_range_and_spread():
    x = inputs.hashed_integers(np.arange(512), 512, salt=1)
    assert x.dtype == np.float64 and x.min() == -8 and x.max() == 8
    counts = np.bincount((x + 8).astype(np.int64).ravel(), minlength=17)
    assert counts.min() > 0.9 * x.size / 17 and counts.max() < 1.1 * x.size / 17
