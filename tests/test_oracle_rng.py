"""Pins of the oracle's counter-based generator (Philox4x64-10, Salmon et
al. SC 2011) and of the word -> [0,1) conversion.

The generator is pinned against NumPy's own Philox4x64-10 bit generator, an
implementation independent of ours: NumPy increments the 256-bit counter
before each block, so counter c of ours is NumPy's state c - 1.
"""
import numpy as np
import pytest

import oracle

MASK = (1 << 64) - 1


def numpy_block(ctr, key):
    c = [int(x) for x in ctr]
    # numpy adds one (with carry) before generating: start from c - 1
    val = c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)
    val = (val - 1) % (1 << 256)
    cc = [(val >> (64 * i)) & MASK for i in range(4)]
    bg = np.random.Philox(counter=np.array(cc, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr", [(1, 0, 0, 0), (0, 0, 0, 0), (5, 7, 9, 11), (MASK, 3, 4, 5),
                                 (123456, 2**40 + 17, 8, 63), (0, MASK, MASK, 1)])
@pytest.mark.parametrize("key", [(0, 0), (123, 456), (MASK, MASK), (2**63 + 1, 0)])
def test_philox_matches_numpy(ctr, key):
    ours = oracle.philox4x64(ctr, key)
    ref = numpy_block(ctr, key)
    assert (ours == ref).all(), (ctr, key, ours, ref)


def test_philox_many_counters_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64)]
        ctr[0] += 1
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        assert (oracle.philox4x64(ctr, key) == numpy_block(ctr, key)).all()


def test_unif_range_and_exactness():
    # (w >> 8) * 2^-24: exact, in [0, 1 - 2^-24], never 1.0
    ws = np.array([0, 1, 255, 256, 2**31, 2**32 - 257, 2**32 - 256, 2**32 - 1], dtype=np.uint64)
    vals = [oracle.unif(int(w)) for w in ws]
    assert vals[0] == 0.0 and vals[1] == 0.0 and vals[2] == 0.0
    assert vals[3] == 2.0**-24
    assert vals[4] == 0.5
    assert vals[-1] == 1.0 - 2.0**-24
    assert vals[-2] == 1.0 - 2.0**-24
    assert vals[-3] == 1.0 - 2.0**-23
    # exhaustive over the 2^24 distinct outputs: float32 represents k * 2^-24 exactly
    k = np.arange(2**24, dtype=np.float64)
    f = (k.astype(np.float32) * np.float32(2.0**-24)).astype(np.float64)
    assert np.array_equal(f, k * 2.0**-24)
    assert f.max() < 1.0


def test_words_uniform_chi2_and_uncorrelated():
    # words of consecutive (pixel) counters: chi-square over 64 bins per word,
    # and no linear correlation between neighbouring counters
    n = 4096
    words = np.zeros((n, 8), np.uint64)
    for p in range(n):
        r = oracle.philox4x64((p, 0, 3, 0), (0, 0))
        for i in range(4):
            words[p, 2 * i] = int(r[i]) & 0xFFFFFFFF
            words[p, 2 * i + 1] = int(r[i]) >> 32
    u = (words >> np.uint64(8)).astype(np.float64) * 2.0**-24
    for j in range(8):
        h = np.bincount((u[:, j] * 64).astype(int), minlength=64)
        chi2 = ((h - n / 64) ** 2 / (n / 64)).sum()
        # 63 dof: mean 63, sd ~ 11.2; 6 sd bound
        assert chi2 < 63 + 6 * 11.3, (j, chi2)
    c = np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]
    assert abs(c) < 6.0 / np.sqrt(n)
    c2 = np.corrcoef(u[:, 0], u[:, 1])[0, 1]
    assert abs(c2) < 6.0 / np.sqrt(n)
