"""The seeded input sampler (no decoder arithmetic): its Philox4x32-10 equals
the published known-answer vectors, it draws each qubit's Pauli by the stated
cumulative thresholds, and a sample depends only on (seed, stream, uid, qubit)."""
import os

import numpy as np
from scipy import stats

from paper_2509_17837_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_sampler_philox_known_answers():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = I.philox4x32_10(tuple(np.uint32(x) for x in v[:4]), (v[4], v[5]))
        assert [int(o) for o in out] == v[6:]
        n += 1
    assert n == 3


def test_sampler_thresholds_and_frequencies():
    """Code of qubit q of sample uid = the cumulative-threshold rule applied
    to word 0 of Philox((seed, stream); (uid, q, 0x200, 0)); frequencies
    agree with the channel (chi-square)."""
    pxyz = I.channel(0.2, 10.0)
    e = I.sample_errors(300, 49, pxyz, 1234, stream=7, uid0=100)
    uid, q = np.meshgrid(np.arange(100, 400), np.arange(49), indexing="ij")
    u = I.philox4x32_10((uid, q, 0x200, 0), (1234, 7))[0].astype(np.int64)
    c1, c2, c3 = (int(np.floor(np.ldexp(v, 32))) for v in (pxyz[0], pxyz[0] + pxyz[1], sum(pxyz)))
    want = np.where(u < c1, I.CODE_X, np.where(u < c2, I.CODE_Y, np.where(u < c3, I.CODE_Z, I.CODE_I)))
    assert np.array_equal(e, want)
    big = I.sample_errors(4000, 121, pxyz, 99)
    counts = np.bincount(big.ravel(), minlength=4)
    exp = big.size * np.array([1 - sum(pxyz), pxyz[2], pxyz[0], pxyz[1]])   # I, Z, X, Y
    assert stats.chisquare(counts, exp).pvalue > 1e-4


def test_sampler_depends_only_on_uid():
    """A sample is the same drawn alone or inside a batch (uid offsets and
    chunking), and other seeds or streams give other samples."""
    pxyz = I.channel(0.15, 100.0)
    batch = I.sample_errors(20000, 121, pxyz, 5, uid0=0)     # spans several chunks
    for i in (0, 1, 8665, 19999):
        assert np.array_equal(I.sample_errors(1, 121, pxyz, 5, uid0=i)[0], batch[i])
    assert not np.array_equal(I.sample_errors(50, 121, pxyz, 6), batch[:50])
    assert not np.array_equal(I.sample_errors(50, 121, pxyz, 5, stream=1), batch[:50])
