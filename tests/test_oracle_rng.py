"""Pins of the oracle's random-number stream (CPU only).

Philox4x32-10 is pinned by the published known-answer vectors; the mapping of
words to uniforms and the counter layout are checked against their stated
definitions and against distributional properties.
"""

import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kats():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            words = [int(x, 16) for x in line.split()]
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expected", _kats())
def test_philox_known_answers(orc, ctr, key, expected):
    out = orc.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expected


def test_uniform_lattice_and_range(orc):
    u1, u2 = orc.uniforms(seed=123, tag=orc.TAG_ALBEDO, unit=5, k0=0, n=100000)
    for u in (u1, u2):
        assert np.all(u >= 0.0) and np.all(u < 1.0)
        # every value is an exact multiple of 2^-24, so 1 - u is exact in FP32
        assert np.all(np.floor(u * 2.0 ** 24) == u * 2.0 ** 24)
        assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_counter_layout(orc):
    """Sample k of (seed, tag, unit) reads Philox block (k>>1, unit, tag, k>>33)
    under key (seed lo, seed hi): words 0,1 for even k, words 2,3 for odd k."""
    seed = 0x0123456789ABCDEF
    ks = [0, 1, 2, 3, 1000001, (1 << 33) + 7, (1 << 40) + 2]
    for k in ks:
        u1, u2 = orc.uniforms(seed, 3, 77, k, 1)
        pair = k >> 1
        w = orc.philox4x32_10([pair & 0xFFFFFFFF, 77, 3, pair >> 32],
                              [seed & 0xFFFFFFFF, seed >> 32])
        a, b = (w[0], w[1]) if k % 2 == 0 else (w[2], w[3])
        assert u1[0] == (int(a) >> 8) * 2.0 ** -24
        assert u2[0] == (int(b) >> 8) * 2.0 ** -24


def test_streams_are_distinct_and_offsettable(orc):
    a1, a2 = orc.uniforms(9, 3, 0, 0, 4096)
    b1, b2 = orc.uniforms(9, 3, 1, 0, 4096)
    c1, c2 = orc.uniforms(9, 2, 0, 0, 4096)
    assert not np.array_equal(a1, b1) and not np.array_equal(a1, c1)
    # a window of the stream equals the stream read from an offset
    d1, d2 = orc.uniforms(9, 3, 0, 1001, 100)
    assert np.array_equal(d1, a1[1001:1101]) and np.array_equal(d2, a2[1001:1101])
    # successive pairs are uncorrelated
    assert abs(np.corrcoef(a1, a2)[0, 1]) < 0.05
