"""Pins of the oracle's Gaussian test matrix (Sec. 3, Fig. rsvd (b1))."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle.philox import gaussian_matrix, philox4x64_10, raw_words


def test_kat_vectors(golden_dir):
    path = os.path.join(golden_dir, "philox4x64_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        w = [int(x, 16) for x in row]
        assert philox4x64_10(tuple(w[0:4]), tuple(w[4:6])) == tuple(w[6:10])


@pytest.mark.parametrize("key,ctr", [((5, 7), (1, 0, 0, 0)), ((123456789, 0), (41, 3, 2, 9)),
                                     ((2**64 - 1, 17), (2**40, 1, 0, 2**63))])
def test_matches_numpy_philox(key, ctr):
    # numpy's Philox (an independent implementation) emits the block of
    # counter+1 first; start it one block earlier to line the two up.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([ctr[0] - 1, *ctr[1:]], dtype=np.uint64))
    ref = [int(x) for x in bg.random_raw(4)]
    assert list(philox4x64_10(ctr, key)) == ref


def test_stream_blocks_match_numpy():
    # blocks 1..8 of stream (bond 0, stream 0, pair 0) = numpy's sequence from counter 0
    words = raw_words(9, bond=0, stream=0, pair=0, seed=99)
    bg = np.random.Philox(key=[99, 0], counter=[0, 0, 0, 0])
    ref = bg.random_raw(32)
    assert np.array_equal(words[4:], ref)


def test_gaussian_moments_and_ks():
    om = gaussian_matrix(200, 60, seed=3, pair=1, stream=2, bond=5).ravel()
    assert abs(om.mean()) < 0.05
    assert abs(om.var() - 1.0) < 0.05
    assert stats.kstest(om, "norm").pvalue > 1e-3
    # even and odd elements (cos and sin halves of Box-Muller) are each N(0, 1)
    assert stats.kstest(om[0::2], "norm").pvalue > 1e-3
    assert stats.kstest(om[1::2], "norm").pvalue > 1e-3
    # and uncorrelated
    assert abs(np.corrcoef(om[0::2], om[1::2])[0, 1]) < 0.05


def test_streams_are_distinct_and_deterministic():
    a = gaussian_matrix(16, 8, 0, 0, 0, 1)
    assert np.array_equal(a, gaussian_matrix(16, 8, 0, 0, 0, 1))
    for other in [(1, 0, 0, 1), (0, 1, 0, 1), (0, 0, 1, 1), (0, 0, 0, 2)]:
        b = gaussian_matrix(16, 8, *other)
        assert not np.allclose(a, b)


def test_element_layout_is_row_major():
    # the element (i, j) of an m x k matrix depends only on e = i*k + j
    a = gaussian_matrix(6, 4, 11, 0, 0, 3).ravel()
    b = gaussian_matrix(4, 6, 11, 0, 0, 3).ravel()
    assert np.array_equal(a, b)
