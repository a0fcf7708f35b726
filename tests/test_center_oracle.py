"""Pins of the fluctuation oracle (Sec. 4.1) against the hand-worked example
and the properties that fix the operation: every block of S' sums to zero,
S - S' is constant across each block, S' is orthogonal to S - S' block by
block (an orthogonal projection), and centring twice changes nothing."""
import os

import numpy as np
import pytest

from oracle.center import block_means, fluctuations

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fluctuations_2x6.txt")


def _golden():
    rows = [list(map(float, ln.split())) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    return np.array(rows[:2]), np.array(rows[2:])


def test_hand_worked_example():
    S, expect = _golden()
    assert np.array_equal(fluctuations(S, 3), expect)


@pytest.mark.parametrize("m,nt,M", [(7, 5, 3), (33, 1, 4), (16, 12, 1)])
def test_block_properties(m, nt, M):
    rng = np.random.default_rng(m * 100 + nt)
    S = rng.standard_normal((m, nt * M)) + 3.0 * rng.standard_normal((m, 1))
    F = fluctuations(S, nt)
    D = S - F
    for k in range(M):
        blk = slice(k * nt, (k + 1) * nt)
        np.testing.assert_allclose(F[:, blk].sum(axis=1), 0.0, atol=1e-12)
        np.testing.assert_allclose(D[:, blk], np.repeat(D[:, blk][:, :1], nt, axis=1), atol=1e-13)
        np.testing.assert_allclose((F[:, blk] * D[:, blk]).sum(), 0.0, atol=1e-10)
    np.testing.assert_allclose(fluctuations(F, nt), F, atol=1e-13)
    np.testing.assert_allclose(block_means(S, nt)[:, 0], D[:, 0], atol=1e-13)


def test_one_column_blocks_vanish_and_bad_blocks_rejected():
    S = np.arange(12.0).reshape(3, 4)
    assert np.array_equal(fluctuations(S, 1), np.zeros_like(S))
    with pytest.raises(ValueError):
        fluctuations(S, 3)
    with pytest.raises(ValueError):
        fluctuations(S, 0)
