"""Pins of the sampled stopping rule (equation 14) on a case small enough to
work by hand, with non-full sampling, so that the per-block sum of n + 1
separate Frobenius norms is told apart from a pooled norm over all sampled
entries (and from other plausible slips: a missing block, a squared norm).

The case: a 3 x 3 matrix (n = 2), |I_1| = |I_2| = 2, rank (1, 1), chidori
sampling (J_1 = I_2, J_2 = I_1), zeta_0 = 1000 so that the first threshold
(700) keeps no entry in S.  Seed 5 draws I_1 = I_2 = {0, 1}, so with

        [ 3  0  a ]
    X = [ 0  1  b ] ,   a, b, c, d, f = 1, 2, 4, 3, 5
        [ c  d  f ]

the blocks are R = diag(3, 1), C_1 = X(:, {0,1}), C_2 = X^T(:, {0,1}).  The
rank-1 truncation of R keeps sigma = 3 with w = v = e_1, so both pseudo-
inverses are e_1 e_1^T / 3, and the Fiber CUR update (equation 8) is
L = (column 0 of X)(row 0 of X) / 3 = [[3, 0, a], [0, 0, 0], [c, 0, ac/3]].
Then C - L is [[0, 0], [0, 1]] on R, [[0, 0], [0, 1], [0, d]] on C_1 and
[[0, 0], [0, 1], [0, b]] on C_2, which gives e^(1) in closed form.
"""
import math

import numpy as np
import pytest

from oracle import draw_sample, rtcur

A, B, C, D, F = 1.0, 2.0, 4.0, 3.0, 5.0
X = np.array([[3.0, 0.0, A], [0.0, 1.0, B], [C, D, F]])
SEED = 5


def _hand_e1():
    num = 1.0 + math.sqrt(1.0 + D * D) + math.sqrt(1.0 + B * B)
    den = (math.sqrt(9.0 + 1.0) + math.sqrt(9.0 + 1.0 + C * C + D * D)
           + math.sqrt(9.0 + 1.0 + A * A + B * B))
    return num / den


def test_sample_is_the_worked_one():
    s = draw_sample(SEED, 0, (3, 3), (2, 2), None)
    assert list(s.I[0]) == [0, 1] and list(s.I[1]) == [0, 1]
    assert list(s.J_cols[0]) == [0, 1] and list(s.J_cols[1]) == [0, 1]


def test_first_update_matches_hand_computation():
    res = rtcur(X, (1, 1), (2, 2), None, 1000.0, 0.7, 0.0, 1, SEED, "F")
    assert res.iters == 1
    L = res.reconstruct()
    want = np.array([[3.0, 0.0, A], [0.0, 0.0, 0.0], [C, 0.0, A * C / 3.0]])
    assert np.allclose(L, want, rtol=0, atol=1e-14)
    assert not any(np.any(sb) for sb in res.SB)   # nothing above 700


def test_error_is_sum_of_block_norms():
    res = rtcur(X, (1, 1), (2, 2), None, 1000.0, 0.7, 0.0, 1, SEED, "F")
    e1 = res.err_hist[0]
    assert e1 == pytest.approx(_hand_e1(), rel=1e-14, abs=0)
    # the readings that equation 14 rules out give visibly different values
    pooled = math.sqrt(1 + (1 + D * D) + (1 + B * B)) / math.sqrt(
        10.0 + (10.0 + C * C + D * D) + (10.0 + A * A + B * B))
    squared = (1 + (1 + D * D) + (1 + B * B)) / (
        10.0 + (10.0 + C * C + D * D) + (10.0 + A * A + B * B))
    core_only = 1.0 / math.sqrt(10.0)
    for other in (pooled, squared, core_only):
        assert abs(other - e1) > 1e-2


def test_denominator_is_sum_of_block_norms():
    res = rtcur(X, (1, 1), (2, 2), None, 1000.0, 0.7, 0.0, 1, SEED, "F")
    want = math.sqrt(10.0) + math.sqrt(35.0) + math.sqrt(15.0)
    assert res.den == pytest.approx(want, rel=1e-15)
