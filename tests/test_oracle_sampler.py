"""Pins for the oracle sampler (Algorithm 1 sampling step; readings in the
sampler module docstring)."""
import itertools
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle.sampler import (Stream, chidori_tuples, decode_columns, draw_sample,
                            encode_columns, floyd_subset, splitmix64_step)
from oracle.rtcur import gather_blocks
from oracle.tensor import unfold

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_sequences():
    # published reference outputs of SplitMix64 (tests/golden/splitmix64.txt)
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for row in rows:
        state = int(row[0])
        for want in row[1:]:
            state, out = splitmix64_step(state)
            assert out == int(want)


@pytest.mark.parametrize("N,m", [(1, 1), (5, 0), (5, 5), (10, 3), (300, 86),
                                 (1000, 999), (90000, 172)])
def test_floyd_subset_is_sorted_unique_in_range(N, m):
    for seed in range(5):
        S = floyd_subset(Stream(seed, 0, 0, 0), m, N)
        assert len(S) == m
        assert S == sorted(set(S))
        assert all(0 <= x < N for x in S)


def test_floyd_subset_uniform_over_subsets():
    # every 3-subset of range(6) equally likely (chi-square, 20 cells)
    counts = {c: 0 for c in itertools.combinations(range(6), 3)}
    trials = 20000
    for seed in range(trials):
        counts[tuple(floyd_subset(Stream(seed, 5, 1, 0), 3, 6))] += 1
    p = stats.chisquare(list(counts.values())).pvalue
    assert p > 1e-4


def test_uniform_below_is_uniform():
    st = Stream(99, 0, 0, 0)
    draws = [st.below(7) for _ in range(70000)]
    counts = np.bincount(draws, minlength=7)
    assert counts.size == 7
    assert stats.chisquare(counts).pvalue > 1e-4


def test_streams_differ_by_key():
    base = [Stream(1, 0, 0, 0).next_u64() for _ in range(1)]
    for key in [(2, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1)]:
        assert Stream(*key).next_u64() != base[0]


def test_decode_matches_c_order_unravel():
    dims = (4, 5, 6, 7)
    for i in range(4):
        rest = tuple(d for j, d in enumerate(dims) if j != i)
        cols = np.arange(int(np.prod(rest)))
        tup = decode_columns(cols, dims, i)
        want = np.stack(np.unravel_index(cols, rest), axis=1)
        assert np.array_equal(tup, want)
        assert np.array_equal(encode_columns(tup, dims, i), cols)


def test_chidori_columns_are_unfolding_columns():
    # chidori: J_i = product of the I_j; then C_i(I_i, :) is the mode-i
    # unfolding of the core subtensor R, entry for entry.
    rng = np.random.default_rng(0)
    dims = (9, 8, 7, 6)
    X = rng.standard_normal(dims)
    s = draw_sample(3, 0, dims, [4, 3, 5, 2])
    blocks = gather_blocks(X, s)
    R = blocks[0]
    for i in range(4):
        C = blocks[1 + i]
        assert np.array_equal(C[s.I[i], :], unfold(R, i))
        # columns: every chidori tuple addresses X directly
        for c in [0, C.shape[1] // 2, C.shape[1] - 1]:
            idx = list(s.J_tuples[i][c])
            idx.insert(i, slice(None))
            assert np.array_equal(C[:, c], X[tuple(idx)])


def test_chidori_tuples_order_last_fastest():
    I = [np.array([1, 4]), np.array([0, 2, 3]), np.array([5, 6])]
    t = chidori_tuples(I, 1)
    assert t.tolist() == [[1, 5], [1, 6], [4, 5], [4, 6]]


def test_fiber_columns_sorted_and_decoded():
    dims = (10, 11, 12)
    s = draw_sample(5, 2, dims, [3, 3, 3], [20, 25, 30])
    X = np.arange(np.prod(dims), dtype=float).reshape(dims)
    blocks = gather_blocks(X, s)
    for i in range(3):
        cols = s.J_cols[i]
        assert np.all(np.diff(cols) > 0)
        C = blocks[1 + i]
        for c in range(0, len(cols), 7):
            idx = list(s.J_tuples[i][c])
            idx.insert(i, slice(None))
            assert np.array_equal(C[:, c], X[tuple(idx)])


def test_kat_file_matches_oracle():
    with open(os.path.join(GOLDEN, "sampler_kat.json")) as f:
        cases = json.load(f)
    for c in cases:
        s = draw_sample(c["seed"], c["t"], c["dims"], c["I_sizes"], c["J_sizes"])
        assert [list(map(int, x)) for x in s.I] == c["I"]
        if c["J_sizes"] is not None:
            assert [list(map(int, x)) for x in s.J_cols] == c["J_cols"]
