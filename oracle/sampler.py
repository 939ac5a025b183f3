"""Oracle sampler: the index sets I_i and J_i of Algorithm 1 (sampling step).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this file; the
HIP library carries its own, independently written implementation of the
same published generator, and the two are compared bit for bit in tests.

Readings of the paper (its text only says the indices are sampled uniformly,
Algorithm 1 and Section 4 sizes rule):

* I_i is a uniformly random subset of [d_i] of size |I_i|, drawn without
  replacement and sorted ascending (I_i is a set in Theorem 2.5).
* J_i is either "chidori" (J_i is the product of the I_j, j != i, the layout
  the paper names in Section 2.2) or "fiber" (a uniformly random subset of
  the prod_{j!=i} d_j columns of the mode-i unfolding, sorted ascending).
* Columns of the mode-i unfolding are numbered in C order: the remaining
  modes in increasing order, the last one fastest.

Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014; public-domain reference code by
S. Vigna).  One stream per (seed, t, mode, which): starting from x = seed,
x <- mix(x) ; x <- mix(x ^ t) ; x <- mix(x ^ (2*mode + which)), where mix(x)
is the SplitMix64 output for state x.  Draws are then successive SplitMix64
outputs from state x.  A uniform integer in [0, N) is floor(u * N / 2^64)
(the high word of the 128-bit product, no rejection).  An m-subset of [0, N)
uses Floyd's algorithm (Bentley and Floyd, "Programming pearls: a sample of
brilliance", CACM 1987) and is then sorted.  t is the resample counter: 0 for
the initial draw, k for the draw that precedes iteration k+1 of RTCUR-R.
"""

from __future__ import annotations

from itertools import product
from typing import List, Optional, Sequence

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MIX_A = 0xBF58476D1CE4E5B9
MIX_B = 0x94D049BB133111EB


def splitmix64_step(state: int):
    """One SplitMix64 step: returns (next_state, output)."""
    state = (state + GOLDEN_GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * MIX_A) & MASK64
    z = ((z ^ (z >> 27)) * MIX_B) & MASK64
    return state, z ^ (z >> 31)


def _mix(x: int) -> int:
    return splitmix64_step(x & MASK64)[1]


class Stream:
    """Draw sequence for one (seed, t, mode, which) key."""

    def __init__(self, seed: int, t: int, mode: int, which: int):
        x = _mix(seed)
        x = _mix(x ^ (t & MASK64))
        x = _mix(x ^ ((2 * mode + which) & MASK64))
        self.state = x

    def next_u64(self) -> int:
        self.state, out = splitmix64_step(self.state)
        return out

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) as the high word of u * n."""
        return (self.next_u64() * n) >> 64


def floyd_subset(stream: Stream, m: int, N: int) -> List[int]:
    """Uniform m-subset of range(N) by Floyd's algorithm, sorted ascending."""
    if not (0 <= m <= N):
        raise ValueError(f"subset size {m} not in [0, {N}]")
    chosen = set()
    for j in range(N - m, N):
        t = stream.below(j + 1)
        chosen.add(j if t in chosen else t)
    return sorted(chosen)


def sample_I(seed: int, t: int, dims: Sequence[int],
             I_sizes: Sequence[int]) -> List[np.ndarray]:
    return [np.array(floyd_subset(Stream(seed, t, i, 0), int(s), int(d)),
                     dtype=np.int64)
            for i, (d, s) in enumerate(zip(dims, I_sizes))]


def other_modes(n: int, i: int) -> List[int]:
    return [j for j in range(n) if j != i]


def decode_columns(cols: np.ndarray, dims: Sequence[int], i: int) -> np.ndarray:
    """Mode-i unfolding column numbers -> index tuples (one row per column).

    Columns are numbered in C order over the remaining modes, last fastest.
    """
    rest = [dims[j] for j in other_modes(len(dims), i)]
    out = np.zeros((len(cols), len(rest)), dtype=np.int64)
    rem = np.array(cols, dtype=np.int64)
    for k in range(len(rest) - 1, -1, -1):
        out[:, k] = rem % rest[k]
        rem = rem // rest[k]
    return out


def encode_columns(tuples: np.ndarray, dims: Sequence[int], i: int) -> np.ndarray:
    rest = [dims[j] for j in other_modes(len(dims), i)]
    col = np.zeros(tuples.shape[0], dtype=np.int64)
    for k, dk in enumerate(rest):
        col = col * dk + tuples[:, k]
    return col


def chidori_tuples(I: Sequence[np.ndarray], i: int) -> np.ndarray:
    """Index tuples of J_i = product of I_j over j != i (last mode fastest)."""
    rest = [I[j] for j in other_modes(len(I), i)]
    return np.array(list(product(*[list(map(int, r)) for r in rest])),
                    dtype=np.int64).reshape(-1, len(rest))


class Sample:
    """One draw of the index sets: I[i] (sorted) and, per mode, the column
    tuples and unfolding column numbers of J_i."""

    def __init__(self, dims, I, J_tuples, chidori: bool):
        self.dims = tuple(int(d) for d in dims)
        self.I = I
        self.J_tuples = J_tuples
        self.J_cols = [encode_columns(J_tuples[i], self.dims, i)
                       for i in range(len(self.dims))]
        self.chidori = chidori


def draw_sample(seed: int, t: int, dims: Sequence[int],
                I_sizes: Sequence[int],
                J_sizes: Optional[Sequence[int]] = None) -> Sample:
    """The index sets for resample counter t.  J_sizes None -> chidori."""
    n = len(dims)
    I = sample_I(seed, t, dims, I_sizes)
    if J_sizes is None:
        J = [chidori_tuples(I, i) for i in range(n)]
        return Sample(dims, I, J, True)
    J = []
    for i in range(n):
        P = 1
        for j in other_modes(n, i):
            P *= int(dims[j])
        cols = floyd_subset(Stream(seed, t, i, 1), int(J_sizes[i]), P)
        J.append(decode_columns(np.array(cols, dtype=np.int64), dims, i))
    return Sample(dims, I, J, False)
