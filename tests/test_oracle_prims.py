"""Pins for the oracle's tensor primitives against their Section 2.1
definitions written out as loops, and for the truncated pseudo-inverse
against an independent LAPACK driver."""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle.rtcur import E_RANK, OracleError, rank_rtol, truncated_pinv
from oracle.tensor import (fold, fro, hard_threshold, mode_product,
                           multi_mode_product, unfold)


def _brute_unfold(T, k):
    # column = C-order position over the remaining modes
    rest = [d for j, d in enumerate(T.shape) if j != k]
    M = np.zeros((T.shape[k], int(np.prod(rest))))
    for idx in itertools.product(*[range(d) for d in T.shape]):
        col = 0
        for j, d in enumerate(T.shape):
            if j != k:
                col = col * d + idx[j]
        M[idx[k], col] = T[idx]
    return M


def test_unfold_matches_definition_and_fold_inverts():
    rng = np.random.default_rng(1)
    T = rng.standard_normal((3, 4, 2, 5))
    for k in range(4):
        assert np.array_equal(unfold(T, k), _brute_unfold(T, k))
        assert np.array_equal(fold(unfold(T, k), k, T.shape), T)


def test_mode_product_matches_definition():
    rng = np.random.default_rng(2)
    T = rng.standard_normal((3, 4, 5))
    for k in range(3):
        A = rng.standard_normal((2, T.shape[k]))
        Y = mode_product(T, A, k)
        shape = list(T.shape)
        shape[k] = 2
        Z = np.zeros(shape)
        for idx in itertools.product(*[range(d) for d in shape]):
            acc = 0.0
            for s in range(T.shape[k]):
                src = list(idx)
                src[k] = s
                acc += T[tuple(src)] * A[idx[k], s]
            Z[idx] = acc
        assert np.allclose(Y, Z, rtol=1e-13, atol=1e-13)
        # matrix form of the definition: Y_(k) = A X_(k)
        assert np.allclose(unfold(Y, k), A @ unfold(T, k), rtol=1e-13, atol=1e-13)


def test_multi_mode_product_order_free():
    # mode products along different modes commute
    rng = np.random.default_rng(3)
    T = rng.standard_normal((3, 4, 5))
    A = [rng.standard_normal((6, d)) for d in T.shape]
    a = multi_mode_product(T, A)
    b = mode_product(mode_product(mode_product(T, A[2], 2), A[0], 0), A[1], 1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_hard_threshold_is_strict():
    D = np.array([-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 1.0000000000000002, 3.0])
    out = hard_threshold(D, 1.0)
    assert out.tolist() == [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0000000000000002, 3.0]


def test_fro_norm():
    A = np.array([[3.0, 4.0], [0.0, 12.0]])
    assert fro(A) == 13.0


def test_truncated_pinv_matches_independent_driver():
    rng = np.random.default_rng(4)
    for (s, m, r) in [(6, 40, 2), (12, 30, 3), (9, 9, 9)]:
        U = rng.standard_normal((s, m))
        W, sig, V, P = truncated_pinv(U, r)
        # rank-r truncation built from an independent LAPACK driver (gesvd)
        Wf, sf, Vtf = scipy.linalg.svd(U, full_matrices=False, lapack_driver="gesvd")
        Ur = (Wf[:, :r] * sf[:r]) @ Vtf[:r]
        Pref = scipy.linalg.pinv(Ur, atol=0.5 * sf[r - 1])
        assert np.allclose(P, Pref, rtol=1e-11, atol=1e-12)
        # Moore-Penrose conditions of the truncation
        assert np.allclose(Ur @ P @ Ur, Ur, atol=1e-11)
        assert np.allclose(P @ Ur @ P, P, atol=1e-11)


def test_truncated_pinv_rank_floor():
    rng = np.random.default_rng(5)
    U = rng.standard_normal((8, 2)) @ rng.standard_normal((2, 30))
    with pytest.raises(OracleError) as ei:
        truncated_pinv(U, 3)
    assert ei.value.status == E_RANK
    assert rank_rtol(86, 7396) == 7396 * 2.0 ** -52
    assert rank_rtol(300, 20) == 300 * 2.0 ** -52


@pytest.mark.parametrize("shape", [(8, 30), (30, 8), (12, 12)])
def test_truncated_pinv_rank_floor_is_sigma_ratio(shape):
    # sigma_r / sigma_1 just above max(s, m) eps is accepted, just below is
    # rejected: U = W diag(sig) V^T with exactly known singular values
    s, m = shape
    rng = np.random.default_rng(7)
    W, _ = np.linalg.qr(rng.standard_normal((s, 3)))
    V, _ = np.linalg.qr(rng.standard_normal((m, 3)))
    floor = max(s, m) * 2.0 ** -52
    ok = (W * np.array([1.0, 0.5, 1e3 * floor])) @ V.T
    Wr, sr, Vr, P = truncated_pinv(ok, 3)
    assert sr[2] / sr[0] == pytest.approx(1e3 * floor, rel=1e-2)
    bad = (W * np.array([1.0, 0.5, 0.0])) @ V.T   # sigma_3 at rounding level
    with pytest.raises(OracleError) as ei:
        truncated_pinv(bad, 3)
    assert ei.value.status == E_RANK
    # rank 2 is fine on the same matrix
    truncated_pinv(bad, 2)


def _bf16_grid(lo_exp, hi_exp):
    # every positive bfloat16 value 2^e * (1 + f/128), f = 0..127, written out
    vals = [2.0 ** e * (1.0 + f / 128.0) for e in range(lo_exp, hi_exp + 1)
            for f in range(128)]
    return np.array(sorted(vals))


def test_round_bf16_special_values():
    from oracle.tensor import round_bf16
    one = 1.0
    cases = {
        1.0: 1.0, 3.0: 3.0, -2.5: -2.5, 0.0: 0.0,
        one + 2.0 ** -8: 1.0,                           # tie: to the even significand
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,           # tie: 1+2^-7 is odd, round up
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # just above the tie
        one + 2.0 ** -8 - 2.0 ** -20: 1.0,              # just below the tie
        -(one + 3 * 2.0 ** -8): -(one + 2.0 ** -6),
        255.5: 256.0,                                   # significand carry
    }
    for x, want in cases.items():
        assert round_bf16(np.array([x]))[0] == want, x


def test_round_bf16_is_nearest_on_the_written_out_grid():
    # brute force: the nearest grid value (ties: the one with even f)
    from oracle.tensor import round_bf16
    grid = _bf16_grid(-6, 6)
    rng = np.random.default_rng(0)
    x = rng.uniform(2.0 ** -5, 60.0, 4000)
    got = round_bf16(x)
    for xi, gi in zip(x, got):
        d = np.abs(grid - xi)
        best = grid[d == d.min()]
        if len(best) == 1:
            assert gi == best[0]
        else:   # exact tie between two neighbours
            m = [b for b in best if int(round((b / 2.0 ** np.floor(np.log2(b)) - 1) * 128)) % 2 == 0]
            assert gi == m[0]
    assert np.array_equal(round_bf16(-x), -got)


def test_bf16_storage_emulation_switches_to_full_precision():
    # with the blocks held in bfloat16 until e^(k) <= 1e-2, the run ends at
    # the same tolerance as the full-precision one and its float64 phase
    # starts from unrounded X (the returned X blocks are the unrounded ones)
    import synth
    from oracle import rtcur
    inst = synth.tucker_plus_sparse((30, 28, 26), (2, 2, 2), alpha=0.1, seed=1)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    full = rtcur(inst.X, inst.ranks, I, tol=1e-6)
    low = rtcur(inst.X, inst.ranks, I, tol=1e-6, storage="bf16")
    assert low.status == 0 and low.err <= 1e-6
    for a, b in zip(low.XB, full.XB):
        assert np.array_equal(a, b)
    k1 = next(k for k, e in enumerate(low.err_hist) if e <= 1e-2)
    assert k1 + 1 < low.iters
    # both recover the same low-rank part (a separating instance)
    Ls = inst.L_star
    for r in (low, full):
        assert np.linalg.norm(r.reconstruct() - Ls) <= 1e-3 * np.linalg.norm(Ls)
    # stopping inside the bfloat16 phase: every C block is bfloat16-exact
    from oracle.tensor import round_bf16
    early = rtcur(inst.X, inst.ranks, I, tol=0.5, storage="bf16")
    for c in early.CB:
        assert np.array_equal(round_bf16(c), c)
