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
