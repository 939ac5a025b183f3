"""Pins for the oracle's L-update (Section 3.1) against results the
mathematics fixes: the Fiber CUR identity (Theorem 2.5), the full-sample case
(a truncated HOSVD projection, Remark on HOSVD), the two-mode case (matrix
CUR, Section 2.2) and the algebra of the truncated pseudo-inverse."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle.rtcur import evaluate, gather_blocks, l_update
from oracle.sampler import draw_sample
from oracle.tensor import mode_product, multi_mode_product, unfold


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # dims, ranks, I sizes, J sizes (None = chidori)
    ((20, 18, 16), (2, 3, 2), (6, 8, 6), None),
    ((20, 18, 16), (2, 3, 2), (6, 8, 6), (10, 12, 10)),
    ((8, 9, 7, 6), (2, 2, 2, 2), (4, 4, 4, 3), None),
    ((8, 9, 7, 6), (2, 2, 2, 2), (4, 4, 4, 3), (9, 9, 9, 9)),
    ((30, 25), (3, 3), (7, 6), None),
]


@pytest.mark.parametrize("dims,ranks,I,J", CASES)
def test_fiber_cur_identity_on_exact_low_rank(dims, ranks, I, J):
    # Theorem 2.5 (ii): A = R x_i (C_i U_i^+) when rank(U_i) = r_i
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=0.0, seed=11)
    Ls = inst.L_star
    s = draw_sample(4, 0, dims, I, J)
    f = l_update(gather_blocks(Ls, s), s, ranks)
    assert _rel(multi_mode_product(f.R, f.A), Ls) < 1e-10
    # the same factors evaluated on the sampled blocks give the blocks back
    for got, want in zip(evaluate(f, s), gather_blocks(Ls, s)):
        assert _rel(got, want) < 1e-10


def test_full_sample_is_truncated_hosvd_projection():
    rng = np.random.default_rng(7)
    dims, ranks = (7, 6, 5), (2, 3, 2)
    X = rng.standard_normal(dims)
    s = draw_sample(0, 0, dims, dims, None)          # every index, chidori
    f = l_update(gather_blocks(X, s), s, ranks)
    proj = []
    for i, r in enumerate(ranks):
        M = unfold(X, i)
        w, Q = np.linalg.eigh(M @ M.T)               # independent route
        W = Q[:, np.argsort(w)[::-1][:r]]
        proj.append(W @ W.T)
    want = multi_mode_product(X, proj)
    assert _rel(multi_mode_product(f.R, f.A), want) < 1e-12


def test_two_modes_reduce_to_matrix_cur():
    # n = 2: L = C U_r^+ R_rows with C = X(:, J), U = X(I, J), R_rows = X(I, :)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((30, 25))
    r = 3
    s = draw_sample(1, 0, X.shape, (7, 6), None)
    f = l_update(gather_blocks(X, s), s, (r, r))
    I, J = s.I[0], s.I[1]
    U = X[np.ix_(I, J)]
    Wf, sf, Vtf = scipy.linalg.svd(U, full_matrices=False, lapack_driver="gesvd")
    Ur = (Wf[:, :r] * sf[:r]) @ Vtf[:r]
    want = X[:, J] @ scipy.linalg.pinv(Ur, atol=0.5 * sf[r - 1]) @ X[I, :]
    assert _rel(multi_mode_product(f.R, f.A), want) < 1e-11


def test_core_form_equals_literal_form():
    # G = R x_i W_i^T, B_i = C_i V_i S_i^-1 give G x_i B_i = R x_i A_i
    inst = synth.tucker_plus_sparse((24, 20, 18), (3, 2, 3), alpha=0.2, seed=3)
    s = draw_sample(2, 0, inst.dims, (9, 8, 9), None)
    blocks = gather_blocks(inst.X, s)
    f = l_update(blocks, s, inst.ranks)
    G = multi_mode_product(f.R, [W.T for W in f.W])
    B = [blocks[1 + i] @ (f.V[i] / f.sig[i]) for i in range(3)]
    assert _rel(multi_mode_product(G, B), multi_mode_product(f.R, f.A)) < 1e-12


def test_sampled_rows_of_A_are_projectors():
    # A_i(I_i, :) = U_i U_i^+ = W_r W_r^T: symmetric, idempotent, trace r
    inst = synth.tucker_plus_sparse((24, 20, 18), (3, 2, 3), alpha=0.2, seed=5)
    s = draw_sample(6, 0, inst.dims, (9, 8, 9), (30, 40, 30))
    f = l_update(gather_blocks(inst.X, s), s, inst.ranks)
    for i, r in enumerate(inst.ranks):
        P = f.A[i][s.I[i], :]
        assert np.allclose(P, P.T, atol=1e-13)
        assert np.allclose(P @ P, P, atol=1e-13)
        assert abs(np.trace(P) - r) < 1e-12


def test_mode_product_with_identity_keeps_tensor():
    rng = np.random.default_rng(9)
    T = rng.standard_normal((4, 5, 6))
    assert np.array_equal(mode_product(T, np.eye(5), 1), T)
