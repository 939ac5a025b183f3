"""Pins for the oracle's whole loop (Algorithm 1): a separately written
brute-force alternating projection on tiny tensors, the threshold schedule
(equation 12), the hard-threshold support (equations 10, 11, 13), the stopping
rule (equation 14), the recovery criterion of the phase-transition study, and
the error paths."""
import math

import numpy as np
import pytest

import synth
from oracle.rtcur import (E_INVAL, E_NONFINITE, E_RANK, NOT_CONVERGED, OK,
                          OracleError, gather_blocks, rtcur)
from oracle.tensor import fro


def _brute_ap(X, ranks, zeta0, gamma, K):
    """Full-tensor HT + truncated-HOSVD alternating projections, written
    directly from the definitions with eigh of the unfolding Grams."""
    n = X.ndim
    L = np.zeros_like(X)
    zeta = zeta0
    errs, Ls = [], []
    for _ in range(K):
        zeta = gamma * zeta
        D = X - L
        S = np.where(np.abs(D) > zeta, D, 0.0)
        C = X - S
        P = C
        for i in range(n):
            M = np.moveaxis(C, i, 0).reshape(C.shape[i], -1)
            w, Q = np.linalg.eigh(M @ M.T)
            W = Q[:, np.argsort(w)[::-1][:ranks[i]]]
            P = np.moveaxis(np.tensordot(W @ W.T, P, axes=(1, i)), 0, i)
        L = P
        errs.append(np.linalg.norm(C - L) / np.linalg.norm(X))
        Ls.append(L)
    return errs, Ls


@pytest.mark.parametrize("variant", ["F", "R"])
def test_full_sample_matches_brute_force_alternating_projections(variant):
    inst = synth.tucker_plus_sparse((7, 6, 8), (2, 2, 2), alpha=0.1, seed=2)
    X = inst.X
    z0 = float(np.max(np.abs(X)))
    K = 12
    res = rtcur(X, (2, 2, 2), X.shape, None, z0, 0.7, 0.0, K, 0, variant)
    errs, Ls = _brute_ap(X, (2, 2, 2), z0, 0.7, K)
    assert res.iters == K
    for a, b in zip(res.err_hist, errs):
        assert abs(a - b) <= 1e-10 * b + 1e-14
    L = res.reconstruct()
    assert np.linalg.norm(L - Ls[-1]) / np.linalg.norm(Ls[-1]) < 1e-10


def test_full_sample_F_equals_R():
    inst = synth.tucker_plus_sparse((9, 8, 7), (2, 2, 2), alpha=0.2, seed=4)
    a = rtcur(inst.X, inst.ranks, inst.dims, None, None, 0.7, 0.0, 8, 3, "F")
    b = rtcur(inst.X, inst.ranks, inst.dims, None, None, 0.7, 0.0, 8, 3, "R")
    assert a.err_hist == b.err_hist
    assert np.array_equal(a.reconstruct(), b.reconstruct())


@pytest.fixture(scope="module")
def cube100():
    inst = synth.config_instance("cube100_r3")
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    return inst, I


def test_threshold_schedule(cube100):
    inst, I = cube100
    res = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 6, 0, "F")
    assert res.zeta0 == float(np.max(np.abs(inst.X)))
    z = res.zeta0
    for got in res.zeta_hist:
        z = 0.7 * z                      # repeated float64 multiplication
        assert got == z
    assert all(b < a for a, b in zip(res.zeta_hist, res.zeta_hist[1:]))


@pytest.mark.parametrize("variant", ["F", "R"])
def test_support_is_strict_threshold_of_previous_residual(cube100, variant):
    inst, I = cube100
    k = 10
    prev = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, k - 1, 0, variant)
    cur = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, k, 0, variant)
    zeta = cur.zeta_hist[-1]
    from oracle.rtcur import evaluate
    LB_prev = evaluate(prev.factors, cur.sample)   # L^(k-1) on this sample
    for b in range(4):
        D = cur.XB[b] - LB_prev[b]
        sup = cur.support[b]
        assert np.all(np.abs(D[sup]) > zeta)
        assert np.all(np.abs(D[~sup]) <= zeta)
        assert np.array_equal(cur.SB[b][sup], D[sup])
        assert np.array_equal(cur.CB[b], cur.XB[b] - cur.SB[b])
    # stopping rule terms: denominator is the sum of block norms of X
    assert cur.den == sum(fro(x) for x in cur.XB)
    e = sum(fro(c - l) for c, l in zip(cur.CB, cur.LB)) / cur.den
    assert e == cur.err_hist[-1]


def test_recovery_criterion_cube100(cube100):
    # success criterion of the phase-transition study: relative error <= 1e-3
    inst, I = cube100
    res = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    assert res.status == OK and res.err <= 1e-5
    L = res.reconstruct()
    assert np.linalg.norm(L - inst.L_star) / np.linalg.norm(inst.L_star) < 1e-3


def test_exact_low_rank_converges_in_one_step():
    inst = synth.tucker_plus_sparse((20, 18, 16), (2, 2, 2), alpha=0.0, seed=1)
    res = rtcur(inst.X, inst.ranks, (8, 8, 8), None, 1e30, 0.7, 1e-12, 5, 0, "F")
    assert res.iters == 1 and res.err < 1e-13


def test_tol_one_returns_before_iterating():
    inst = synth.tucker_plus_sparse((10, 10, 10), (2, 2, 2), alpha=0.1, seed=1)
    res = rtcur(inst.X, inst.ranks, (6, 6, 6), None, None, 0.7, 1.0, 5, 0, "F")
    assert res.iters == 0 and res.status == OK


def test_not_converged_status():
    inst = synth.tucker_plus_sparse((20, 20, 20), (2, 2, 2), alpha=0.6, seed=1)
    res = rtcur(inst.X, inst.ranks, (12, 12, 12), None, None, 0.7, 1e-12, 3, 0, "F")
    assert res.iters == 3 and res.status == NOT_CONVERGED


def test_zero_tensor_returns_zero():
    X = np.zeros((6, 7, 8))
    res = rtcur(X, (1, 1, 1), (3, 3, 3), None, 1.0, 0.7, 1e-5, 10, 0, "F")
    assert res.status == OK and res.iters == 0
    assert not np.any(res.reconstruct())


def test_rank_deficient_raises():
    inst = synth.tucker_plus_sparse((12, 12, 12), (1, 1, 1), alpha=0.0, seed=1)
    with pytest.raises(OracleError) as ei:
        rtcur(inst.X, (2, 2, 2), (6, 6, 6), None, None, 0.7, 1e-5, 5, 0, "F")
    assert ei.value.status == E_RANK


def test_nonfinite_raises():
    X = np.ones((6, 6, 6))
    X[1, 2, 3] = np.nan
    with pytest.raises(OracleError) as ei:
        rtcur(X, (1, 1, 1), (6, 6, 6), None, None, 0.7, 1e-5, 5, 0, "F")
    assert ei.value.status == E_NONFINITE


@pytest.mark.parametrize("kw", [
    dict(ranks=(3, 1, 1), I=(2, 2, 2)),           # r > |I|
    dict(ranks=(1, 1, 1), I=(7, 2, 2)),           # |I| > d
    dict(gamma=1.0), dict(gamma=0.0), dict(tol=-1.0), dict(max_iter=0),
    dict(J=(100, 2, 2)),                          # |J| > prod of other dims
])
def test_invalid_arguments(kw):
    X = np.ones((6, 6, 6))
    args = dict(ranks=(1, 1, 1), I=(3, 3, 3), J=None, gamma=0.7, tol=1e-5,
                max_iter=5)
    args.update(kw)
    with pytest.raises(OracleError) as ei:
        rtcur(X, args["ranks"], args["I"], args["J"], None, args["gamma"],
              args["tol"], args["max_iter"], 0, "F")
    assert ei.value.status == E_INVAL


def test_resample_counter_of_final_iterate(cube100):
    # RTCUR-R: iteration 1 uses the t = 0 draw, iteration k+1 the t = k draw,
    # so the final iterate of a K-iteration run lives on the t = K-1 sample.
    from oracle.sampler import draw_sample
    inst, I = cube100
    for K in (1, 2, 3):
        res = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, K, 5, "R")
        want = draw_sample(5, K - 1, inst.dims, I, None)
        assert all(np.array_equal(a, b) for a, b in zip(res.sample.I, want.I))
        blocks = gather_blocks(inst.X.astype(np.float64), want)
        assert all(np.array_equal(a, b) for a, b in zip(res.XB, blocks))


def test_threshold_schedule_multipliers():
    # a schedule of multipliers c_k of zeta_0 replaces the first thresholds;
    # c_k = gamma^k reproduces equation 12 (up to the rounding of gamma^k),
    # and beyond the schedule the decay continues from its last value
    import math

    import synth
    from oracle import rtcur
    inst = synth.tucker_plus_sparse((20, 18, 16), (2, 2, 2), alpha=0.1, seed=2)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    base = rtcur(inst.X, inst.ranks, I, tol=0.0, max_iter=6)
    geo = rtcur(inst.X, inst.ranks, I, tol=0.0, max_iter=6,
                schedule=[0.7 ** (k + 1) for k in range(3)])
    for a, b in zip(base.zeta_hist, geo.zeta_hist):
        assert math.isclose(a, b, rel_tol=1e-14)
    c = [0.5, 0.3, 0.2]
    res = rtcur(inst.X, inst.ranks, I, tol=0.0, max_iter=6, schedule=c)
    z0 = res.zeta0
    assert res.zeta_hist[:3] == [z0 * 0.5, z0 * 0.3, z0 * 0.2]
    z = z0 * 0.2
    for k in range(3, 6):
        z *= 0.7
        assert res.zeta_hist[k] == z
