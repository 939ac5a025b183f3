"""Pins for the oracle's full-grid outlier output: on the sampled blocks it
must reproduce the loop's own S when thresholded against the previous
iterate (the S-update of equation 11 restricted to the blocks), it must
recover the planted outliers of an easy instance, and the strict threshold
of equation 10 decides ties."""
import numpy as np

import synth
from oracle import outliers, rtcur
from oracle.sampler import draw_sample


def test_exact_low_rank_has_no_outliers():
    inst = synth.tucker_plus_sparse((14, 12, 10), (2, 2, 2), alpha=0.0, seed=3)
    res = rtcur(inst.X, inst.ranks, (8, 8, 8), None, None, 0.7, 1e-12, 30, 0, "F")
    S, L = outliers(res, inst.X)
    assert np.max(np.abs(L - inst.L_star)) <= 1e-9 * np.max(np.abs(inst.L_star))
    # residual rounding stays below every threshold of the loop
    assert not np.any(S)


def test_recovers_planted_support_cube100():
    inst = synth.config_instance("cube100_r3")
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    res = rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    S, L = outliers(res, inst.X)
    truth = inst.S_star != 0
    found = S != 0
    zeta = res.zeta_hist[-1]
    resid = np.abs(L - inst.L_star).max()
    # L is recovered to well below the final threshold ...
    assert resid < 0.1 * zeta
    # ... so every clean entry stays below it (no false outliers) and every
    # planted value clear of the threshold band is found, with S = S* + (L* - L)
    assert not np.any(found & ~truth)
    clear = truth & (np.abs(inst.S_star) > zeta + resid)
    assert np.all(found[clear])
    assert np.all(np.abs(S[found] - inst.S_star[found]) <= resid)
    # only planted values inside the band |S*| <= zeta + resid may be missed
    assert np.all(np.abs(inst.S_star[truth & ~found]) <= zeta + resid)
    # S equals X - L exactly where kept
    assert np.array_equal(S[found], (inst.X - L)[found])


def test_strict_threshold_and_explicit_zeta():
    inst = synth.tucker_plus_sparse((10, 9, 8), (2, 2, 2), alpha=0.1, seed=5)
    res = rtcur(inst.X, inst.ranks, (6, 6, 6), None, None, 0.7, 0.0, 3, 0, "F")
    L = res.reconstruct()
    D = inst.X - L
    z = float(np.abs(D).flat[17])        # a tie: |D| == zeta is not an outlier
    S, _ = outliers(res, inst.X, z)
    assert S.flat[17] == 0.0
    assert np.array_equal(S != 0, np.abs(D) > z)
    # default threshold is the last one the loop used
    S2, _ = outliers(res, inst.X)
    assert np.array_equal(S2 != 0, np.abs(D) > res.zeta_hist[-1])


def test_matches_loop_support_on_sampled_core():
    # on the core block, HT_zeta_K(X - L^(K-1)) is the loop's S^K; the full
    # grid output uses L^K instead, so compare it with the oracle's own
    # block-level threshold of X - L^K
    inst = synth.tucker_plus_sparse((16, 14, 12), (2, 2, 2), alpha=0.15, seed=7)
    res = rtcur(inst.X, inst.ranks, (9, 9, 9), None, None, 0.7, 0.0, 5, 0, "F")
    S, L = outliers(res, inst.X)
    samp = res.sample
    core = np.ix_(*samp.I)
    assert np.allclose(L[core], res.LB[0], rtol=0, atol=1e-12 * np.abs(L).max())
    Dk = inst.X[core] - res.LB[0]
    assert np.array_equal(S[core] != 0, np.abs(Dk) > res.zeta_hist[-1])
