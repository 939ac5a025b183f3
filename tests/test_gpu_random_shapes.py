"""GPU parity on seeded random problem shapes: 2 to 4 modes, uneven sizes
and ranks, chidori and fibre sampling, RTCUR-F and RTCUR-R, float64 and
float32 blocks, each against the FP64 oracle for a fixed number of
iterations (tol = 0), at the same bars as the named workloads."""
import math

import numpy as np
import pytest

import synth
from oracle import E_INVAL, E_RANK, OracleError
from oracle import rtcur as oracle_rtcur

from _parity import compare, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


EPS = 2.0 ** -52


def _multilinear(ranks):
    """The largest ranks <= the drawn ones that a tensor can have as its
    multilinear rank: r_i <= prod_{j != i} r_j for every i (the mode-i
    unfolding of a Tucker tensor has rank at most the product of the other
    ranks; with n = 2 both ranks are the matrix rank).  Drawn ranks beyond
    that ask for more rank than the low-rank part has."""
    r = list(ranks)
    changed = True
    while changed:
        changed = False
        for i in range(len(r)):
            p = int(np.prod([r[j] for j in range(len(r)) if j != i]))
            if r[i] > p:
                r[i], changed = p, True
    return r


def _in_rank_band(res, ranks, I):
    """The library reported E_RANK where the oracle, whose floor is
    max(|I_i|, |J_i|) eps (its SVD's own accuracy), did not: allowed only when
    some U_i the oracle met had sigma_r / sigma_1 below the library's floor,
    at most sqrt(64 r_i |I_i| eps) (its Gram resolves the square of that
    ratio)."""
    band = max(math.sqrt(64.0 * r * s * EPS) for r, s in zip(ranks, I))
    return res.min_sig_ratio <= band


def _slice_limit(n):
    """Entries of one sampled core slice, r_{n-1} prod_{0<l<n-1} |I_l|, that
    the library accepts."""
    return 4096 if n == 3 else 2048


def _case(k):
    rng = np.random.default_rng(1000 + k)
    n = int(rng.integers(2, 5))
    dims = [int(rng.integers(6, 40 if n == 4 else 90)) for _ in range(n)]
    ranks = _multilinear([int(rng.integers(1, min(6, d) + 1)) for d in dims])
    # sample sizes between r_i and d_i; the core slice stays within its limit
    I = [int(rng.integers(r, d + 1)) for r, d in zip(ranks, dims)]
    fiber = bool(rng.integers(0, 2)) and n >= 3
    J = None
    if fiber:
        J = []
        for i in range(n):
            P = int(np.prod([dims[j] for j in range(n) if j != i]))
            J.append(int(rng.integers(ranks[i], min(P, 400) + 1)))
    variant = "R" if rng.integers(0, 3) == 0 else "F"
    dtype = "f32" if rng.integers(0, 3) == 0 else "f64"
    alpha = float(rng.uniform(0.0, 0.3))
    return n, dims, ranks, I, J, variant, dtype, alpha


def _wide_case(k):
    # 3 modes, ranks 6..12 (16-column path), samples up to the full mode
    rng = np.random.default_rng(5000 + k)
    dims = [int(rng.integers(40, 110)) for _ in range(3)]
    ranks = [int(rng.integers(6, 13)) for _ in range(3)]
    I = [int(rng.integers(r + 2, d + 1)) for r, d in zip(ranks, dims)]
    variant = "R" if k % 4 == 3 else "F"
    dtype = "f32" if k % 3 == 2 else "f64"
    return 3, dims, ranks, I, None, variant, dtype, float(rng.uniform(0.05, 0.3))


@pytest.mark.parametrize("k", [f"s{j}" for j in range(40)] + [f"w{j}" for j in range(8)])
def test_random_shape(k):
    kind, j = k[0], int(k[1:])
    n, dims, ranks, I, J, variant, dtype, alpha = _case(j) if kind == "s" else _wide_case(j)
    k = j if kind == "s" else 100 + j
    slice_ = ranks[-1] * int(np.prod(I[1:-1])) if n > 2 else ranks[-1]
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=alpha, seed=50 + k)
    X = inst.X if dtype == "f64" else inst.X.astype(np.float32)
    K = 4
    label = f"{dims} r={ranks} I={I} J={J} {variant} {dtype}"
    if slice_ > _slice_limit(n) or int(np.prod(ranks)) > 4096:
        # outside the documented limits: rejected before any device work
        _, info, _ = run_gpu(X, inst.ranks, I, J, tol=0.0, max_iter=K, seed=7 + k,
                             variant=variant, check=False,
                             dtype=torch.float64 if dtype == "f64" else torch.float32)
        assert info.status == E_INVAL, (label, info.status)
        return
    try:
        res = oracle_rtcur(X, inst.ranks, I, J, None, 0.7, 0.0, K, 7 + k, variant)
        want = None
    except OracleError as e:
        # invalid sizes, or the oracle's rank floor (the library's rank test
        # flags whenever the oracle's does): the library must agree
        assert e.status in (E_INVAL, E_RANK), label
        res, want = None, e.status
    h, info, _ = run_gpu(X, inst.ranks, I, J, tol=0.0, max_iter=K, seed=7 + k,
                         variant=variant, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    if res is None:
        assert info.status == want, (label, info.status, want)
        return
    if info.status == E_RANK:
        assert _in_rank_band(res, ranks, I), (label, res.min_sig_ratio)
        return
    assert info.status >= 0, label
    assert info.iters == res.iters == K, label
    compare(res, h, info, fp64=dtype == "f64", label=label)


@pytest.mark.parametrize("j", range(8))
def test_random_shape_to_tolerance(j):
    # to tol 1e-6 in float64: the iteration count must match the oracle's
    # (unless e^(k) sits within 1e-9 of tol) and so must the returned iterate
    n, dims, ranks, I, J, variant, _, alpha = _case(200 + j)
    slice_ = ranks[-1] * int(np.prod(I[1:-1])) if n > 2 else ranks[-1]
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=min(alpha, 0.15), seed=300 + j)
    label = f"{dims} r={ranks} I={I} J={J} {variant} to tol"
    if slice_ > _slice_limit(n) or int(np.prod(ranks)) > 4096:
        # outside the documented limits: rejected before any device work
        _, info, _ = run_gpu(inst.X, inst.ranks, I, J, tol=1e-6, max_iter=100, seed=3 + j,
                             variant=variant, check=False)
        assert info.status == E_INVAL, (label, info.status)
        return
    try:
        res = oracle_rtcur(inst.X, inst.ranks, I, J, None, 0.7, 1e-6, 100, 3 + j, variant)
    except OracleError as e:
        assert e.status in (E_INVAL, E_RANK), label
        h, info, _ = run_gpu(inst.X, inst.ranks, I, J, tol=1e-6, max_iter=100, seed=3 + j,
                             variant=variant, check=False)
        assert info.status == e.status, (label, info.status, e.status)
        return
    h, info, _ = run_gpu(inst.X, inst.ranks, I, J, tol=1e-6, max_iter=100, seed=3 + j,
                         variant=variant, check=False)
    if info.status == E_RANK:
        assert _in_rank_band(res, ranks, I), (label, res.min_sig_ratio)
        return
    assert info.status >= 0, label
    near = any(abs(e - 1e-6) <= 1e-9 * 1e-6 for e in res.err_hist)
    if not near:
        assert info.iters == res.iters, (label, info.iters, res.iters)
    if info.iters == res.iters:
        compare(res, h, info, fp64=True, label=label)


@pytest.mark.parametrize("variant,dtype", [("F", "f64"), ("F", "f32"), ("R", "f64")])
def test_large_core_slice(variant, dtype):
    # three modes with a sampled core slice of r_2 |I_1| = 12 * 250 = 3000
    # entries (beyond half the common slice buffer): the larger k_zcore
    # instance, against the oracle over K = 4 iterations
    dims, ranks, I = [40, 250, 40], [4, 6, 12], [20, 250, 30]
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=0.2, seed=77)
    X = inst.X if dtype == "f64" else inst.X.astype(np.float32)
    K = 4
    label = f"{dims} r={ranks} I={I} {variant} {dtype}"
    res = oracle_rtcur(X, inst.ranks, I, None, None, 0.7, 0.0, K, 5, variant)
    h, info, _ = run_gpu(X, inst.ranks, I, None, tol=0.0, max_iter=K, seed=5,
                         variant=variant, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    assert info.status >= 0, (label, info.status)
    assert info.iters == res.iters == K, label
    compare(res, h, info, fp64=dtype == "f64", label=label)
