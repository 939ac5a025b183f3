"""GPU parity at the edges of the truncated SVD (equation 9, Theorem 2.5's
rank condition), on ill-conditioned low-rank parts, on the hand-worked
stopping-rule case, and for stream ordering in the binding.

The rank band.  The oracle rejects U_i when sigma_r / sigma_1 <=
max(|I_i|, |J_i|) 2^-52 (what its LAPACK SVD resolves).  The library's
eigensolver sees the Gram U_i U_i^T, whose eigenvalue ratio is the square of
that, and flags when its bound 1 / (||T||_F ||T^-1||_F) on lambda_r /
lambda_1 falls to 64 |I_i| 2^-52: surely when sigma_r / sigma_1 <=
sqrt(64 |I_i| 2^-52), never above sqrt(64 r |I_i| 2^-52).  Between the two
floors the library returns E_RANK and the oracle a result; the tests below
build U_i with a known singular-value ratio in each region."""
import math

import numpy as np
import pytest

import synth
from oracle import OracleError
from oracle import rtcur as oracle_rtcur

from _parity import compare, rel, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = 2.0 ** -52


def _superdiagonal(dims, g, seed):
    """sum_k g_k u_k (x) v_k (x) w_k with orthonormal factor columns: every
    unfolding has singular values exactly |g_k| (up to rounding)."""
    rng = np.random.default_rng(seed)
    fac = [np.linalg.qr(rng.standard_normal((d, len(g))))[0] for d in dims]
    X = np.zeros(dims)
    for k, gk in enumerate(g):
        X += gk * np.einsum("a,b,c->abc", fac[0][:, k], fac[1][:, k], fac[2][:, k])
    return X


def _band_upper(s, r):
    return math.sqrt(64.0 * r * s * EPS)


@pytest.mark.parametrize("ratio,expect", [
    (1e-3, "both_ok"),      # above the library's floor
    (1e-9, "band"),         # between the two floors
    (0.0, "both_rank"),     # exactly rank deficient
])
def test_rank_band(ratio, expect):
    import paper_2108_10448_amd as rt
    dims = (14, 12, 10)
    X = _superdiagonal(dims, [1.0, ratio], seed=4)
    ranks, I = (2, 2, 2), dims           # full sampling: U_i = X_(i)
    zeta0 = 1e3 * float(np.max(np.abs(X)))   # no entry ever thresholded
    try:
        res = oracle_rtcur(X, ranks, I, None, zeta0, 0.7, 0.0, 3, 0, "F")
        ostat = 0
    except OracleError as e:
        res, ostat = None, e.status
    h, info, _ = run_gpu(X, ranks, I, zeta0=zeta0, tol=0.0, max_iter=3, check=False)
    print(f"[rank band] ratio {ratio}: oracle {ostat} "
          f"(min sigma ratio {res.min_sig_ratio if res else None}), library {info.status}",
          flush=True)
    if expect == "both_ok":
        assert ostat == 0 and info.status >= 0
        compare(res, h, info, label=f"rank band {ratio}")
    elif expect == "band":
        assert ostat == 0 and info.status == rt.E_RANK
        assert res.min_sig_ratio <= _band_upper(max(I), 2)
        # far above the oracle's own floor, max(s, m) eps (m = 168 here)
        assert res.min_sig_ratio > 1e3 * 168 * EPS
    else:
        assert ostat == rt.E_RANK and info.status == rt.E_RANK


@pytest.mark.parametrize("variant", ["F", "R"])
def test_fp32_ill_conditioned(variant):
    # the low-rank part's unfoldings have sigma_5 / sigma_1 of 6e-5 to 3e-4;
    # the sampled U_i the loop meets reach kappa = sigma_1 / sigma_r of about
    # 180 (RTCUR-F) and beyond (RTCUR-R): the float32 eigensolver's stopping
    # scale follows the weakest pair
    inst = synth.tucker_plus_sparse((90, 80, 70), (5, 5, 5), alpha=0.15, seed=3,
                                    spread=300.0)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    X = inst.X.astype(np.float32)
    h, info, _ = run_gpu(X, inst.ranks, I, variant=variant, dtype=torch.float32, check=False)
    assert info.status >= 0 and info.eig_unconverged == 0
    res = oracle_rtcur(X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, variant)
    ref = oracle_rtcur(X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, variant)
    print(f"[kappa] min sigma ratio {ref.min_sig_ratio:.3e} iters gpu {info.iters} "
          f"oracle {ref.iters}", flush=True)
    assert ref.min_sig_ratio < 1e-2
    assert abs(info.iters - ref.iters) <= 1
    compare(res, h, info, fp64=False, label=f"kappa>=100 fp32 {variant}")


def test_worked_stopping_rule_case():
    # the 3 x 3 case worked by hand in tests/test_oracle_error_rule.py
    X = np.array([[3.0, 0.0, 1.0], [0.0, 1.0, 2.0], [4.0, 3.0, 5.0]])
    h, info, _ = run_gpu(X, (1, 1), (2, 2), zeta0=1000.0, tol=0.0, max_iter=1, seed=5,
                         check=False)
    want = (1.0 + math.sqrt(10.0) + math.sqrt(5.0)) / (
        math.sqrt(10.0) + math.sqrt(35.0) + math.sqrt(15.0))
    assert info.iters == 1
    assert abs(info.err - want) <= 1e-14 * want
    res = oracle_rtcur(X, (1, 1), (2, 2), None, 1000.0, 0.7, 0.0, 1, 5, "F")
    compare(res, h, info, label="worked 3x3")


def test_stream_ordering_with_producer_kernel():
    # X is produced by device work queued on torch's current stream; the
    # handle runs on a stream of its own.  The binding makes the handle's
    # stream wait, so the solve sees the finished X.
    import paper_2108_10448_amd as rt
    inst = synth.tucker_plus_sparse((80, 70, 60), (3, 3, 3), alpha=0.2, seed=9)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 4, 0, "F")
    side = torch.cuda.Stream()
    h = rt.create(0, stream=side)
    host = torch.from_numpy(inst.X).pin_memory()
    X = torch.empty(inst.dims, dtype=torch.float64, device="cuda:0")
    # a long chain of kernels on the current stream ends in the real X
    big = torch.randn(4096, 4096, device="cuda:0", dtype=torch.float64)
    for _ in range(6):
        big = torch.tanh(big @ big.T / 4096.0)
    X.copy_(host, non_blocking=True)
    X.mul_(2.0).add_(big[0, 0] * 0.0).mul_(0.5)
    info = rt.solve(h, X, inst.ranks, I, tol=0.0, max_iter=4, check=False)
    L = rt.reconstruct(h)
    torch.cuda.synchronize()
    assert info.iters == 4
    assert rel(L.cpu().numpy(), res.reconstruct()) <= 1e-10
    compare(res, h, info, label="stream ordering")
    rt.destroy(h)
