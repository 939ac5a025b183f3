"""The eigensolver's guarded stage below rank 16 (RP = 4 here), against the
oracle: the data has multilinear rank (4, 3, 3) with the mode-0 unfolding's
fourth singular value 0.97 of its third, and the solve asks for (3, 3, 3).
The sampled mode-0 Gram then has lambda_4 / lambda_3 near 0.94, too slow for
the plain subspace iteration, so the eigensolver takes the guarded
(Rayleigh-Ritz) stage with m = 4 columns, which converges at the noise level
of lambda_5. Five iterations from the same sample, float64 and float32
blocks, each within the usual parity bar of the oracle."""
import numpy as np
import pytest

import synth
from oracle import rtcur as oracle_rtcur

from _parity import compare, run_gpu

torch = pytest.importorskip("torch")


def slow_gap_instance(dims=(90, 80, 70), ratio=0.97, alpha=0.1, seed=3):
    """X = L + S with L of multilinear rank (4, 3, 3): a core whose mode-0
    unfolding has singular values (1, 0.8, 0.6, 0.6 ratio), orthonormal
    factors, S sparse (Bernoulli(alpha) support, values uniform in
    [-mean|L|, mean|L|])."""
    rng = np.random.default_rng(seed)
    r = (4, 3, 3)
    core = rng.standard_normal(r)
    u, _, vt = np.linalg.svd(core.reshape(r[0], -1), full_matrices=False)
    sv = np.array([1.0, 0.8, 0.6, 0.6 * ratio])
    core = ((u * sv) @ vt).reshape(r)
    U = [np.linalg.qr(rng.standard_normal((d, k)))[0] for d, k in zip(dims, r)]
    L = np.einsum("abc,ia,jb,kc->ijk", core, *U)
    L /= np.abs(L).mean()
    supp = rng.random(dims) < alpha
    S = np.where(supp, rng.uniform(-1.0, 1.0, dims), 0.0)
    return L + S


def test_slow_gap_instance_has_the_gap():
    # (a property of the input, checked on the host: the low-rank part's
    # mode-0 spectrum has the planted ratio)
    X = slow_gap_instance(alpha=0.0)
    sv = np.linalg.svd(X.reshape(X.shape[0], -1), compute_uv=False)
    assert abs(sv[3] / sv[2] - 0.97) < 1e-9 and sv[4] < 1e-9 * sv[0]


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_guarded_stage_rank_below_16(dtype):
    X = slow_gap_instance()
    if dtype == "f32":
        X = X.astype(np.float32)
    ranks = (3, 3, 3)
    I, _ = synth.sample_sizes(X.shape, ranks, 3.0)
    K = 5
    res = oracle_rtcur(X, ranks, I, None, None, 0.7, 0.0, K, 11, "F")
    h, info, _ = run_gpu(X, ranks, I, tol=0.0, max_iter=K, seed=11, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    print(f"[guarded] {dtype}: eig steps {info.eig_steps} unconverged "
          f"{info.eig_unconverged} err {info.err:.6e} oracle {res.err:.6e}", flush=True)
    assert info.iters == K and info.eig_unconverged == 0
    compare(res, h, info, fp64=dtype == "f64", label=f"slow gap {dtype}")
