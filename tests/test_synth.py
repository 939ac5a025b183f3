"""The seeded generators themselves (input construction, not the method):
shapes, determinism and the stated properties of each recipe."""
import numpy as np

import synth


def test_tucker_plus_sparse_recipe():
    a = synth.tucker_plus_sparse((12, 10, 8), (2, 3, 2), alpha=0.25, seed=4)
    b = synth.tucker_plus_sparse((12, 10, 8), (2, 3, 2), alpha=0.25, seed=4)
    assert np.array_equal(a.X, b.X)
    assert np.allclose(a.X, a.L_star + a.S_star)
    # multilinear rank of L*: each unfolding has rank r_i
    for i, r in enumerate(a.ranks):
        U = np.moveaxis(a.L_star, i, 0).reshape(a.dims[i], -1)
        sv = np.linalg.svd(U, compute_uv=False)
        assert sv[r - 1] > 1e-8 * sv[0] and (len(sv) == r or sv[r] < 1e-10 * sv[0])
    amp = a.meta["amp"]
    vals = a.S_star[a.S_star != 0]
    assert np.all(np.abs(vals) <= amp)
    assert 0.15 < np.mean(a.S_star != 0) < 0.35


def test_video_like_recipe():
    v = synth.video_like((48, 64, 3, 60), side=(6, 14), seed=1, storage=np.float64)
    w = synth.video_like((48, 64, 3, 60), side=(6, 14), seed=1, storage=np.float64)
    assert np.array_equal(v.X, w.X)
    assert v.X.shape == (48, 64, 3, 60)
    assert np.allclose(v.X, v.L_star + v.S_star)
    # nonnegative background scaled to max 1, Tucker rank (10, 10, 3, 5)
    assert v.L_star.min() >= 0.0 and np.isclose(v.L_star.max(), 1.0)
    for i, r in enumerate(v.ranks):
        U = np.moveaxis(v.L_star, i, 0).reshape(v.dims[i], -1)
        sv = np.linalg.svd(U, compute_uv=False)
        assert len(sv) == r or sv[r] < 1e-10 * sv[0]
    # the foreground is the same in every colour channel's support, and its
    # realised coverage of (pixel, frame) pairs is near the 5 % target
    occ = v.S_star != 0
    assert np.array_equal(occ[:, :, 0, :], occ[:, :, 1, :])
    cov = float(np.mean(occ[:, :, 0, :]))
    assert abs(cov - v.meta["coverage"]) < 1e-12
    assert 0.035 < cov < 0.065


def test_device_recipe_matches_the_host_recipe_in_distribution():
    # the torch-drawn variant (on the CPU here): exact multilinear rank,
    # orthonormal-factor scale, Bernoulli(alpha) support, values within amp,
    # reproducible per seed
    import torch
    X, L = synth.tucker_plus_sparse_device((30, 28, 26), (3, 2, 4), 0.25, seed=7, device="cpu")
    assert X.dtype == torch.float32 and L.dtype == torch.float64 and X.shape == (30, 28, 26)
    assert X.is_contiguous() and L.is_contiguous()
    Ln = L.numpy()
    for k, r in enumerate((3, 2, 4)):
        sv = np.linalg.svd(np.moveaxis(Ln, k, 0).reshape(Ln.shape[k], -1), compute_uv=False)
        assert sv[r - 1] > 1e-8 * sv[0] and sv[r] < 1e-12 * sv[0]
    S = X.double().numpy() - Ln
    supp = np.abs(S) > 1e-5 * np.abs(Ln).mean()
    assert abs(supp.mean() - 0.25) < 0.02
    amp = np.abs(Ln).mean()
    assert np.abs(S).max() <= amp * (1 + 1e-6) + 1e-6
    X2, _ = synth.tucker_plus_sparse_device((30, 28, 26), (3, 2, 4), 0.25, seed=7, device="cpu")
    assert torch.equal(X, X2)
