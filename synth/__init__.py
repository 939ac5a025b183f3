"""Seeded synthetic inputs for robust tensor PCA: X = L* + S*.

This module draws test and benchmark inputs only.  It holds none of the
RTCUR arithmetic: the oracle under ``oracle/`` and the HIP library both take
the tensor it returns as a plain input, and neither imports the other.

Recipe (the synthetic experiment of Section 4.1, restated with the choices
written out in the design doc):

* L* = G x_1 U_1 x_2 ... x_n U_n with core G of i.i.d. N(0,1) entries and
  factors U_i whose columns are the Q factor of a d_i x r_i i.i.d. N(0,1)
  matrix (``orthonormal=False`` keeps the raw Gaussian factors, as the paper's
  text does);
* the support of S* is Bernoulli(alpha) per entry, and its values are i.i.d.
  uniform in [-c * mean|L*|, c * mean|L*|];
* draw order from ``numpy.random.default_rng(seed)``: core, U_1 .. U_n,
  support mask, values.  X is formed in float64 and then cast to the storage
  dtype, so float32 storage upcasts back to float64 exactly.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

__all__ = ["Instance", "tucker_plus_sparse", "video_like", "batch_specs",
           "sample_sizes", "CONFIGS", "config_instance"]


@dataclass
class Instance:
    X: np.ndarray                      # observed tensor, storage dtype
    L_star: np.ndarray                 # low-rank part, float64
    S_star: np.ndarray                 # sparse part, float64 (dense array)
    dims: tuple
    ranks: tuple
    alpha: float
    seed: int
    meta: dict = field(default_factory=dict)


def _tucker(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Full tensor core x_1 U_1 ... x_n U_n (input construction only)."""
    out = core
    for k, U in enumerate(factors):
        # contract axis k of `out` with the columns of U, put the new axis back
        out = np.moveaxis(np.tensordot(U, out, axes=(1, k)), 0, k)
    return out


def tucker_plus_sparse(dims: Sequence[int], ranks: Sequence[int], alpha: float,
                       c: float = 1.0, seed: int = 0,
                       storage=np.float64, orthonormal: bool = True,
                       keep_parts: bool = True, spread: float = 1.0) -> Instance:
    """Low-multilinear-rank tensor plus Bernoulli(alpha) sparse outliers.

    spread > 1 scales the core's slices along every mode by a geometric
    sequence from 1 down to 1/spread (after the draws, so the draw order is
    unchanged): the unfoldings' singular values then spread over about that
    factor, an ill-conditioned low-rank part."""
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    if len(dims) != len(ranks):
        raise ValueError("dims and ranks must have the same length")
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    if spread != 1.0:
        for k, r in enumerate(ranks):
            w = spread ** (-np.arange(r) / max(r - 1, 1))
            shape = [1] * len(ranks)
            shape[k] = r
            core = core * w.reshape(shape)
    factors = []
    for d, r in zip(dims, ranks):
        Y = rng.standard_normal((d, r))
        if orthonormal:
            Y = np.linalg.qr(Y)[0]
        factors.append(Y)
    L = _tucker(core, factors)
    mask = rng.random(dims) < alpha
    amp = c * float(np.mean(np.abs(L)))
    vals = rng.uniform(-amp, amp, size=int(mask.sum()))
    S = np.zeros(dims, dtype=np.float64)
    S[mask] = vals
    X = (L + S).astype(storage)
    meta = {"amp": amp, "support": int(mask.sum()), "c": c,
            "orthonormal": orthonormal}
    if not keep_parts:
        return Instance(X, None, None, dims, ranks, alpha, seed, meta)
    return Instance(X, L, S, dims, ranks, alpha, seed, meta)


def tucker_plus_sparse_device(dims: Sequence[int], ranks: Sequence[int], alpha: float,
                              seed: int, device, c: float = 1.0):
    """The recipe of tucker_plus_sparse drawn with torch on `device` (for
    training sets too large to draw on the host): N(0,1) core, QR-orthonormal
    N(0,1) factors, Bernoulli(alpha) support, values U[-amp, amp] with
    amp = c mean|L*|, in that order from one torch.Generator seeded with
    `seed` (a different stream of numbers than numpy's for the same seed).
    Returns (X float32, L* float64) on the device."""
    import torch
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    L = torch.randn(ranks, generator=g, device=device, dtype=f64)
    for k, (d, r) in enumerate(zip(dims, ranks)):
        U = torch.linalg.qr(torch.randn((d, r), generator=g, device=device, dtype=f64))[0]
        L = torch.movedim(torch.tensordot(U, L, dims=([1], [k])), 0, k)
    mask = torch.rand(dims, generator=g, device=device, dtype=f64) < alpha
    amp = c * float(L.abs().mean())
    vals = (torch.rand(dims, generator=g, device=device, dtype=f64) * 2.0 - 1.0) * amp
    L = L.contiguous()
    X = (L + torch.where(mask, vals, torch.zeros_like(vals))).to(torch.float32).contiguous()
    return X, L


def video_like(dims: Sequence[int] = (240, 320, 3, 400),
               ranks: Sequence[int] = (10, 10, 3, 5), n_rects: int = 40,
               side: tuple = (20, 60), coverage: float = 0.05, seed: int = 0,
               storage=np.float32, keep_parts: bool = True) -> Instance:
    """Video-shaped 4-mode tensor (height x width x colour x frame).

    Background L*: Tucker rank ``ranks`` with i.i.d. U[0, 1] core and factors
    (nonnegative), scaled so that max L* = 1.  Foreground S*: ``n_rects``
    axis-aligned rectangles with sides uniform in ``side`` pixels, one
    intensity U[0, 1] per rectangle and colour channel, each visible during a
    window of frames in which it moves at a constant velocity (clipped at the
    frame border).  Window lengths are scaled once so that the covered share
    of (pixel, frame) pairs is close to ``coverage``; the realised share is
    returned in ``meta["coverage"]``.  X = L* + S* in float64, then cast to
    the storage dtype.  Draw order: core, factors, rectangles (size, start,
    velocity, window start, window length, intensities).
    """
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    if len(dims) != 4:
        raise ValueError("video_like draws height x width x colour x frame")
    H, W, CH, F = dims
    rng = np.random.default_rng(seed)
    core = rng.random(ranks)
    factors = [rng.random((d, r)) for d, r in zip(dims, ranks)]
    L = _tucker(core, factors)
    L /= float(L.max())
    sides = rng.integers(side[0], side[1] + 1, size=(n_rects, 2))
    y0 = rng.uniform(0, H - sides[:, 0])
    x0 = rng.uniform(0, W - sides[:, 1])
    vel = rng.uniform(-3.0, 3.0, size=(n_rects, 2))
    t_start = rng.random(n_rects)
    t_len = rng.uniform(0.5, 1.5, size=n_rects)
    inten = rng.random((n_rects, CH))

    def windows(scale):
        lens = np.maximum(1, np.round(scale * t_len)).astype(int)
        starts = np.floor(t_start * np.maximum(F - lens, 0)).astype(int)
        return starts, lens

    def paint(scale, S=None):
        starts, lens = windows(scale)
        occ = np.zeros((F, H, W), dtype=bool) if S is None else None
        for k in range(n_rects):
            h, w = int(sides[k, 0]), int(sides[k, 1])
            for f in range(starts[k], min(F, starts[k] + lens[k])):
                dt = f - starts[k]
                y = int(round(min(max(y0[k] + vel[k, 0] * dt, 0), H - h)))
                x = int(round(min(max(x0[k] + vel[k, 1] * dt, 0), W - w)))
                if S is None:
                    occ[f, y:y + h, x:x + w] = True
                else:
                    S[y:y + h, x:x + w, :, f] += inten[k]
        return None if S is None else S, (occ.mean() if occ is not None else None)

    # one calibration step of the window length towards the target share
    base = coverage * F * H * W / float(np.sum(sides[:, 0] * sides[:, 1]))
    _, cov0 = paint(base)
    scale = base * coverage / max(cov0, 1e-12)
    _, cov = paint(scale)
    S = np.zeros(dims, dtype=np.float64)
    paint(scale, S)
    X = (L + S).astype(storage)
    meta = {"coverage": float(cov), "window_scale": float(scale)}
    if not keep_parts:
        return Instance(X, None, None, dims, ranks, coverage, seed, meta)
    return Instance(X, L, S, dims, ranks, coverage, seed, meta)


def batch_specs(count: int = 64, dmin: int = 64, dmax: int = 256, rmin: int = 2,
                rmax: int = 8, amin: float = 0.1, amax: float = 0.4, seed: int = 0):
    """Shapes of a batch of independent 3-mode instances of uneven sizes: per
    instance and mode d ~ U{dmin..dmax} and r ~ U{rmin..rmax}, and
    alpha ~ U[amin, amax], drawn from default_rng(seed) in that order.
    Returns a list of dicts (dims, ranks, alpha, seed = seed + j) for
    tucker_plus_sparse."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        dims = tuple(int(x) for x in rng.integers(dmin, dmax + 1, size=3))
        ranks = tuple(int(x) for x in rng.integers(rmin, rmax + 1, size=3))
        alpha = float(rng.uniform(amin, amax))
        out.append({"dims": dims, "ranks": ranks, "alpha": alpha, "seed": seed + j})
    return out


def sample_sizes(dims: Sequence[int], ranks: Sequence[int],
                 upsilon: float = 3.0, fiber: bool = False):
    """|I_i| = ceil(upsilon r_i ln d_i) clamped to d_i (Section 4 sizes rule).

    With ``fiber=True`` also returns |J_i| = ceil(upsilon r_i ln prod_{j!=i} d_j)
    clamped to prod_{j!=i} d_j; otherwise J sizes are None (chidori).
    """
    dims = [int(d) for d in dims]
    I = [min(d, int(math.ceil(upsilon * r * math.log(d)))) for d, r in
         zip(dims, ranks)]
    if not fiber:
        return I, None
    J = []
    for i, r in enumerate(ranks):
        P = 1
        for j, d in enumerate(dims):
            if j != i:
                P *= d
        J.append(min(P, int(math.ceil(upsilon * r * math.log(P)))))
    return I, J


# Named workloads.  Each is a dict of generator and solver settings.
CONFIGS = {
    # 100^3 float64, rank 3, alpha 0.2 (small case the oracle finishes fast)
    "cube100_r3": dict(dims=(100, 100, 100), ranks=(3, 3, 3), alpha=0.2,
                       c=1.0, storage=np.float64, upsilon=3.0, gamma=0.7,
                       tol=1e-5, max_iter=100, seed=0),
    # 300^3 float32 storage, rank 5, alpha 0.3 (the headline workload)
    "cube300_r5": dict(dims=(300, 300, 300), ranks=(5, 5, 5), alpha=0.3,
                       c=1.0, storage=np.float32, upsilon=3.0, gamma=0.7,
                       tol=1e-5, max_iter=100, seed=0),
}


def config_instance(name: str, seed: Optional[int] = None, **over) -> Instance:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    return tucker_plus_sparse(cfg["dims"], cfg["ranks"], cfg["alpha"],
                              c=cfg["c"], seed=cfg["seed"] if seed is None
                              else seed, storage=cfg["storage"])
