"""Oracle for the differentiable unrolled RTCUR-F: K iterations of Algorithm 1
on one fixed sample (RTCUR-F, Section 3.4) with the per-iteration thresholds
zeta_1..zeta_K given as inputs instead of the geometric schedule of
equation 12, written with plain PyTorch CPU float64 operations so that
torch.autograd supplies the reference gradient with respect to the
thresholds and to X.

TEST INFRASTRUCTURE ONLY.  Only tests/ and the benchmark's CPU leg may import
this module; the HIP library never does, and the two share no code.

The hard threshold of equation 10 has zero derivative in zeta almost
everywhere, so the differentiable form replaces it, and only it, by a
smooth gate:

    S = D * sigmoid((|D| / zeta - 1) / tau)          (tau > 0)

which tends to the hard threshold as tau -> 0; tau = 0 is the hard
threshold itself (then this is exactly the oracle's RTCUR-F with that
schedule).  Everything else is Algorithm 1's L-update in its literal form
(equations 8-9): U_i = C_i(I_i, :), A_i = C_i U_i^+ with U_i^+ the
pseudo-inverse of the rank-r_i truncation, L = R x_i A_i evaluated on the
sampled blocks (chidori sampling, three or more modes).  The truncated
pseudo-inverse is formed as U_i^T (U_i U_i^T)_r^+, the Moore-Penrose inverse
of the rank-r truncation written through the Gram's eigendecomposition
(the same operator as V_r S_r^-1 W_r^T of the SVD; torch.linalg.eigh and its
autograd rule supply the derivative).
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from .sampler import draw_sample


def gate(D: torch.Tensor, zeta, tau: float) -> torch.Tensor:
    """The threshold step S = HT_zeta(D) (tau = 0, equation 10, strict) or its
    smooth form D * sigmoid((|D| / zeta - 1) / tau)."""
    if tau == 0.0:
        return torch.where(D.abs() > zeta, D, torch.zeros_like(D))
    return D * torch.sigmoid((D.abs() / zeta - 1.0) / tau)


def _mode_product(T: torch.Tensor, A: torch.Tensor, k: int) -> torch.Tensor:
    """T x_k A (A of shape (J, d_k)): every mode-k fibre multiplied by A."""
    return torch.movedim(torch.tensordot(A, T, dims=([1], [k])), 0, k)


def _unfold(T: torch.Tensor, k: int) -> torch.Tensor:
    return torch.movedim(T, k, 0).reshape(T.shape[k], -1)


def blocks_of(X: torch.Tensor, samp) -> List[torch.Tensor]:
    """R = X(I_1..I_n) and C_i = X_(i)(:, J_i) (chidori J_i)."""
    n = X.dim()
    idx = [torch.as_tensor(np.asarray(I), dtype=torch.long) for I in samp.I]
    R = X
    for k in range(n):
        R = torch.index_select(R, k, idx[k])
    out = [R]
    for i in range(n):
        Ci = X
        for k in range(n):
            if k != i:
                Ci = torch.index_select(Ci, k, idx[k])
        out.append(_unfold(Ci, i))
    return out


def truncated_pinv_gram(U: torch.Tensor, r: int) -> torch.Tensor:
    """U^+ of the rank-r truncation of U: U^T (U U^T)_r^+ with
    (U U^T)_r^+ = V_r diag(1 / lambda_r) V_r^T from the Gram's top r
    eigenpairs."""
    lam, V = torch.linalg.eigh(U @ U.T)        # ascending
    Vr, lr = V[:, -r:], lam[-r:]
    return U.T @ ((Vr / lr) @ Vr.T)


def evaluate(R: torch.Tensor, A: Sequence[torch.Tensor], I) -> List[torch.Tensor]:
    """L = R x_i A_i on the sampled blocks (chidori): on R every factor is
    its rows at I_i; on C_i factor i is whole."""
    n = R.dim()
    idx = [torch.as_tensor(np.asarray(v), dtype=torch.long) for v in I]
    rows = [A[j][idx[j], :] for j in range(n)]
    LR = R
    for j in range(n):
        LR = _mode_product(LR, rows[j], j)
    out = [LR]
    for i in range(n):
        T = R
        for j in range(n):
            T = _mode_product(T, A[i] if j == i else rows[j], j)
        out.append(_unfold(T, i))
    return out


def unrolled(X: torch.Tensor, ranks: Sequence[int], I_sizes: Sequence[int],
             zetas: torch.Tensor, tau: float, seed: int = 0) -> List[torch.Tensor]:
    """L^K on the sampled blocks [R, C_1 .. C_n] after K = len(zetas)
    iterations of RTCUR-F started from L^0 = 0, iteration k thresholding with
    zetas[k - 1].  X (float64, any requires_grad) and zetas are torch
    tensors; the sample is drawn for seed and resample counter 0 (chidori)."""
    n = X.dim()
    samp = draw_sample(seed, 0, tuple(X.shape), I_sizes, None)
    XB = blocks_of(X, samp)
    LB = [torch.zeros_like(b) for b in XB]
    idx = [torch.as_tensor(np.asarray(v), dtype=torch.long) for v in samp.I]
    for k in range(len(zetas)):
        CB = [XB[b] - gate(XB[b] - LB[b], zetas[k], tau) for b in range(n + 1)]
        A = []
        for i in range(n):
            Ci = CB[1 + i]
            A.append(Ci @ truncated_pinv_gram(Ci[idx[i], :], int(ranks[i])))
        LB = evaluate(CB[0], A, samp.I)
    return LB
