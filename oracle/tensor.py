"""Oracle tensor primitives (Section 2.1 definitions), plain numpy float64.

TEST INFRASTRUCTURE ONLY; never imported by the product path.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np


def unfold(T: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding T_(k) (Definition of matricization, Section 2.1).

    Rows are indexed by mode k; columns run over the remaining modes in C
    order (increasing mode number, last fastest).
    """
    return np.moveaxis(T, k, 0).reshape(T.shape[k], -1)


def fold(M: np.ndarray, k: int, shape: Sequence[int]) -> np.ndarray:
    """Inverse of unfold for a tensor of the given shape."""
    rest = [shape[j] for j in range(len(shape)) if j != k]
    return np.moveaxis(M.reshape([shape[k]] + rest), 0, k)


def mode_product(T: np.ndarray, A: np.ndarray, k: int) -> np.ndarray:
    """Y = T x_k A with A of shape (J, d_k): Y_(k) = A T_(k) (mode-k product
    definition, Section 2.1)."""
    return np.moveaxis(np.tensordot(A, T, axes=(1, k)), 0, k)


def multi_mode_product(T: np.ndarray, mats) -> np.ndarray:
    """T x_1 A_1 x_2 ... x_n A_n, applied in mode order."""
    out = T
    for k, A in enumerate(mats):
        out = mode_product(out, A, k)
    return out


def hard_threshold(D: np.ndarray, zeta: float) -> np.ndarray:
    """HT_zeta (equation 10): keep an entry iff its magnitude is strictly
    greater than zeta, else zero."""
    return np.where(np.abs(D) > zeta, D, 0.0)


def fro(A: np.ndarray) -> float:
    """Frobenius norm, sqrt of the sum of squares (Section 1.2)."""
    return float(np.sqrt(np.sum(A * A)))


def round_bf16(A: np.ndarray) -> np.ndarray:
    """Each value rounded to the nearest bfloat16 (8 significant bits: the
    sign, an 8-bit exponent and 7 stored fraction bits), ties to the even
    significand; finite normal values only.  Used to hold the sampled blocks
    at bfloat16 storage precision (the mixed-precision mode); not part of
    the paper's algorithm, which is stated in exact arithmetic."""
    A = np.asarray(A, dtype=np.float64)
    m, e = np.frexp(A)                  # A = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)   # rint: ties to even
