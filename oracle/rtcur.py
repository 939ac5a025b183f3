"""Oracle RTCUR: Algorithm 1 with the L-update of Section 3.1, the partial
S-update of Section 3.3 (equation 13), the sampled stopping rule (equation 14)
and both variants of Section 3.4.  Plain numpy, float64 throughout.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module; the HIP library never does, and the
two share no code.

The oracle deliberately uses the literal form of the L-update,
L = R x_i (C_i U_i^+) (equation 8), evaluated on the sampled blocks, and
calls LAPACK (numpy.linalg.svd) for the truncated SVD.

Readings of the paper where it is silent (each listed in the design doc):

* blocks: the sampled set is the core subtensor R (rows I_1 x ... x I_n) and
  the n fiber blocks C_i = X_(i)(:, J_i).  Each block keeps its own S and its
  own error, even where blocks overlap (equations 13 and 14 treat them
  separately);
* threshold: zeta_{k+1} = gamma * zeta_k by repeated float64 multiplication,
  applied before the hard threshold, so the first threshold is gamma*zeta_0;
  zeta_0 <= 0 means max|X| over the whole tensor;
* hard threshold keeps |x| > zeta strictly (equation 10);
* e^(0) = 1 (E^(0) = X on the blocks); the loop stops when e^(k) <= tol or
  after max_iter L-updates (status NOT_CONVERGED);
* RTCUR-R draws a fresh sample before every iteration after the first
  (resample counter t = k before iteration k+1), gathers X there, evaluates the
  stored L^(k) there, and computes e^(k+1) and its denominator on that sample;
* rank test: Theorem 2.5 needs rank(U_i) = r_i; the truncated SVD is rejected
  (status E_RANK) when sigma_r <= max(|I_i|, |J_i|) * 2^-52 * sigma_1, the
  level below which LAPACK's SVD of U_i cannot tell sigma_r from rounding
  (its backward error is a small multiple of max(|I_i|, |J_i|) eps sigma_1).
  The library's eigensolver works on the Gram U_i U_i^T and resolves less
  (reading R14): it may report E_RANK where this oracle does
  not, never the other way round.

Besides the result, each run records the smallest sigma_r / sigma_1 met in
any truncated SVD (Result.min_sig_ratio), so that a test can tell whether a
rank report of the library lies in that documented band.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from .sampler import Sample, draw_sample
from .tensor import (fro, hard_threshold, mode_product, multi_mode_product, round_bf16,
                     unfold)

OK = 0
NOT_CONVERGED = 1
E_INVAL = -1
E_RANK = -4
E_NONFINITE = -5


class OracleError(Exception):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def rank_rtol(s: int, m: int) -> float:
    """Relative singular-value floor of the rank test for an s x m U_i:
    max(s, m) * 2^-52 (see module doc)."""
    return max(int(s), int(m)) * 2.0 ** -52


@dataclass
class Factors:
    """Fiber CUR components of L: R (core subtensor of X - S) and
    A_i = C_i U_i^+ (d_i x |I_i|).  Also keeps the truncated SVD of each U_i
    (W: |I_i| x r_i, sig: r_i, V: |J_i| x r_i) for tests."""
    R: np.ndarray
    A: List[np.ndarray]
    W: List[np.ndarray] = field(default_factory=list)
    sig: List[np.ndarray] = field(default_factory=list)
    V: List[np.ndarray] = field(default_factory=list)


@dataclass
class Result:
    status: int
    iters: int
    err_hist: List[float]          # e^(1) .. e^(k)
    zeta_hist: List[float]         # zeta_1 .. zeta_k
    zeta0: float
    den: float                     # denominator of e^(k) on the final sample
    sample: Optional[Sample]       # the sample the final iterate lives on
    XB: List[np.ndarray]           # X on the blocks [R, C_1 .. C_n]
    CB: List[np.ndarray]           # X - S^(k) on the blocks
    SB: List[np.ndarray]           # S^(k) on the blocks
    LB: List[np.ndarray]           # L^(k) on the blocks
    factors: Optional[Factors]
    dims: tuple = ()
    min_sig_ratio: float = 1.0     # smallest sigma_r / sigma_1 of any U_i seen
    DB: List[np.ndarray] = field(default_factory=list)  # X - L^(k-1) on the
                                   # blocks: the residual the last threshold saw

    @property
    def err(self) -> float:
        return self.err_hist[-1] if self.err_hist else 1.0

    @property
    def support(self) -> List[np.ndarray]:
        return [s != 0 for s in self.SB]

    def reconstruct(self) -> np.ndarray:
        """Full L = R x_1 A_1 ... x_n A_n (equation 8 on the whole grid)."""
        if self.factors is None:
            return np.zeros(self.dims)
        return multi_mode_product(self.factors.R, self.factors.A)


def gather_blocks(X: np.ndarray, samp: Sample) -> List[np.ndarray]:
    """R = X(I_1, .., I_n) and C_i = X_(i)(:, J_i) (Algorithm 1, Section 3.1)."""
    R = X[np.ix_(*samp.I)]
    C = [unfold(X, i)[:, samp.J_cols[i]] for i in range(X.ndim)]
    return [R] + C


def truncated_pinv(U: np.ndarray, r: int):
    """SVD_r(U) and its Moore-Penrose pseudo-inverse V_r S_r^-1 W_r^T."""
    W, sig, Vt = np.linalg.svd(U, full_matrices=False)
    if not np.all(np.isfinite(sig)):
        raise OracleError(E_NONFINITE, "non-finite singular values")
    if sig[0] == 0.0 or sig[r - 1] <= rank_rtol(U.shape[0], U.shape[1]) * sig[0]:
        raise OracleError(E_RANK, "U_i has numerical rank below r_i")
    Wr, sr, Vr = W[:, :r], sig[:r], Vt[:r].T
    pinv = Vr @ (Wr / sr).T
    return Wr, sr, Vr, pinv


def l_update(CB: List[np.ndarray], samp: Sample, ranks: Sequence[int]) -> Factors:
    """Step (II) of Algorithm 1: R, C_i, U_i from X - S (equation 9), then
    A_i = C_i U_i^+ so that L = R x_i A_i (equation 8)."""
    n = len(samp.dims)
    R = CB[0].copy()
    f = Factors(R, [])
    for i in range(n):
        C = CB[1 + i]
        U = C[samp.I[i], :]
        Wr, sr, Vr, pinv = truncated_pinv(U, int(ranks[i]))
        f.A.append(C @ pinv)
        f.W.append(Wr)
        f.sig.append(sr)
        f.V.append(Vr)
    return f


def evaluate(f: Factors, samp: Sample) -> List[np.ndarray]:
    """L = R x_i A_i on the sampled blocks only (Section 3.3: the full L is
    never formed)."""
    n = len(samp.dims)
    rows = [f.A[j][samp.I[j], :] for j in range(n)]
    out = [multi_mode_product(f.R, rows)]
    letters = "abcdefghijkl"[:n]
    for i in range(n):
        if samp.chidori:
            mats = [f.A[j] if j == i else rows[j] for j in range(n)]
            out.append(unfold(multi_mode_product(f.R, mats), i))
            continue
        # fiber columns: contract R over every mode j != i with the row of
        # A_j picked by the column's index in mode j, then apply A_i.
        others = [j for j in range(n) if j != i]
        ops = [f.R]
        subs = [letters]
        for k, j in enumerate(others):
            ops.append(f.A[j][samp.J_tuples[i][:, k], :])
            subs.append("z" + letters[j])
        expr = ",".join(subs) + "->" + letters[i] + "z"
        core_cols = np.einsum(expr, *ops, optimize=True)
        out.append(f.A[i] @ core_cols)
    return out


# e^(k) at which the bfloat16-storage emulation goes over to full precision
BF16_SWITCH = 1e-2


def rtcur(X: np.ndarray, ranks: Sequence[int], I_sizes: Sequence[int],
          J_sizes: Optional[Sequence[int]] = None, zeta0: Optional[float] = None,
          gamma: float = 0.7, tol: float = 1e-5, max_iter: int = 100,
          seed: int = 0, variant: str = "F", storage: str = "f64",
          schedule: Optional[Sequence[float]] = None) -> Result:
    """Robust Tensor CUR (Algorithm 1).  variant "F" keeps the first sample,
    "R" resamples before every iteration after the first (Section 3.4).

    storage "f64" is the algorithm as stated.  storage "bf16" (variant F
    only) emulates bfloat16 storage of the sampled blocks, the precision in
    which the mixed-precision mode takes its decisions: while e^(k) >
    max(tol, BF16_SWITCH), X on the blocks and every C = X - S are held
    rounded to bfloat16 (the denominator of e^(k) from the rounded X); once
    e^(k) <= max(tol, BF16_SWITCH) the loop continues (if e^(k) > tol) with
    the unrounded X, its denominator and unrounded C.  All arithmetic stays
    float64; the returned XB is the unrounded X.

    schedule (multipliers c_1..c_n of zeta_0) replaces equation 12's decay
    for the first n thresholds: zeta_k = zeta_0 c_k for k <= n, then
    zeta_k = gamma zeta_(k-1) (repeated multiplication) beyond; None is the
    geometric schedule zeta_k = gamma zeta_(k-1) throughout.

    Raises OracleError(E_INVAL / E_RANK / E_NONFINITE) on the error paths.
    """
    if schedule is not None and (len(schedule) < 1 or
                                 not all(math.isfinite(c) and c > 0 for c in schedule)):
        raise OracleError(E_INVAL, "schedule multipliers must be positive and finite")
    if storage not in ("f64", "bf16") or (storage == "bf16" and variant != "F"):
        raise OracleError(E_INVAL, "storage must be f64, or bf16 with variant F")
    X = np.asarray(X, dtype=np.float64)
    n = X.ndim
    dims = X.shape
    _validate(dims, ranks, I_sizes, J_sizes, gamma, tol, max_iter, variant)

    if zeta0 is None or zeta0 <= 0:
        zeta0 = float(np.max(np.abs(X)))
        if not math.isfinite(zeta0):
            raise OracleError(E_NONFINITE, "X has non-finite entries")

    samp = draw_sample(seed, 0, dims, I_sizes, J_sizes)
    XB = _checked_gather(X, samp)
    XB_exact = XB
    low = storage == "bf16"            # blocks held at bfloat16 precision
    if low:
        XB = [round_bf16(b) for b in XB]
    den = sum(fro(b) for b in XB)
    zero = [np.zeros_like(b) for b in XB]
    if den == 0.0:
        return Result(OK, 0, [], [], zeta0, den, samp, XB_exact, [b.copy() for b in XB],
                      zero, zero, None, dims)

    LB = [np.zeros_like(b) for b in XB]
    CB = [b.copy() for b in XB]
    SB = [np.zeros_like(b) for b in XB]
    DB: List[np.ndarray] = []
    f = None
    zeta = float(zeta0)
    k = 0
    e = 1.0
    min_ratio = 1.0
    e_hist: List[float] = []
    z_hist: List[float] = []
    while e > tol and k < max_iter:
        if variant == "R" and k >= 1:
            samp = draw_sample(seed, k, dims, I_sizes, J_sizes)
            XB = XB_exact = _checked_gather(X, samp)
            den = sum(fro(b) for b in XB)
            LB = evaluate(f, samp)
        if schedule is not None and k < len(schedule):
            zeta = float(zeta0) * float(schedule[k])
        else:
            zeta = gamma * zeta
        # Step (I): partial S-update on the blocks (equations 11 and 13)
        DB = [XB[b] - LB[b] for b in range(n + 1)]
        SB = [hard_threshold(DB[b], zeta) for b in range(n + 1)]
        CB = [XB[b] - SB[b] for b in range(n + 1)]
        if low:
            CB = [round_bf16(c) for c in CB]
        # Step (II): Fiber CUR L-update (equations 8 and 9)
        f = l_update(CB, samp, ranks)
        min_ratio = min([min_ratio] + [float(sg[-1] / sg[0]) for sg in f.sig])
        LB = evaluate(f, samp)
        k += 1
        # Stopping rule (equation 14): E = X - L - S = C - L on the blocks
        e = sum(fro(CB[b] - LB[b]) for b in range(n + 1)) / den
        if not math.isfinite(e):
            raise OracleError(E_NONFINITE, "non-finite relative error")
        e_hist.append(e)
        z_hist.append(zeta)
        if low and e <= max(tol, BF16_SWITCH):
            # the remaining iterations (if any) at full precision
            low = False
            XB = XB_exact
            den = sum(fro(b) for b in XB)
    status = OK if e <= tol else NOT_CONVERGED
    return Result(status, k, e_hist, z_hist, float(zeta0), den, samp, XB_exact, CB,
                  SB, LB, f, dims, min_ratio, DB)


def outliers(res: Result, X: np.ndarray, zeta: Optional[float] = None):
    """Full-grid outliers: the S-update of equation 11 applied to every entry
    of X, S = HT_zeta(X - L) with the strict threshold of equation 10 and
    L = res.reconstruct().  zeta None (or <= 0): the returned iterate's
    threshold zeta_K, zeta_0 when no iteration ran.  Returns (S, L)."""
    X = np.asarray(X, dtype=np.float64)
    L = res.reconstruct()
    if zeta is None or zeta <= 0:
        zeta = res.zeta_hist[-1] if res.iters > 0 else res.zeta0
    return hard_threshold(X - L, zeta), L


def _checked_gather(X, samp):
    XB = gather_blocks(X, samp)
    for b in XB:
        if not np.all(np.isfinite(b)):
            raise OracleError(E_NONFINITE, "X has non-finite sampled entries")
    return XB


def _validate(dims, ranks, I_sizes, J_sizes, gamma, tol, max_iter, variant):
    n = len(dims)
    bad = []
    if n < 2:
        bad.append("need at least 2 modes")
    if len(ranks) != n or len(I_sizes) != n:
        bad.append("ranks / I_sizes length")
    if J_sizes is not None and len(J_sizes) != n:
        bad.append("J_sizes length")
    if not bad:
        for i in range(n):
            r, s, d = int(ranks[i]), int(I_sizes[i]), int(dims[i])
            if not (1 <= r <= s <= d):
                bad.append(f"mode {i}: need 1 <= r <= |I| <= d")
            P = 1
            for j in range(n):
                if j != i:
                    P *= int(dims[j])
            if J_sizes is None:
                m = 1
                for j in range(n):
                    if j != i:
                        m *= int(I_sizes[j])
            else:
                m = int(J_sizes[i])
            if not (1 <= m <= P) or m < r:
                bad.append(f"mode {i}: need r <= |J| <= prod of other dims")
    if not (0.0 < gamma < 1.0):
        bad.append("gamma must lie in (0, 1)")
    if not (tol >= 0.0):
        bad.append("tol must be >= 0")
    if max_iter < 1:
        bad.append("max_iter must be >= 1")
    if variant not in ("F", "R"):
        bad.append("variant must be F or R")
    if bad:
        raise OracleError(E_INVAL, "; ".join(bad))
