"""Python binding of librtcur, Robust Tensor CUR (RTCUR) on one gfx950 GPU.

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  The functions
mirror the C ABI in include/rtcur.h:

    create(device=0, stream=None, variant="F", dtype=torch.float64) -> Handle
        (dtype torch.bfloat16: bfloat16 blocks, then the FP32 refinement sweep)
    solve(handle, X, ranks, I_sizes=None, J_sizes=None, ...) -> Info
    solve_batch(handles, Xs, ranks, I_sizes=None, ...) -> (infos, Ls)
    reconstruct(handle, out=None, dtype=None) -> torch.Tensor
    reconstruct_noalloc(handle, out) -> out   (static device scratch only)
    outliers(handle, X, zeta=None, with_L=False) -> S or (S, L)
    destroy(handle)
    get_indices / get_history / get_block / get_tucker / sample
    set_profiling / get_profile
    unroll_plan(dims, ranks, I_sizes, K, seed) -> UnrollPlan (see unrolled.py:
        the differentiable K-iteration RTCUR-F behind torch.autograd)

The library must have been built (``python -m paper_2108_10448_amd.build``);
importing the binding never falls back to anything else.
"""

from __future__ import annotations

import ctypes
import math
import os
import warnings
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtcur.so")

OK, NOT_CONVERGED = 0, 1
E_INVAL, E_NOMEM, E_HIP, E_RANK, E_NONFINITE, E_STATE = -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
FIXED, RESAMPLE = 0, 1
BLOCK_X, BLOCK_C, BLOCK_L, BLOCK_SUPPORT = 0, 1, 2, 3

SYMBOLS = ["rtcur_create", "rtcur_solve", "rtcur_reconstruct", "rtcur_outliers",
           "rtcur_destroy",
           "rtcur_get_indices", "rtcur_get_history", "rtcur_get_block",
           "rtcur_get_tucker", "rtcur_sample", "rtcur_set_profiling",
           "rtcur_get_profile", "rtcur_strerror", "rtcur_last_error", "rtcur_solve_batch",
           "rtcur_reconstruct_noalloc", "rtcur_set_schedule", "rtcur_unroll_create", "rtcur_unroll_blocks",
           "rtcur_unroll_forward", "rtcur_unroll_backward", "rtcur_unroll_destroy",
           "rtcur_unroll_last_error", "rtcur_autotune", "rtcur_autotune_clear",
           "rtcur_set_tiles", "rtcur_set_graphs"]


class RtcurInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("err", ctypes.c_double), ("zeta", ctypes.c_double),
                ("zeta0", ctypes.c_double), ("eig_steps", ctypes.c_int32),
                ("status", ctypes.c_int32), ("eig_unconverged", ctypes.c_int32),
                ("solve_ms", ctypes.c_double), ("batch_slot", ctypes.c_int32),
                ("batch_seq", ctypes.c_int32)]


class RTCURError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load librtcur.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run "
                           "`python -m paper_2108_10448_amd.build`")
    # torch first: its HIP runtime is the one both sides must share (the
    # library resolves libamdhip64 against what is already loaded)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_uint64, ctypes.c_double)
    p64 = ctypes.POINTER(ctypes.c_int64)
    pd = ctypes.POINTER(ctypes.c_double)
    L.rtcur_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_int,
                               ctypes.c_int]
    L.rtcur_solve.argtypes = [vp, vp, ctypes.c_int, i32, p64,
                              ctypes.POINTER(ctypes.c_int32), p64, p64, dbl, dbl,
                              dbl, i32, u64, ctypes.POINTER(RtcurInfo)]
    L.rtcur_reconstruct.argtypes = [vp, vp, ctypes.c_int]
    L.rtcur_reconstruct_noalloc.argtypes = [vp, vp, ctypes.c_int]
    L.rtcur_set_schedule.argtypes = [vp, pd, i32]
    L.rtcur_autotune.argtypes = [vp, vp, ctypes.c_int, i32, p64, ctypes.POINTER(ctypes.c_int32),
                                 p64, p64, i32, i32, u64, ctypes.POINTER(ctypes.c_int32), pd, pd]
    L.rtcur_autotune_clear.argtypes = []
    L.rtcur_set_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.rtcur_set_graphs.argtypes = [vp, i32]
    L.rtcur_solve_batch.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp),
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_int32), p64,
                                    ctypes.POINTER(ctypes.c_int32), p64, p64, pd, dbl, dbl,
                                    i32, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(vp),
                                    ctypes.c_int, ctypes.POINTER(RtcurInfo),
                                    ctypes.POINTER(ctypes.c_int32)]
    L.rtcur_outliers.argtypes = [vp, vp, ctypes.c_int, dbl, vp, vp, ctypes.c_int]
    L.rtcur_destroy.argtypes = [vp]
    L.rtcur_get_indices.argtypes = [vp, i32, i32, p64, i64, p64]
    L.rtcur_get_history.argtypes = [vp, pd, pd, i32, ctypes.POINTER(ctypes.c_int32)]
    L.rtcur_get_block.argtypes = [vp, i32, i32, pd, i64, p64]
    L.rtcur_get_tucker.argtypes = [vp, pd, ctypes.POINTER(pd)]
    L.rtcur_sample.argtypes = [u64, i64, i32, p64, p64, p64, i32, i32, p64, i64, p64]
    L.rtcur_set_profiling.argtypes = [vp, i32]
    L.rtcur_get_profile.argtypes = [vp, i32, ctypes.c_char_p, i32, pd,
                                    ctypes.POINTER(ctypes.c_int64)]
    L.rtcur_unroll_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, i32, p64,
                                      ctypes.POINTER(ctypes.c_int32), p64, i32, u64]
    L.rtcur_unroll_blocks.argtypes = [vp, p64, p64, i64]
    L.rtcur_unroll_forward.argtypes = [vp, vp, ctypes.c_int, pd, dbl, vp]
    L.rtcur_unroll_backward.argtypes = [vp, vp, pd, vp]
    L.rtcur_unroll_destroy.argtypes = [vp]
    L.rtcur_unroll_last_error.argtypes = [vp]
    L.rtcur_unroll_last_error.restype = ctypes.c_char_p
    L.rtcur_strerror.argtypes = [ctypes.c_int]
    L.rtcur_strerror.restype = ctypes.c_char_p
    L.rtcur_last_error.argtypes = [vp]
    L.rtcur_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name not in ("rtcur_strerror", "rtcur_last_error", "rtcur_unroll_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().rtcur_strerror(status).decode()


def _i64(seq) -> ctypes.Array:
    return (ctypes.c_int64 * len(seq))(*[int(v) for v in seq])


def default_sizes(dims: Sequence[int], ranks: Sequence[int], upsilon: float = 3.0,
                  fiber: bool = False):
    """|I_i| = ceil(upsilon r_i ln d_i) (the sample-size rule of Section 4),
    clamped to d_i; with fiber=True also |J_i| = ceil(upsilon r_i ln prod d_j)."""
    I = [min(int(d), int(math.ceil(upsilon * r * math.log(d)))) for d, r in zip(dims, ranks)]
    if not fiber:
        return I, None
    J = []
    for i, r in enumerate(ranks):
        P = 1
        for j, d in enumerate(dims):
            if j != i:
                P *= int(d)
        J.append(min(P, int(math.ceil(upsilon * r * math.log(P)))))
    return I, J


def sample(seed: int, t: int, dims, I_sizes, J_sizes, mode: int, which: int) -> np.ndarray:
    """The library's own sampler (host only): I_mode (which=0) or J_mode
    column numbers (which=1) for resample counter t."""
    L = lib()
    n = len(dims)
    ln = ctypes.c_int64(0)
    Jarr = _i64(J_sizes) if J_sizes is not None else None
    rc = L.rtcur_sample(seed, t, n, _i64(dims), _i64(I_sizes), Jarr, mode, which,
                        None, 0, ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, strerror(rc))
    out = np.zeros(ln.value, dtype=np.int64)
    rc = L.rtcur_sample(seed, t, n, _i64(dims), _i64(I_sizes), Jarr, mode, which,
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ln.value,
                        ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, strerror(rc))
    return out


@dataclass
class Info:
    status: int
    iters: int
    converged: bool
    err: float
    zeta: float
    zeta0: float
    eig_steps: int
    eig_unconverged: int = 0
    solve_ms: float = 0.0      # host wall-clock time of the solve
    batch_slot: int = -1       # batch: index of the handle that solved it
    batch_seq: int = -1        # batch: position in that handle's sequence


def _info(rc, c) -> "Info":
    return Info(rc, c.iters, bool(c.converged), c.err, c.zeta, c.zeta0, c.eig_steps,
                c.eig_unconverged, c.solve_ms, c.batch_slot, c.batch_seq)


class Handle:
    """Owns an rtcur_t; closes it on destroy() or garbage collection."""

    def __init__(self, ptr, device, variant, dtype, stream=None):
        self.ptr = ptr
        self.device = device
        self.variant = variant
        self.dtype = dtype
        self.stream = stream   # the torch stream the library launches on
        self.dims = None
        self.ranks = None

    def __del__(self):
        try:
            destroy(self)
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().rtcur_last_error(self.ptr).decode() if self.ptr else ""


def _torch():
    import torch
    return torch


def create(device: int = 0, stream=None, variant: str = "F", dtype=None) -> Handle:
    """rtcur_create on `device`, bound to `stream` (a torch stream or a raw
    hipStream_t; default: torch's current stream of that device).  variant
    "F" (fixed samples) or "R" (resample).  Every call on the handle first
    makes its stream wait for the work queued so far on torch's current
    stream (which produced X and last used the output buffers)."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    cdt = F64 if dtype == torch.float64 else (BF16 if dtype == torch.bfloat16 else F32)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    elif not hasattr(stream, "cuda_stream"):
        stream = torch.cuda.ExternalStream(int(stream), device=f"cuda:{device}")
    sptr = ctypes.c_void_p(stream.cuda_stream)
    out = ctypes.c_void_p()
    rc = lib().rtcur_create(ctypes.byref(out), device, sptr,
                            FIXED if variant == "F" else RESAMPLE, cdt)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_create: {strerror(rc)}")
    return Handle(out, device, variant, dtype, stream)


def _order(h: Handle) -> None:
    """The handle's stream waits for everything queued so far on torch's
    current stream of its device: the producer of X, and the last users of
    any output buffer the caching allocator hands out on that stream.  The
    library's calls return after their own device work has finished, so
    the results need no ordering the other way."""
    torch = _torch()
    cur = torch.cuda.current_stream(h.device)
    if h.stream is not None and h.stream.cuda_stream != cur.cuda_stream:
        h.stream.wait_stream(cur)


def destroy(h: Handle) -> None:
    if h is not None and h.ptr:
        lib().rtcur_destroy(h.ptr)
        h.ptr = None


def solve(h: Handle, X, ranks: Sequence[int], I_sizes: Optional[Sequence[int]] = None,
          J_sizes: Optional[Sequence[int]] = None, *, upsilon: float = 3.0,
          zeta0: Optional[float] = None, gamma: float = 0.7, tol: float = 1e-5,
          max_iter: int = 100, seed: int = 0, check: bool = True) -> Info:
    """rtcur_solve on the device tensor X (float32/float64, C-contiguous)."""
    torch = _torch()
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise TypeError("X must be a device torch.Tensor")
    if X.dtype not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    if not X.is_contiguous():
        raise ValueError("X must be C-contiguous")
    dims = list(X.shape)
    if I_sizes is None:
        I_sizes, _ = default_sizes(dims, ranks, upsilon)
    info = RtcurInfo()
    r32 = (ctypes.c_int32 * len(ranks))(*[int(r) for r in ranks])
    _order(h)
    rc = lib().rtcur_solve(h.ptr, ctypes.c_void_p(X.data_ptr()),
                           F64 if X.dtype == torch.float64 else F32, len(dims),
                           _i64(dims), r32, _i64(I_sizes),
                           _i64(J_sizes) if J_sizes is not None else None,
                           float(zeta0) if zeta0 else 0.0, float(gamma), float(tol),
                           int(max_iter), int(seed) & ((1 << 64) - 1),
                           ctypes.byref(info))
    h.dims, h.ranks = dims, list(ranks)
    if rc < 0 and check:
        raise RTCURError(rc, f"rtcur_solve: {strerror(rc)}: {h.last_error()}")
    if rc == NOT_CONVERGED and check:
        warnings.warn(f"RTCUR did not reach tol in {max_iter} iterations (e={info.err:.3e})")
    return _info(rc, info)


def set_schedule(h: Handle, multipliers=None) -> None:
    """rtcur_set_schedule: thresholds zeta_k = multipliers[k-1] zeta_0 for
    the first len(multipliers) iterations of the following solves, then the
    decay by gamma; None (or empty) restores the geometric schedule."""
    c = np.ascontiguousarray(np.asarray([] if multipliers is None else multipliers,
                                        dtype=np.float64).reshape(-1))
    rc = lib().rtcur_set_schedule(h.ptr, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                  if c.size else None, int(c.size))
    if rc != OK:
        raise RTCURError(rc, f"rtcur_set_schedule: {strerror(rc)}: {h.last_error()}")


def autotune(h: Handle, X, ranks: Sequence[int], I_sizes: Optional[Sequence[int]] = None,
             J_sizes: Optional[Sequence[int]] = None, *, upsilon: float = 3.0, iters: int = 4,
             reps: int = 2, seed: int = 0) -> dict:
    """rtcur_autotune: times tile shapes on this problem and records the
    fastest in the library's process-wide table for its sizes.  Returns
    {"ht_rows", "gram_chunk", "bfac_sub", "tuned_ms", "default_ms"}."""
    torch = _torch()
    if not isinstance(X, torch.Tensor) or not X.is_cuda or not X.is_contiguous():
        raise TypeError("X must be a C-contiguous device torch.Tensor")
    if X.dtype not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    dims = list(X.shape)
    if I_sizes is None:
        I_sizes, _ = default_sizes(dims, ranks, upsilon)
    r32 = (ctypes.c_int32 * len(ranks))(*[int(r) for r in ranks])
    tile = (ctypes.c_int32 * 3)()
    tms, dms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _order(h)
    rc = lib().rtcur_autotune(h.ptr, ctypes.c_void_p(X.data_ptr()),
                              F64 if X.dtype == torch.float64 else F32, len(dims), _i64(dims),
                              r32, _i64(I_sizes),
                              _i64(J_sizes) if J_sizes is not None else None, int(iters),
                              int(reps), int(seed) & ((1 << 64) - 1), tile, ctypes.byref(tms),
                              ctypes.byref(dms))
    h.dims, h.ranks = dims, list(ranks)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_autotune: {strerror(rc)}: {h.last_error()}")
    return {"ht_rows": tile[0], "gram_chunk": tile[1], "bfac_sub": tile[2],
            "tuned_ms": tms.value, "default_ms": dms.value}


def set_tiles(h: Handle, tile=None) -> None:
    """rtcur_set_tiles: (rows per threshold tile, Gram chunk columns, B
    sub-chunks) for this handle's solves; None: back to the tuned table."""
    if tile is None:
        rc = lib().rtcur_set_tiles(h.ptr, None)
    else:
        t = (ctypes.c_int32 * 3)(*[int(v) for v in tile])
        rc = lib().rtcur_set_tiles(h.ptr, t)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_set_tiles: {strerror(rc)}: {h.last_error()}")


def set_graphs(h: Handle, enable: bool) -> None:
    """rtcur_set_graphs: RTCUR-F steady-state iteration pairs as replayed
    HIP graphs (bit-for-bit the same results; off by default)."""
    rc = lib().rtcur_set_graphs(h.ptr, 1 if enable else 0)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_set_graphs: {strerror(rc)}")


def autotune_clear() -> None:
    """rtcur_autotune_clear: every later solve uses the built-in tile rule."""
    lib().rtcur_autotune_clear()


def solve_batch(handles: Sequence[Handle], Xs, ranks, I_sizes=None, J_sizes=None, *,
                upsilon: float = 3.0, zeta0=None, gamma: float = 0.7, tol: float = 1e-5,
                max_iter: int = 100, seeds=None, with_L: bool = False, L_dtype=None,
                check: bool = True):
    """rtcur_solve_batch: instance j is device tensor Xs[j] with ranks[j],
    I_sizes[j] (default upsilon sizes) and J_sizes[j] (or chidori); one host
    thread per handle, each taking the next instance (largest first) from one
    work queue; Info.batch_slot / batch_seq say which handle solved it, when.
    All Xs share one dtype.  Returns (infos, Ls) with Ls the full
    reconstructions when with_L, else None."""
    torch = _torch()
    count = len(Xs)
    if count == 0:
        return [], ([] if with_L else None)
    if len(ranks) != count:
        raise ValueError("one rank tuple per instance")
    dt = Xs[0].dtype
    for X in Xs:
        if not isinstance(X, torch.Tensor) or not X.is_cuda or not X.is_contiguous():
            raise TypeError("every X must be a C-contiguous device torch.Tensor")
        if X.dtype != dt or dt not in (torch.float32, torch.float64):
            raise TypeError("every X must have the same float32/float64 dtype")
    K = 4
    dims = (ctypes.c_int64 * (K * count))()
    rk = (ctypes.c_int32 * (K * count))()
    Is = (ctypes.c_int64 * (K * count))()
    Js = (ctypes.c_int64 * (K * count))() if J_sizes is not None else None
    nn = (ctypes.c_int32 * count)()
    for j, X in enumerate(Xs):
        d = list(X.shape)
        nn[j] = len(d)
        Ij = I_sizes[j] if I_sizes is not None else default_sizes(d, ranks[j], upsilon)[0]
        for q in range(len(d)):
            dims[K * j + q] = d[q]
            rk[K * j + q] = int(ranks[j][q])
            Is[K * j + q] = int(Ij[q])
            if Js is not None:
                Js[K * j + q] = int(J_sizes[j][q])
    xs = (ctypes.c_void_p * count)(*[X.data_ptr() for X in Xs])
    z0 = (ctypes.c_double * count)(*[float(z) if z else 0.0 for z in zeta0]) \
        if zeta0 is not None else None
    sd = (ctypes.c_uint64 * count)(*[int(s) & ((1 << 64) - 1) for s in
                                     (seeds if seeds is not None else range(count))])
    Ls = None
    lo = None
    odt = L_dtype or dt
    if odt not in (torch.float32, torch.float64):
        raise TypeError("L_dtype must be float32 or float64")
    if with_L:
        Ls = [torch.empty(X.shape, dtype=odt, device=X.device) for X in Xs]
        lo = (ctypes.c_void_p * count)(*[L.data_ptr() for L in Ls])
    hs = (ctypes.c_void_p * len(handles))(*[h.ptr for h in handles])
    for h in handles:
        _order(h)
    infos = (RtcurInfo * count)()
    st = (ctypes.c_int32 * count)()
    rc = lib().rtcur_solve_batch(hs, len(handles), count, xs,
                                 F64 if dt == torch.float64 else F32, nn, dims, rk, Is, Js,
                                 z0, float(gamma), float(tol), int(max_iter), sd, lo,
                                 F64 if odt == torch.float64 else F32, infos, st)
    last = {}
    for j in range(count):
        t = infos[j].batch_slot
        if 0 <= t < len(handles) and infos[j].batch_seq >= last.get(t, (-1, -1))[0]:
            last[t] = (infos[j].batch_seq, j)
    for t, (_, j) in last.items():
        handles[t].dims, handles[t].ranks = list(Xs[j].shape), list(ranks[j])
    if rc < 0 and check:
        raise RTCURError(rc, f"rtcur_solve_batch: {strerror(rc)}")
    out = [_info(st[j], infos[j]) for j in range(count)]
    return out, Ls


def _out_dtype(h: Handle):
    """Default output dtype: the handle's, float32 for a bfloat16 handle."""
    torch = _torch()
    return torch.float32 if h.dtype == torch.bfloat16 else h.dtype


def reconstruct(h: Handle, out=None, dtype=None):
    """rtcur_reconstruct: the full L into `out` (allocated if None)."""
    torch = _torch()
    if out is None:
        out = torch.empty(h.dims, dtype=dtype or _out_dtype(h), device=f"cuda:{h.device}")
    if out.dtype not in (torch.float32, torch.float64) or not out.is_contiguous():
        raise TypeError("out must be a C-contiguous float32/float64 tensor")
    _order(h)
    rc = lib().rtcur_reconstruct(h.ptr, ctypes.c_void_p(out.data_ptr()),
                                 F64 if out.dtype == torch.float64 else F32)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_reconstruct: {strerror(rc)}: {h.last_error()}")
    return out


def reconstruct_noalloc(h: Handle, out):
    """rtcur_reconstruct_noalloc: the full L into the caller's `out` with the
    library's static device scratch (no device allocation in the library);
    queued on the handle's stream, which torch's current stream is then made
    to wait for."""
    torch = _torch()
    if not isinstance(out, torch.Tensor) or not out.is_cuda or not out.is_contiguous():
        raise TypeError("out must be a C-contiguous device tensor")
    if out.dtype not in (torch.float32, torch.float64):
        raise TypeError("out must be float32 or float64")
    if list(out.shape) != list(h.dims):
        raise ValueError(f"out has shape {tuple(out.shape)}, the solve had {tuple(h.dims)}")
    _order(h)
    rc = lib().rtcur_reconstruct_noalloc(h.ptr, ctypes.c_void_p(out.data_ptr()),
                                         F64 if out.dtype == torch.float64 else F32)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_reconstruct_noalloc: {strerror(rc)}: {h.last_error()}")
    cur = torch.cuda.current_stream(h.device)
    if h.stream is not None and h.stream.cuda_stream != cur.cuda_stream:
        cur.wait_stream(h.stream)
    return out


def outliers(h: Handle, X, zeta: Optional[float] = None, *, with_L: bool = False,
             dtype=None):
    """rtcur_outliers: S = HT_zeta(X - L) over the whole tensor (zeta None:
    the returned iterate's threshold), and L too when with_L; X is the
    solved device tensor.  Returns S, or (S, L)."""
    torch = _torch()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.is_contiguous()):
        raise TypeError("X must be a C-contiguous device torch.Tensor")
    if X.dtype not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    if tuple(X.shape) != tuple(h.dims):
        raise ValueError(f"X has shape {tuple(X.shape)}, the solve had {tuple(h.dims)}")
    odt = dtype or _out_dtype(h)
    if odt not in (torch.float32, torch.float64):
        raise TypeError("output dtype must be float32 or float64")
    S = torch.empty(h.dims, dtype=odt, device=X.device)
    L_ = torch.empty(h.dims, dtype=odt, device=X.device) if with_L else None
    _order(h)
    rc = lib().rtcur_outliers(h.ptr, ctypes.c_void_p(X.data_ptr()),
                              F64 if X.dtype == torch.float64 else F32,
                              float(zeta) if zeta is not None else 0.0,
                              ctypes.c_void_p(S.data_ptr()),
                              ctypes.c_void_p(L_.data_ptr()) if with_L else None,
                              F64 if odt == torch.float64 else F32)
    if rc != OK:
        raise RTCURError(rc, f"rtcur_outliers: {strerror(rc)}: {h.last_error()}")
    return (S, L_) if with_L else S


def get_indices(h: Handle, mode: int, which: int) -> np.ndarray:
    L = lib()
    ln = ctypes.c_int64(0)
    rc = L.rtcur_get_indices(h.ptr, mode, which, None, 0, ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, h.last_error())
    out = np.zeros(ln.value, dtype=np.int64)
    L.rtcur_get_indices(h.ptr, mode, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        ln.value, ctypes.byref(ln))
    return out


def get_history(h: Handle):
    L = lib()
    ln = ctypes.c_int32(0)
    rc = L.rtcur_get_history(h.ptr, None, None, 0, ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, h.last_error())
    e = np.zeros(ln.value)
    z = np.zeros(ln.value)
    pd = ctypes.POINTER(ctypes.c_double)
    L.rtcur_get_history(h.ptr, e.ctypes.data_as(pd), z.ctypes.data_as(pd), ln.value,
                        ctypes.byref(ln))
    return e, z


def get_block(h: Handle, block: int, what: int) -> np.ndarray:
    """A sampled block as float64 (block 0 = R with shape (s_1..s_n), block
    1+i = C_i with shape (d_i, m_i))."""
    L = lib()
    ln = ctypes.c_int64(0)
    rc = L.rtcur_get_block(h.ptr, block, what, None, 0, ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, h.last_error())
    out = np.zeros(ln.value)
    rc = L.rtcur_get_block(h.ptr, block, what,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ln.value,
                           ctypes.byref(ln))
    if rc != OK:
        raise RTCURError(rc, h.last_error())
    return out


def get_tucker(h: Handle):
    """(core G of shape ranks, [B_i of shape (d_i, r_i)]) as float64 arrays."""
    L = lib()
    core = np.zeros(h.ranks)
    Bs = [np.zeros((d, r)) for d, r in zip(h.dims, h.ranks)]
    pd = ctypes.POINTER(ctypes.c_double)
    arr = (pd * len(Bs))(*[b.ctypes.data_as(pd) for b in Bs])
    rc = L.rtcur_get_tucker(h.ptr, core.ctypes.data_as(pd), arr)
    if rc != OK:
        raise RTCURError(rc, h.last_error())
    return core, Bs


PROFILE_KINDS = ("absmax", "gather", "ht", "gram", "eig", "zcore", "bfac", "bred", "hexp",
                 "decide")


def set_profiling(h: Handle, enable: bool, kinds=None) -> None:
    """rtcur_set_profiling: HIP-event timing of the launches of `kinds`
    (names from PROFILE_KINDS; None: every kernel)."""
    if not enable:
        mask = 0
    elif kinds is None:
        mask = -1
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << PROFILE_KINDS.index(k)
    rc = lib().rtcur_set_profiling(h.ptr, mask)
    if rc != OK:
        raise RTCURError(rc, h.last_error())


def get_profile(h: Handle) -> dict:
    """{kernel name: (total ms, launches)} accumulated while profiling."""
    L = lib()
    out = {}
    kind = 0
    while True:
        name = ctypes.create_string_buffer(64)
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        if L.rtcur_get_profile(h.ptr, kind, name, 64, ctypes.byref(ms), ctypes.byref(cnt)) != OK:
            break
        out[name.value.decode()] = (ms.value, cnt.value)
        kind += 1
    return out


class UnrollPlan:
    """An rtcur_unroll_t: the sample, workspace and checkpoints of one
    differentiable unrolled RTCUR-F pass (float64, three modes)."""

    def __init__(self, ptr, device, dims, ranks, I_sizes, K, seed, stream):
        self.ptr = ptr
        self.device = device
        self.dims = list(dims)
        self.ranks = list(ranks)
        self.I_sizes = list(I_sizes)
        self.K = K
        self.seed = seed
        self.stream = stream
        self.generation = 0     # forward passes run so far (backward checks it)
        n = ctypes.c_int64(0)
        rc = lib().rtcur_unroll_blocks(ptr, ctypes.byref(n), None, 0)
        if rc != OK:
            raise RTCURError(rc, "rtcur_unroll_blocks")
        self.n_blk = n.value

    def last_error(self) -> str:
        return lib().rtcur_unroll_last_error(self.ptr).decode() if self.ptr else ""

    def block_index(self) -> np.ndarray:
        """Offset in X of every block entry, in block-buffer order."""
        out = np.zeros(self.n_blk, dtype=np.int64)
        rc = lib().rtcur_unroll_blocks(self.ptr, None,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       self.n_blk)
        if rc != OK:
            raise RTCURError(rc, self.last_error())
        return out

    def close(self):
        if self.ptr:
            lib().rtcur_unroll_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unroll_plan(dims, ranks, I_sizes=None, K=15, seed=0, device=0, stream=None,
                upsilon=3.0) -> UnrollPlan:
    """rtcur_unroll_create on `device` (stream: torch's current by default)."""
    torch = _torch()
    if I_sizes is None:
        I_sizes, _ = default_sizes(dims, ranks, upsilon)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    out = ctypes.c_void_p()
    r32 = (ctypes.c_int32 * len(ranks))(*[int(r) for r in ranks])
    rc = lib().rtcur_unroll_create(ctypes.byref(out), device, ctypes.c_void_p(stream.cuda_stream),
                                   len(dims), _i64(dims), r32, _i64(I_sizes), int(K),
                                   int(seed) & ((1 << 64) - 1))
    if rc != OK:
        raise RTCURError(rc, f"rtcur_unroll_create: {strerror(rc)}")
    return UnrollPlan(out, device, dims, ranks, I_sizes, K, seed, stream)


def unroll_forward(plan: UnrollPlan, X, zetas, tau: float, L_out=None):
    """rtcur_unroll_forward: L^K on the blocks (float64 device tensor of
    plan.n_blk entries); zetas: K thresholds (any sequence / tensor)."""
    torch = _torch()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.is_contiguous()):
        raise TypeError("X must be a C-contiguous device tensor")
    if X.dtype not in (torch.float32, torch.float64) or list(X.shape) != plan.dims:
        raise TypeError("X must be float32/float64 with the planned dims")
    z = np.ascontiguousarray(np.asarray(
        zetas.detach().cpu().numpy() if isinstance(zetas, torch.Tensor) else zetas,
        dtype=np.float64).reshape(-1))
    if z.size != plan.K:
        raise ValueError(f"need {plan.K} thresholds, got {z.size}")
    if L_out is None:
        L_out = torch.empty(plan.n_blk, dtype=torch.float64, device=X.device)
    cur = torch.cuda.current_stream(plan.device)
    if plan.stream.cuda_stream != cur.cuda_stream:
        plan.stream.wait_stream(cur)
    rc = lib().rtcur_unroll_forward(plan.ptr, ctypes.c_void_p(X.data_ptr()),
                                    F64 if X.dtype == torch.float64 else F32,
                                    z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    float(tau), ctypes.c_void_p(L_out.data_ptr()))
    if rc != OK:
        raise RTCURError(rc, f"rtcur_unroll_forward: {strerror(rc)}: {plan.last_error()}")
    plan.generation += 1
    return L_out


def unroll_backward(plan: UnrollPlan, L_bar):
    """rtcur_unroll_backward of the plan's last forward: (zeta_bar as a
    float64 numpy array of K, X_bar as a float64 device tensor)."""
    torch = _torch()
    L_bar = L_bar.detach().to(dtype=torch.float64).contiguous()
    if L_bar.numel() != plan.n_blk or not L_bar.is_cuda:
        raise ValueError("L_bar must be a device tensor of n_blk entries")
    zb = np.zeros(plan.K)
    Xb = torch.empty(plan.dims, dtype=torch.float64, device=L_bar.device)
    cur = torch.cuda.current_stream(plan.device)
    if plan.stream.cuda_stream != cur.cuda_stream:
        plan.stream.wait_stream(cur)
    rc = lib().rtcur_unroll_backward(plan.ptr, ctypes.c_void_p(L_bar.data_ptr()),
                                     zb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ctypes.c_void_p(Xb.data_ptr()))
    if rc != OK:
        raise RTCURError(rc, f"rtcur_unroll_backward: {strerror(rc)}: {plan.last_error()}")
    return zb, Xb
