"""rtcur_reconstruct_noalloc (the allocation-free variant of rtcur_reconstruct,
its temporaries in the library's static per-device scratch) against
rtcur_reconstruct through the C ABI: the same L bit for bit, on two calls in
a row where the second solve is smaller, in float64 and float32, for a solve
that did no iteration (L = 0), and the size limit reported before any work."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve(h, inst, iters, dtype):
    import paper_2108_10448_amd as rt
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    X = torch.from_numpy(inst.X.astype(np.float64 if dtype == torch.float64 else np.float32))
    X = X.to("cuda:0")
    info = rt.solve(h, X, inst.ranks, I, tol=0.0, max_iter=iters, check=False)
    assert info.status >= 0, h.last_error()
    return X


def _both(h, dtype):
    """L from rtcur_reconstruct and from rtcur_reconstruct_noalloc (the
    latter into a buffer first filled with NaN, so that every entry must be
    written), each called through the C ABI."""
    import paper_2108_10448_amd as rt
    L = rt.lib()
    code = rt.F64 if dtype == torch.float64 else rt.F32
    ref = torch.empty(h.dims, dtype=dtype, device="cuda:0")
    out = torch.full(h.dims, float("nan"), dtype=dtype, device="cuda:0")
    torch.cuda.synchronize()
    assert L.rtcur_reconstruct(h.ptr, ctypes.c_void_p(ref.data_ptr()), code) == rt.OK
    rc = L.rtcur_reconstruct_noalloc(h.ptr, ctypes.c_void_p(out.data_ptr()), code)
    assert rc == rt.OK, h.last_error()
    torch.cuda.synchronize()   # the entry point only queues its kernels
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_reconstruct_twice(dtype):
    import paper_2108_10448_amd as rt
    dt = torch.float64 if dtype == "f64" else torch.float32
    h = rt.create(0, dtype=dt)
    big = synth.tucker_plus_sparse((64, 56, 48), (4, 3, 5), alpha=0.2, seed=11)
    small = synth.tucker_plus_sparse((30, 26, 22), (2, 3, 2), alpha=0.2, seed=12)
    for inst in (big, small):                 # second call: a smaller input
        print(f"[noalloc] {dtype} dims {inst.dims} ranks {inst.ranks}", flush=True)
        _solve(h, inst, 5, dt)
        ref, out = _both(h, dt)
        assert np.all(np.isfinite(out))
        assert np.array_equal(out, ref), float(np.max(np.abs(out - ref)))
        # and against the library's own Tucker factors (an independent sum)
        core, Bs = rt.get_tucker(h)
        L = np.einsum("abc,xa,yb,zc->xyz", core, *Bs)
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert np.linalg.norm(out - L) <= tol * np.linalg.norm(L)
    rt.destroy(h)


def test_noalloc_four_modes_rank16_then_smaller():
    import paper_2108_10448_amd as rt
    h = rt.create(0, dtype=torch.float32)
    a = synth.tucker_plus_sparse((40, 44, 3, 30), (10, 10, 3, 5), alpha=0.1, seed=2)
    b = synth.tucker_plus_sparse((20, 18, 3, 16), (3, 3, 2, 2), alpha=0.1, seed=3)
    for inst in (a, b):
        print(f"[noalloc] 4-mode dims {inst.dims} ranks {inst.ranks}", flush=True)
        _solve(h, inst, 3, torch.float32)
        ref, out = _both(h, torch.float32)
        assert np.array_equal(out, ref)
    rt.destroy(h)


def test_noalloc_zero_iterations_gives_zero():
    import paper_2108_10448_amd as rt
    h = rt.create(0, dtype=torch.float64)
    inst = synth.tucker_plus_sparse((24, 20, 16), (2, 2, 2), alpha=0.1, seed=4)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    X = torch.from_numpy(inst.X).to("cuda:0")
    info = rt.solve(h, X, inst.ranks, I, tol=1.0, max_iter=5, check=False)
    assert info.iters == 0
    ref, out = _both(h, torch.float64)
    assert np.array_equal(out, np.zeros(inst.dims)) and np.array_equal(ref, out)
    rt.destroy(h)


def test_noalloc_size_limit_and_state():
    import paper_2108_10448_amd as rt
    L = rt.lib()
    h = rt.create(0, dtype=torch.float64)
    dummy = torch.empty(8, dtype=torch.float64, device="cuda:0")
    # no solve yet
    assert L.rtcur_reconstruct_noalloc(h.ptr, ctypes.c_void_p(dummy.data_ptr()),
                                       rt.F64) == rt.E_STATE
    # 4 x 1100 x 1100, rank 2 (RP = 4): the expansion needs 4 * 8 * 1.21e6
    # bytes = 38.7 MB (fits); rank 5 (RP = 8) needs 77 MB (does not)
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.standard_normal((4, 1100, 1100))).to("cuda:0")
    for ranks, fits in (((2, 2, 2), True), ((4, 5, 5), False)):
        print(f"[noalloc] size limit ranks {ranks}", flush=True)
        info = rt.solve(h, X, ranks, [4, 40, 40], tol=0.0, max_iter=1, check=False)
        assert info.status >= 0, h.last_error()
        out = torch.empty(h.dims, dtype=torch.float64, device="cuda:0")
        rc = L.rtcur_reconstruct_noalloc(h.ptr, ctypes.c_void_p(out.data_ptr()), rt.F64)
        if fits:
            assert rc == rt.OK
            torch.cuda.synchronize()
            ref = rt.reconstruct(h)
            assert torch.equal(out, ref)
        else:
            assert rc == rt.E_INVAL and "static scratch" in h.last_error()
    rt.destroy(h)
