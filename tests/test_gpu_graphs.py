"""Replayed iteration graphs (RTCUR-F's steady-state iteration pairs captured
once and replayed, with the iteration index kept on the device) against the
same solve launched kernel by kernel (profiling on, which turns the graphs
off): every result equal bit for bit, for float64, float32 and the
bfloat16-then-float32 mode, over several solves on one handle (the cached
graph replayed across solves, and captured again after a schedule change and
for new sizes)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(rt, h, n):
    e, z = rt.get_history(h)
    blocks = [rt.get_block(h, b, w) for b in range(n + 1)
              for w in (rt.BLOCK_C, rt.BLOCK_L, rt.BLOCK_SUPPORT)]
    core, B = rt.get_tucker(h)
    return e, z, blocks, core, B


def _assert_same(a, b, label):
    ea, za, ba, ca, Ba = a
    eb, zb, bb, cb, Bb = b
    assert np.array_equal(ea, eb), f"{label}: e history"
    assert np.array_equal(za, zb), f"{label}: zeta history"
    for q, (x, y) in enumerate(zip(ba, bb)):
        assert np.array_equal(x, y), f"{label}: block item {q}"
    assert np.array_equal(ca, cb), f"{label}: core"
    for x, y in zip(Ba, Bb):
        assert np.array_equal(x, y), f"{label}: factor"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_graph_replays_equal_direct_launches(dtype):
    import paper_2108_10448_amd as rt
    cases = [synth.tucker_plus_sparse((60, 56, 50), (3, 3, 3), alpha=0.2, seed=41),
             synth.tucker_plus_sparse((48, 40, 44), (4, 2, 3), alpha=0.15, seed=42)]
    hg = rt.create(0, variant="F", dtype=dtype)
    hd = rt.create(0, variant="F", dtype=dtype)
    rt.set_graphs(hg, True)
    rt.set_graphs(hd, True)
    rt.set_profiling(hd, True)   # (which turns the graphs off)
    # the first case twice (the graph replayed from the cache), then with a
    # schedule, then the second case (new sizes)
    runs = [(0, None), (0, None), (0, [0.8, 0.6, 0.5, 0.3]), (1, None)]
    for q, (ci, sched) in enumerate(runs):
        inst = cases[ci]
        I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
        X = torch.from_numpy(inst.X).to("cuda:0")
        for h in (hg, hd):
            rt.set_schedule(h, sched)
        ig = rt.solve(hg, X, inst.ranks, I, tol=1e-5, max_iter=60)
        idr = rt.solve(hd, X, inst.ranks, I, tol=1e-5, max_iter=60)
        label = f"{dtype} run {q}"
        print(f"[graphs] {label}: iters {ig.iters} / {idr.iters}", flush=True)
        assert ig.iters == idr.iters and ig.iters >= 6, label
        assert ig.err == idr.err and ig.converged == idr.converged, label
        _assert_same(_state(rt, hg, 3), _state(rt, hd, 3), label)
    rt.destroy(hg)
    rt.destroy(hd)
