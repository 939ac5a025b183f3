"""Tile shapes and the autotuner.

* Every tile shape (rows per threshold tile 8 / 16 / 32, Gram chunk columns,
  B-factor sub-chunks) meets the oracle parity bar on shapes whose block row
  counts are not multiples of the tile height (ragged last tiles), in float64
  and float32 blocks.
* rtcur_autotune returns a valid tile shape no slower than the built-in rule
  (the rule is its first candidate), records it in the process-wide table,
  and a later solve of those sizes on another handle uses it: equal bit for
  bit to a solve with the same tiles set explicitly, and within the parity
  bar of the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import rtcur as oracle_rtcur

from _parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(dims, ranks, seed, storage=np.float64):
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=0.2, seed=seed, storage=storage)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    return inst, I


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tile", [(8, 0, 0), (32, 512, 2), (16, 4096, 4), (32, 256, 8)])
def test_tile_shapes_meet_parity(dtype, tile):
    import paper_2108_10448_amd as rt
    inst, I = _case((70, 61, 45), (3, 4, 2), seed=77)
    K = 6
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, K, 0, "F")
    h = rt.create(0, variant="F", dtype=dtype)
    rt.set_tiles(h, tile)
    X = torch.from_numpy(inst.X).to("cuda:0")
    info = rt.solve(h, X, inst.ranks, I, tol=0.0, max_iter=K, check=False)
    print(f"[tiles] {tile} {dtype} status {info.status} err {info.err:.6e}", flush=True)
    compare(res, h, info, fp64=dtype == torch.float64, label=f"tiles {tile} {dtype}")
    rt.destroy(h)


def test_set_tiles_rejects_bad_shapes():
    import paper_2108_10448_amd as rt
    h = rt.create(0)
    for bad in [(12, 0, 0), (16, 300, 0), (16, 0, -1), (16, 0, 65)]:
        with pytest.raises(rt.RTCURError):
            rt.set_tiles(h, bad)
    rt.set_tiles(h, None)
    rt.destroy(h)


def test_autotune_records_and_is_used():
    import paper_2108_10448_amd as rt
    inst, I = _case((100, 90, 80), (3, 3, 3), seed=5, storage=np.float32)
    X = torch.from_numpy(inst.X).to("cuda:0")
    rt.autotune_clear()
    try:
        ht = rt.create(0, dtype=torch.float32)
        got = rt.autotune(ht, X, inst.ranks, I, iters=4, reps=2)
        print(f"[autotune] {got}", flush=True)
        assert got["ht_rows"] in (8, 16, 32)
        assert got["gram_chunk"] in (0, 512, 1024, 2048, 4096, 8192)
        assert got["bfac_sub"] in (0, 2, 4, 8)
        assert 0 < got["tuned_ms"] <= got["default_ms"]
        # a new handle plans these sizes with the tuned tiles: bit for bit
        # what the same tiles set explicitly give
        ha = rt.create(0, dtype=torch.float32)
        hb = rt.create(0, dtype=torch.float32)
        rt.set_tiles(hb, (got["ht_rows"], got["gram_chunk"], got["bfac_sub"]))
        ia = rt.solve(ha, X, inst.ranks, I, tol=1e-5, check=False)
        ib = rt.solve(hb, X, inst.ranks, I, tol=1e-5, check=False)
        assert ia.iters == ib.iters and ia.err == ib.err
        for b in range(4):
            assert np.array_equal(rt.get_block(ha, b, rt.BLOCK_C), rt.get_block(hb, b, rt.BLOCK_C))
        res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, ia.iters, 0, "F")
        compare(res, ha, ia, fp64=False, label="autotuned float32")
        for h in (ht, ha, hb):
            rt.destroy(h)
    finally:
        rt.autotune_clear()
