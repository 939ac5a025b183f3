"""GPU parity on the workload shapes the benchmark reports: the video-shaped
4-mode recipe run to its tolerance (FP64, FP32 and bfloat16 blocks with the
FP32 refinement sweep), RTCUR-R with FP32 blocks on the 300^3 workload, and
instances of the 64-tensor batch recipe at their real shapes against the
oracle.  Bars as in test_gpu_parity.py."""
import numpy as np
import pytest

import synth
from oracle import rtcur as oracle_rtcur

from _parity import compare, rel, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class _OracleRuns:
    """Oracle runs of one instance for a given number of iterations (tol =
    0), computed once each."""

    def __init__(self, X, ranks, I, variant="F", storage="f64"):
        self.X, self.ranks, self.I, self.variant = X, ranks, I, variant
        self.storage = storage
        self.cache = {}

    def at(self, K):
        if K not in self.cache:
            self.cache[K] = oracle_rtcur(self.X, self.ranks, self.I, None, None, 0.7, 0.0,
                                         K, 0, self.variant, storage=self.storage)
        return self.cache[K]


@pytest.fixture(scope="module")
def video_tol():
    # the video recipe at half the frame side and half the frames (the
    # oracle runs it to tolerance in about 30 s), upsilon = 2
    inst = synth.video_like((120, 160, 3, 200), side=(10, 30), storage=np.float32)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 2.0)
    ref = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    runs = _OracleRuns(inst.X, inst.ranks, I)
    runs.cache[ref.iters] = ref
    return inst, I, ref, runs


def test_video_to_tolerance_fp64(video_tol):
    inst, I, ref, _ = video_tol
    h, info, _ = run_gpu(inst.X, inst.ranks, I, check=False)
    assert info.converged and info.iters == ref.iters
    compare(ref, h, info, label="video 120x160x3x200 to tol fp64")


def test_video_to_tolerance_f32(video_tol):
    import paper_2108_10448_amd as rt
    inst, I, ref, runs = video_tol
    h, info, _ = run_gpu(inst.X, inst.ranks, I, dtype=torch.float32, check=False)
    assert info.converged and abs(info.iters - ref.iters) <= 1
    res = runs.at(info.iters)
    compare(res, h, info, fp64=False, label="video to tol f32")
    L = rt.reconstruct(h)
    assert L.dtype == torch.float32
    assert rel(L.cpu().numpy().astype(np.float64), res.reconstruct()) < 1e-4


def test_video_to_tolerance_bf16(video_tol):
    # bfloat16 blocks until e^(k) <= 1e-2, then the float32 sweep, against
    # the oracle holding its blocks at the same storage precision (the
    # decisions of the bfloat16 phase depend on it); the distance to the
    # plain float64 oracle is reported: on this workload, whose low-rank part
    # does not separate (true error 0.2), the early rounding moves the path
    import paper_2108_10448_amd as rt
    inst, I, ref, _ = video_tol
    h, info, _ = run_gpu(inst.X, inst.ranks, I, dtype=torch.bfloat16, check=False)
    low = _OracleRuns(inst.X, inst.ranks, I, storage="bf16")
    assert info.converged and abs(info.iters - ref.iters) <= 1
    res = low.at(info.iters)
    compare(res, h, info, fp64=False, label="video to tol bf16 (bf16-storage oracle)")
    L = rt.reconstruct(h).cpu().numpy().astype(np.float64)
    assert rel(L, res.reconstruct()) < 1e-4
    full = ref if ref.iters == info.iters else oracle_rtcur(
        inst.X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, "F")
    print(f"[video bf16] L against the float64-storage oracle: "
          f"{rel(L, full.reconstruct()):.3e}", flush=True)


def test_cube300_resample_fp32():
    inst = synth.config_instance("cube300_r5")
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    h, info, _ = run_gpu(inst.X, inst.ranks, I, variant="R", dtype=torch.float32, check=False)
    assert info.converged
    ref = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "R")
    assert abs(info.iters - ref.iters) <= 1
    res = ref if info.iters == ref.iters else oracle_rtcur(
        inst.X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, "R")
    compare(res, h, info, fp64=False, label="cube300 R fp32")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_recipe_against_oracle(dtype):
    # four instances of the 64-tensor batch recipe at their real shapes,
    # solved together for a fixed number of iterations, each against the
    # oracle run on the same float32-stored tensor
    import paper_2108_10448_amd as rt
    specs = [synth.batch_specs()[j] for j in (1, 2, 6, 9)]
    K = 4
    insts, Xs, ranks, I, seeds = [], [], [], [], []
    tdt = torch.float32 if dtype == "f32" else torch.float64
    for sp in specs:
        inst = synth.tucker_plus_sparse(sp["dims"], sp["ranks"], sp["alpha"], seed=sp["seed"],
                                        storage=np.float32, keep_parts=False)
        insts.append(inst)
        Xs.append(torch.from_numpy(inst.X).to("cuda:0"))
        ranks.append(sp["ranks"])
        I.append(synth.sample_sizes(sp["dims"], sp["ranks"], 3.0)[0])
        seeds.append(sp["seed"])
    streams = [torch.cuda.Stream() for _ in range(2)]
    hs = [rt.create(0, stream=st, dtype=tdt) for st in streams]
    infos, Ls = rt.solve_batch(hs, Xs, ranks, I, tol=0.0, max_iter=K, seeds=seeds,
                               with_L=True, L_dtype=torch.float64, check=False)
    torch.cuda.synchronize()
    for j, inst in enumerate(insts):
        res = oracle_rtcur(inst.X, ranks[j], I[j], None, None, 0.7, 0.0, K, seeds[j], "F")
        print(f"[batch oracle] {specs[j]['dims']} r={ranks[j]} I={I[j]} "
              f"err gpu {infos[j].err:.6e} oracle {res.err:.6e}", flush=True)
        assert infos[j].iters == K and infos[j].eig_unconverged == 0
        etol = 1e-9 if dtype == "f64" else 2e-3
        assert abs(infos[j].err - res.err) <= etol * res.err
        ltol = 1e-10 if dtype == "f64" else 1e-4
        assert rel(Ls[j].cpu().numpy(), res.reconstruct()) <= ltol
    for h in hs:
        rt.destroy(h)
