"""GPU parity: the HIP library through its C ABI against the FP64 oracle on
the same seeded inputs.  Bars: indices bit-exact; zeta history exact; e^(k)
to 1e-9 relative; support exact and L (sampled blocks and full grid) to
1e-10 in FP64; support >= 99.99 % and L to 1e-4 in FP32."""
import os

import numpy as np
import pytest

import synth
from oracle import OracleError
from oracle import outliers as oracle_outliers
from oracle import rtcur as oracle_rtcur

from _parity import compare, rel, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    import paper_2108_10448_amd as rt
    assert os.path.exists(rt.LIB_PATH), "librtcur.so is not built"
    assert torch.cuda.is_available(), "no HIP device"
    rt.lib()


@pytest.fixture(scope="module")
def cube100():
    inst = synth.config_instance("cube100_r3")
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    return inst, I


@pytest.mark.parametrize("K", [1, 2, 5])
def test_fixed_iterations_fp64_cube100(cube100, K):
    inst, I = cube100
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, K, 0, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=0.0, max_iter=K, check=False)
    assert info.iters == K
    compare(res, h, info, label=f"cube100 F K={K}")


@pytest.mark.parametrize("variant", ["F", "R"])
def test_to_tolerance_fp64_cube100(cube100, variant):
    inst, I = cube100
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, variant)
    h, info, _ = run_gpu(inst.X, inst.ranks, I, variant=variant)
    assert info.iters == res.iters and info.converged
    compare(res, h, info, label=f"cube100 {variant} tol")


def test_fp32_compute_cube100(cube100):
    inst, I = cube100
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    h, info, _ = run_gpu(inst.X.astype(np.float32), inst.ranks, I, dtype=torch.float32)
    assert abs(info.iters - res.iters) <= 1 and info.converged
    res2 = oracle_rtcur(inst.X.astype(np.float32), inst.ranks, I, None, None, 0.7, 0.0,
                        info.iters, 0, "F")
    compare(res2, h, info, fp64=False, label="cube100 F fp32")


def test_fiber_sampling_fp64():
    inst = synth.tucker_plus_sparse((60, 50, 40), (3, 2, 3), alpha=0.15, seed=3)
    I, J = synth.sample_sizes(inst.dims, inst.ranks, 3.0, fiber=True)
    res = oracle_rtcur(inst.X, inst.ranks, I, J, None, 0.7, 0.0, 6, 9, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, I, J, tol=0.0, max_iter=6, seed=9, check=False)
    compare(res, h, info, label="fiber 60x50x40")


def test_four_modes_ragged_fp64():
    inst = synth.tucker_plus_sparse((23, 19, 3, 17), (3, 2, 2, 2), alpha=0.1, seed=5)
    I = (9, 8, 3, 7)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 8, 2, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=0.0, max_iter=8, seed=2, check=False)
    compare(res, h, info, label="4-mode ragged")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_four_modes_wide_ranks(dtype):
    # the video-shaped rank pattern (10, 10, 3, 5): ranks above 8 in a 4-mode
    # tensor, the colour-like mode fully sampled (s = d = r = 3)
    inst = synth.tucker_plus_sparse((40, 44, 3, 30), (10, 10, 3, 5), alpha=0.1, seed=12)
    I = (30, 32, 3, 16)
    X = inst.X if dtype == "f64" else inst.X.astype(np.float32)
    res = oracle_rtcur(X, inst.ranks, I, None, None, 0.7, 0.0, 10, 4, "F")
    h, info, _ = run_gpu(X, inst.ranks, I, tol=0.0, max_iter=10, seed=4, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    compare(res, h, info, fp64=dtype == "f64", label=f"4-mode r=(10,10,3,5) {dtype}")


@pytest.fixture(scope="module")
def video_small():
    # the video recipe (nonnegative Tucker background, moving rectangles) at a
    # quarter of the frame size and half the frames; upsilon = 2 sample sizes
    inst = synth.video_like((120, 160, 3, 200), side=(10, 30), storage=np.float32)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 2.0)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 5, 0, "F")
    return inst, I, res


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_video_shaped(video_small, dtype):
    # the samples' spectra have sigma_{r+1} / sigma_r up to 0.98 here, which
    # takes the eigensolver's guarded (Rayleigh-Ritz) iteration
    inst, I, res = video_small
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=0.0, max_iter=5, seed=0, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    print(f"[video] eig steps {info.eig_steps} unconverged {info.eig_unconverged}", flush=True)
    assert info.eig_unconverged == 0
    compare(res, h, info, fp64=dtype == "f64", label=f"video 120x160x3x200 {dtype}")


def test_solve_batch_uneven_instances():
    # six instances of uneven shapes and ranks over three handles on their
    # own streams: each equals the oracle and, bit for bit, a single solve
    import paper_2108_10448_amd as rt
    specs = synth.batch_specs(count=6, dmin=24, dmax=60, rmin=2, rmax=5, seed=7)
    insts = [synth.tucker_plus_sparse(**sp) for sp in specs]
    Xs = [torch.from_numpy(i.X).to("cuda:0") for i in insts]
    ranks = [i.ranks for i in insts]
    I = [synth.sample_sizes(i.dims, i.ranks, 3.0)[0] for i in insts]
    seeds = [sp["seed"] + 100 for sp in specs]
    streams = [torch.cuda.Stream() for _ in range(3)]
    hs = [rt.create(0, stream=st) for st in streams]
    infos, Ls = rt.solve_batch(hs, Xs, ranks, I, tol=0.0, max_iter=6, seeds=seeds,
                               with_L=True, check=False)
    torch.cuda.synchronize()
    for j, inst in enumerate(insts):
        print(f"[batch] {inst.dims} r={inst.ranks} status {infos[j].status} "
              f"iters {infos[j].iters} err {infos[j].err:.6e}", flush=True)
        assert infos[j].status == rt.NOT_CONVERGED and infos[j].iters == 6
        res = oracle_rtcur(inst.X, inst.ranks, I[j], None, None, 0.7, 0.0, 6, seeds[j], "F")
        assert abs(infos[j].err - res.err) <= 1e-9 * res.err
        assert rel(Ls[j].cpu().numpy(), res.reconstruct()) <= 1e-10
        h1 = rt.create(0)
        rt.solve(h1, Xs[j], ranks[j], I[j], tol=0.0, max_iter=6, seed=seeds[j], check=False)
        L1 = rt.reconstruct(h1)
        torch.cuda.synchronize()
        assert torch.equal(L1, Ls[j])
        rt.destroy(h1)
    # the work queue: every instance solved once, each handle's solves
    # numbered 0, 1, ..; each handle keeps the state of the last instance it
    # solved
    for t in range(len(hs)):
        mine = sorted((infos[j].batch_seq, j) for j in range(len(Xs))
                      if infos[j].batch_slot == t)
        assert [q for q, _ in mine] == list(range(len(mine)))
        if mine:
            Lt = rt.reconstruct(hs[t])
            torch.cuda.synchronize()
            assert torch.equal(Lt, Ls[mine[-1][1]])
    assert all(0 <= infos[j].batch_slot < len(hs) for j in range(len(Xs)))
    assert all(infos[j].solve_ms > 0 for j in range(len(Xs)))
    for h in hs:
        rt.destroy(h)


@pytest.fixture(scope="module")
def video_full():
    # the video-shaped workload at its full size (240 x 320 x 3 x 400, float32
    # storage, upsilon = 2), the oracle run for three iterations
    inst = synth.video_like()
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 2.0)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 3, 0, "F")
    return inst, I, res


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_video_full_size(video_full, dtype):
    inst, I, res = video_full
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=0.0, max_iter=3, seed=0, check=False,
                         dtype=torch.float64 if dtype == "f64" else torch.float32)
    assert info.eig_unconverged == 0
    compare(res, h, info, fp64=dtype == "f64", label=f"video 240x320x3x400 {dtype}")


def test_batch_recipe_instances():
    # the first six instances of the 64-tensor batch recipe (shapes up to
    # 256^3, ranks 2..8): solved together over three handles, each equals
    # its single solve bit for bit and converges
    import paper_2108_10448_amd as rt
    specs = synth.batch_specs()[:6]
    Xs, ranks, I, seeds = [], [], [], []
    for sp in specs:
        inst = synth.tucker_plus_sparse(sp["dims"], sp["ranks"], sp["alpha"], seed=sp["seed"],
                                        storage=np.float32, keep_parts=False)
        Xs.append(torch.from_numpy(inst.X).to("cuda:0"))
        ranks.append(sp["ranks"])
        I.append(synth.sample_sizes(sp["dims"], sp["ranks"], 3.0)[0])
        seeds.append(sp["seed"])
    streams = [torch.cuda.Stream() for _ in range(3)]
    hs = [rt.create(0, stream=st, dtype=torch.float32) for st in streams]
    infos, Ls = rt.solve_batch(hs, Xs, ranks, I, seeds=seeds, with_L=True, check=False)
    torch.cuda.synchronize()
    for j in range(len(Xs)):
        print(f"[batch] {specs[j]['dims']} r={specs[j]['ranks']} iters {infos[j].iters} "
              f"err {infos[j].err:.3e}", flush=True)
        assert infos[j].status == rt.OK and infos[j].converged
        h1 = rt.create(0, dtype=torch.float32)
        info1 = rt.solve(h1, Xs[j], ranks[j], I[j], seed=seeds[j], check=False)
        L1 = rt.reconstruct(h1)
        torch.cuda.synchronize()
        assert info1.iters == infos[j].iters and info1.err == infos[j].err
        assert torch.equal(L1, Ls[j])
        rt.destroy(h1)
    for h in hs:
        rt.destroy(h)


def test_two_modes_fp64():
    inst = synth.tucker_plus_sparse((300, 257), (4, 4), alpha=0.1, seed=8)
    I = (40, 37)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-8, 60, 4, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=1e-8, max_iter=60, seed=4, check=False)
    assert info.iters == res.iters
    compare(res, h, info, label="2-mode")


@pytest.mark.parametrize("dims,ranks,I", [
    # ranks 9..16 take the 16-column path; the small samples keep the Gram
    # in LDS, the larger ones in global memory
    ((80, 70, 60), (10, 12, 9), (40, 44, 36)),
    ((200, 190, 180), (11, 16, 13), (150, 140, 130)),
    # the largest sample the library takes, |I_i| = 256, with a ragged third mode
    ((300, 260, 40), (4, 4, 3), (256, 256, 40)),
])
def test_wide_ranks_and_max_sample(dims, ranks, I):
    inst = synth.tucker_plus_sparse(dims, ranks, alpha=0.2, seed=11)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, 4, 3, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, I, tol=0.0, max_iter=4, seed=3, check=False)
    compare(res, h, info, label=f"{dims} r={ranks} I={I}")


def test_shape_limits_rejected():
    import paper_2108_10448_amd as rt
    h = rt.create(0)
    X = torch.zeros((40, 300, 30), dtype=torch.float64, device="cuda:0")
    for ranks, I in [((17, 2, 2), (20, 20, 20)),      # r_i <= 16
                     ((2, 2, 2), (20, 257, 20)),      # |I_i| <= 256
                     ((5, 2, 2), (4, 20, 20))]:       # r_i <= |I_i|
        with pytest.raises(rt.RTCURError) as e:
            rt.solve(h, X, ranks, I)
        assert e.value.status == rt.E_INVAL
    X4 = torch.zeros((12, 12, 12, 12), dtype=torch.float64, device="cuda:0")
    with pytest.raises(rt.RTCURError) as e:
        rt.solve(h, X4, (9, 9, 9, 9), (10, 10, 10, 10))    # prod r_i = 6561 > 4096
    assert e.value.status == rt.E_INVAL
    # four modes: core slice r_3 |I_1| |I_2| = 4 * 30 * 30 > 2048 (with three
    # modes r_2 |I_1| <= 16 * 256 always fits)
    X4 = torch.zeros((12, 30, 30, 12), dtype=torch.float64, device="cuda:0")
    with pytest.raises(rt.RTCURError) as e:
        rt.solve(h, X4, (2, 2, 2, 4), (10, 30, 30, 10))
    assert e.value.status == rt.E_INVAL
    # the handle still solves a valid problem afterwards
    inst = synth.tucker_plus_sparse((16, 16, 16), (2, 2, 2), alpha=0.1, seed=2)
    info = rt.solve(h, torch.from_numpy(inst.X).cuda(), (2, 2, 2), (8, 8, 8), check=False)
    assert info.status in (rt.OK, rt.NOT_CONVERGED)
    rt.destroy(h)


def test_full_sampling_and_given_zeta0():
    inst = synth.tucker_plus_sparse((20, 18, 16), (2, 2, 2), alpha=0.1, seed=6)
    res = oracle_rtcur(inst.X, inst.ranks, inst.dims, None, 3.0, 0.8, 0.0, 7, 1, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, inst.dims, zeta0=3.0, gamma=0.8, tol=0.0,
                         max_iter=7, seed=1, check=False)
    assert info.zeta0 == 3.0
    compare(res, h, info, label="full sampling")


def test_not_converged_status():
    import paper_2108_10448_amd as rt
    inst = synth.tucker_plus_sparse((30, 30, 30), (2, 2, 2), alpha=0.5, seed=1)
    res = oracle_rtcur(inst.X, inst.ranks, (15, 15, 15), None, None, 0.7, 1e-12, 4, 0, "F")
    h, info, _ = run_gpu(inst.X, inst.ranks, (15, 15, 15), tol=1e-12, max_iter=4, check=False)
    assert info.status == rt.NOT_CONVERGED and info.iters == 4
    compare(res, h, info, label="not converged")


def test_zero_tensor_and_tol_one():
    import paper_2108_10448_amd as rt
    X = np.zeros((12, 10, 8))
    h, info, _ = run_gpu(X, (1, 1, 1), (4, 4, 4), check=False)
    assert info.status == rt.OK and info.iters == 0
    L = rt.reconstruct(h).cpu().numpy()
    assert not np.any(L)
    inst = synth.tucker_plus_sparse((12, 10, 8), (2, 2, 2), alpha=0.1, seed=1)
    h, info, _ = run_gpu(inst.X, inst.ranks, (6, 6, 6), tol=1.0, check=False)
    assert info.status == rt.OK and info.iters == 0


def test_rank_deficient_and_nonfinite():
    import paper_2108_10448_amd as rt
    inst = synth.tucker_plus_sparse((16, 16, 16), (1, 1, 1), alpha=0.0, seed=1)
    with pytest.raises(OracleError):
        oracle_rtcur(inst.X, (2, 2, 2), (8, 8, 8), None, None, 0.7, 1e-5, 5, 0, "F")
    h, info, _ = run_gpu(inst.X, (2, 2, 2), (8, 8, 8), max_iter=5, check=False)
    assert info.status == rt.E_RANK
    X = np.ones((8, 8, 8))
    X[1, 2, 3] = np.nan
    h, info, _ = run_gpu(X, (1, 1, 1), (8, 8, 8), check=False)
    assert info.status == rt.E_NONFINITE
    # the handle stays usable after an error
    inst = synth.tucker_plus_sparse((16, 16, 16), (2, 2, 2), alpha=0.1, seed=2)
    info = rt.solve(h, torch.from_numpy(inst.X).cuda(), (2, 2, 2), (8, 8, 8), check=False)
    assert info.status in (rt.OK, rt.NOT_CONVERGED)


def test_bitwise_deterministic(cube100):
    import paper_2108_10448_amd as rt
    inst, I = cube100
    h1, i1, _ = run_gpu(inst.X, inst.ranks, I)
    h2, i2, _ = run_gpu(inst.X, inst.ranks, I)
    assert i1.iters == i2.iters
    assert np.array_equal(rt.get_history(h1)[0], rt.get_history(h2)[0])
    for b in range(4):
        assert np.array_equal(rt.get_block(h1, b, rt.BLOCK_C), rt.get_block(h2, b, rt.BLOCK_C))


@pytest.fixture(scope="module")
def cube300():
    inst = synth.config_instance("cube300_r5")
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    return inst, I


@pytest.mark.parametrize("variant", ["F", "R"])
def test_cube300_fp64_compute(cube300, variant):
    # headline workload: 300^3 float32 storage, rank 5, alpha 0.3, FP64 compute
    inst, I = cube300
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, variant)
    h, info, _ = run_gpu(inst.X, inst.ranks, I, variant=variant)
    assert info.iters == res.iters and info.converged
    compare(res, h, info, label=f"cube300 {variant} fp64")


def test_cube300_fp32_compute(cube300):
    inst, I = cube300
    h, info, _ = run_gpu(inst.X, inst.ranks, I, dtype=torch.float32)
    assert info.converged
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, "F")
    assert abs(info.iters - oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5,
                                         100, 0, "F").iters) <= 1
    out = compare(res, h, info, fp64=False, label="cube300 F fp32")
    L = torch.empty(inst.dims, dtype=torch.float32, device="cuda:0")
    import paper_2108_10448_amd as rt
    rt.reconstruct(h, out=L)
    assert rel(L.cpu().numpy().astype(np.float64), res.reconstruct()) < 1e-4


@pytest.mark.parametrize("workload", ["cube100", "cube300"])
def test_bf16_blocks_with_fp32_refinement(cube100, cube300, workload):
    # bfloat16 blocks until e^(k) <= 1e-2, then the FP32 refinement sweep:
    # the returned iterate meets the reduced-precision bar against the FP64
    # oracle run for the same number of iterations
    import paper_2108_10448_amd as rt
    inst, I = cube100 if workload == "cube100" else cube300
    h, info, _ = run_gpu(inst.X, inst.ranks, I, dtype=torch.bfloat16)
    e, _ = rt.get_history(h)
    print(f"[bf16] {workload} iters {info.iters} e {[f'{x:.3e}' for x in e]}", flush=True)
    assert info.converged and info.eig_unconverged == 0
    ref = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    assert abs(info.iters - ref.iters) <= 1
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, "F")
    # e^(k) of the bfloat16 iterations carries the blocks' rounding (2^-9
    # relative per stored entry) in its numerator: bounded by 2 * 2^-9
    compare(res, h, info, fp64=False, label=f"{workload} bf16", eabs=2 * 2.0 ** -9)
    L = rt.reconstruct(h)
    assert L.dtype == torch.float32
    assert rel(L.cpu().numpy().astype(np.float64), res.reconstruct()) < 1e-4


def _outlier_compare(S_g, L_g, S_o, L_o, exact, tol, label):
    sg, so = S_g != 0, S_o != 0
    agree = float(np.mean(sg == so))
    if exact:
        assert np.array_equal(sg, so), f"{label}: support differs at {np.sum(sg != so)} entries"
    else:
        assert agree >= 0.9999, f"{label}: support agreement {agree}"
    both = sg & so
    eS = rel(S_g[both], S_o[both])
    eL = rel(L_g, L_o)
    print(f"[parity] outliers {label}: support agree {agree:.6f}, S {eS:.2e}, L {eL:.2e}")
    assert eS <= tol and eL <= tol


def test_outliers_fp64_cube100(cube100):
    import paper_2108_10448_amd as rt
    inst, I = cube100
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 1e-5, 100, 0, "F")
    h, info, X = run_gpu(inst.X, inst.ranks, I)
    assert info.iters == res.iters
    S_g, L_g = rt.outliers(h, X, with_L=True)
    S_o, L_o = oracle_outliers(res, inst.X)
    _outlier_compare(S_g.cpu().numpy(), L_g.cpu().numpy(), S_o, L_o, True, 1e-10, "cube100")
    # an explicit threshold, S only
    z = 10 * res.zeta_hist[-1]
    S_g = rt.outliers(h, X, z).cpu().numpy()
    S_o, _ = oracle_outliers(res, inst.X, z)
    _outlier_compare(S_g, L_g.cpu().numpy(), S_o, L_o, True, 1e-10, "cube100 zeta")


def test_outliers_fp32_cube300(cube300):
    import paper_2108_10448_amd as rt
    inst, I = cube300
    h, info, X = run_gpu(inst.X, inst.ranks, I, dtype=torch.float32)
    res = oracle_rtcur(inst.X, inst.ranks, I, None, None, 0.7, 0.0, info.iters, 0, "F")
    S_g, L_g = rt.outliers(h, X, with_L=True)
    S_o, L_o = oracle_outliers(res, inst.X)
    _outlier_compare(S_g.double().cpu().numpy(), L_g.double().cpu().numpy(), S_o, L_o, False,
                     1e-4, "cube300 fp32")


def test_outliers_without_iterations():
    import paper_2108_10448_amd as rt
    inst = synth.tucker_plus_sparse((12, 10, 8), (2, 2, 2), alpha=0.1, seed=1)
    res = oracle_rtcur(inst.X, inst.ranks, (6, 6, 6), None, None, 0.7, 1.0, 100, 0, "F")
    h, info, X = run_gpu(inst.X, inst.ranks, (6, 6, 6), tol=1.0, check=False)
    assert info.iters == 0 == res.iters
    S_g, L_g = rt.outliers(h, X, with_L=True)
    S_o, L_o = oracle_outliers(res, inst.X)
    assert not np.any(L_g.cpu().numpy())
    assert np.array_equal(S_g.cpu().numpy(), S_o)


def test_handle_reuse_across_sizes_and_samplings():
    # one handle solves, in turn: A, B (same sizes as A, other data and seed:
    # the layout and work lists of A are reused), C (other sizes and fibre
    # sampling), then A again; each equals the oracle (FP64 bar)
    import paper_2108_10448_amd as rt
    h = rt.create(0)
    a = synth.tucker_plus_sparse((40, 36, 30), (3, 2, 3), alpha=0.2, seed=21)
    b = synth.tucker_plus_sparse((40, 36, 30), (3, 2, 3), alpha=0.3, seed=22)
    c = synth.tucker_plus_sparse((28, 33, 25), (2, 3, 2), alpha=0.2, seed=23)
    Ia = synth.sample_sizes(a.dims, a.ranks, 3.0)[0]
    Ic, Jc = synth.sample_sizes(c.dims, c.ranks, 3.0, fiber=True)
    cases = [(a, Ia, None, 5), (b, Ia, None, 6), (c, Ic, Jc, 7), (a, Ia, None, 8)]
    for inst, I, J, seed in cases:
        X = torch.from_numpy(inst.X).to("cuda:0")
        info = rt.solve(h, X, inst.ranks, I, J, tol=0.0, max_iter=5, seed=seed, check=False)
        torch.cuda.synchronize()
        res = oracle_rtcur(inst.X, inst.ranks, I, J, None, 0.7, 0.0, 5, seed, "F")
        assert info.iters == res.iters == 5
        compare(res, h, info, label=f"reuse {inst.dims} seed {seed}")
    rt.destroy(h)
